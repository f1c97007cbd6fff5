"""Mie-series pins and the frequency-domain MoM against Mie."""
import math

import numpy as np
import pytest

from oracle import excitation, mie, physics as ph
from oracle_cases import dense_z, l2_band_params, sphere


def test_rayleigh_limit():
    a = 0.5
    for ka in (0.02, 0.05):
        assert mie.backscatter(ka, a) / (math.pi * a * a) == pytest.approx(9 * ka ** 4, rel=2e-3)


def test_optical_limit_and_theorem():
    a = 1.0
    assert mie.backscatter(80.0, a) / (math.pi * a * a) == pytest.approx(1.0, abs=0.01)
    for ka in (0.3, 3.0, 12.0):
        ext, sca = mie.cross_sections(ka, a)
        assert ext == pytest.approx(sca, rel=1e-10)


def test_bistatic_backscatter_consistent():
    TH, PH, d, th = mie.sphere_grid(19, 8)
    ka = math.pi
    sig = mie.rcs_theta_mie(ka, 0.5, [0, 0, -1.0], [1.0, 0, 0], d, th)
    assert sig[0, 0] == pytest.approx(mie.backscatter(ka, 0.5), rel=1e-10)


@pytest.mark.parametrize("f", [200e6, 300e6])
def test_fd_mom_against_mie(f):
    s = sphere()
    dt, ng = l2_band_params()
    Z = dense_z(dt, 300e6, ng, (f,))[-1]
    w = 2 * math.pi * f
    V = excitation.excitation(s, 1, 1.0, [[0, 0, -1.0]], [[1.0, 0, 0]], 1e30, 0.0, f)[0, 0] / (1j * w)
    I = np.linalg.solve(Z, V)
    TH, PH, d, th = mie.sphere_grid(91, 180)
    sm = mie.rcs_theta_mie(2 * math.pi * f / ph.C0 * 0.5, 0.5, [0, 0, -1.0], [1.0, 0, 0], d, th)
    sc = mie.rcs_theta_current(s, I, f, d, th)
    # eq. (2) dB-error (no square root) on the coarse 480-unknown sphere
    assert mie.db_error(sc, sm, TH) < 1e-4
    assert sc[0, 0] == pytest.approx(sm[0, 0], rel=0.2)
