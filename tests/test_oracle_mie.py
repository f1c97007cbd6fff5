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


def test_envelope_rcs_matches_fd_rcs_in_band():
    """The RCS post-processed from the time-domain far-field envelopes of an
    ET march (Sec. 2.4) equals the frequency-domain MoM RCS at each frequency
    of a narrow band: at f_c (the CPPIF partition of unity makes the discrete
    march's DC response the FD solution), and off-centre to the march's
    second-order time discretisation.  A dropped dt, a wrong pulse-spectrum
    width or a wrong polarisation projection fails it."""
    from oracle import farfield, march
    fc = 300e6
    s = sphere()
    dt, ng = l2_band_params(frac=0.01)
    fbw = 0.01 * fc
    sigma = 3.0 / (2 * math.pi * fbw)
    td = 8 * sigma
    nt = int(math.ceil((td + 8 * sigma) / dt))
    dfs = (0.0, fbw / 4, -fbw / 2)
    Z = dense_z(dt, fc, ng, tuple(fc + d for d in dfs))
    V = excitation.excitation(s, nt, dt, [[0, 0, -1.0]], [[1.0, 0, 0]], sigma, td, fc)
    I = march.march_dense(Z[:ng + 1], V)
    TH, PH, d, th = mie.sphere_grid(13, 24)
    U = farfield.FarField(s, d.reshape(-1, 3), dt, fc).apply(I)
    for i, (df, tol) in enumerate(zip(dfs, (2e-4, 2e-4, 5e-3))):
        f = fc + df
        se = mie.rcs_envelope(U[:, 0], dt, df, sigma, th.reshape(-1, 3)).reshape(TH.shape)
        Vf = excitation.excitation(s, 1, 1.0, [[0, 0, -1.0]], [[1.0, 0, 0]], 1e30, 0.0, f)[0, 0] / (1j * 2 * math.pi * f)
        sf = mie.rcs_theta_current(s, np.linalg.solve(Z[ng + 1 + i], Vf), f, d, th)
        assert np.abs(se - sf).max() / sf.max() < tol, df
        assert mie.db_error(se, sf, TH) < 1e-5


def test_db_error_hand_computed():
    """Eq. (2) on four directions whose RCS values are whole decibels, worked
    by hand: the reference peaks at 20 dB, so TH = 20 - 80 = -60 dB; both
    patterns are clipped at TH and shifted by -TH (reference 80, 70, 0, 30;
    test 77, 70, 20, 0), and the (theta, phi) quadrature weight is sin(theta)."""
    theta = np.array([math.pi / 6, math.pi / 2, math.pi / 3, math.pi / 4])
    ref_db = np.array([20.0, 10.0, -70.0, -30.0])
    sig_db = np.array([17.0, 10.0, -40.0, -65.0])
    w = [0.5, 1.0, math.sqrt(3) / 2, math.sqrt(2) / 2]
    num = w[0] * 3 ** 2 + w[1] * 0 + w[2] * 20 ** 2 + w[3] * 30 ** 2
    den = w[0] * 80 ** 2 + w[1] * 70 ** 2 + w[2] * 0 ** 2 + w[3] * 30 ** 2
    e = mie.db_error(10.0 ** (sig_db / 10), 10.0 ** (ref_db / 10), theta)
    assert e == pytest.approx(num / den, rel=1e-12)
    # the floor is relative to the reference's peak, not to 0 dB: with a
    # 50 dB floor TH = -30 dB, so the last two directions of both patterns
    # clip to 0 (reference 50, 40, 0, 0; test 47, 40, 0, 0)
    e50 = mie.db_error(10.0 ** (sig_db / 10), 10.0 ** (ref_db / 10), theta, floor_db=50.0)
    assert e50 == pytest.approx(w[0] * 3 ** 2 / (w[0] * 50 ** 2 + w[1] * 40 ** 2), rel=1e-12)
