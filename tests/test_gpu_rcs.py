"""Radar cross section from the GPU march (Sec. 2.4), through the C ABI:
etaim_rcs against the oracle's envelope RCS on the same far-field envelopes
(parity), and the whole path (march, far field, RCS) against the exact
frequency-domain MoM RCS of the sphere in a narrow band, with the eq. (2)
dB error computed by the library and by the oracle."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from gpu_cases import gpu_problem, oracle_aim, rel
from oracle import excitation, mie
from oracle_cases import dense_z

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def test_rcs_from_the_march(torch):
    from paper_1408_7060_amd import db_error
    name = W.SPHERE_L2_NARROW.name
    wl = W.WORKLOADS[name]
    s, A, vals, p = oracle_aim(name)
    nt = 60
    kh, pp = wl.incidence()
    V = excitation.excitation(s, nt, p["dt"], kh, pp, wl.sigma, wl.td, wl.f0)
    P = gpu_problem(name, tol=1e-13, nt=nt)
    I, _ = P.march(torch.from_numpy(np.ascontiguousarray(V)).cuda())
    TH, PH, d, th = mie.sphere_grid(13, 24)
    pol = th.reshape(-1, 3)
    U = P.farfield(d.reshape(-1, 3), I)
    fbw = wl.frac_bw * wl.f0
    dfs = (0.0, fbw / 4)
    sg = P.rcs(U, pol, dfs, wl.sigma).cpu().numpy()
    assert sg.shape == (len(dfs), 1, pol.shape[0])
    Uc = U.cpu().numpy()
    Z = dense_z(p["dt"], wl.f0, p["ng"], tuple(wl.f0 + x for x in dfs))
    for i, df in enumerate(dfs):
        ref = mie.rcs_envelope(Uc[:, 0], p["dt"], df, wl.sigma, pol)
        e = rel(sg[i, 0], ref)
        _say("rcs df", df, "parity rel", e)
        assert e <= 1e-12
        f = wl.f0 + df
        Vf = excitation.excitation(s, 1, 1.0, kh, pp, 1e30, 0.0, f)[0, 0] / (1j * 2 * math.pi * f)
        sf = mie.rcs_theta_current(s, np.linalg.solve(Z[p["ng"] + 1 + i], Vf), f, d, th).ravel()
        dbe = db_error(sg[i, 0], sf, np.sin(TH).ravel())
        _say("  vs exact FD MoM: max rel", np.abs(sg[i, 0] - sf).max() / sf.max(), "dB error", dbe)
        assert dbe == pytest.approx(mie.db_error(sg[i, 0].reshape(TH.shape), sf.reshape(TH.shape), TH), rel=1e-10)
        assert dbe < 1e-5
        assert np.abs(sg[i, 0] - sf).max() / sf.max() < 1e-2
    with pytest.raises(Exception) as ei:
        P.rcs(U, pol, dfs, 0.0)
    assert ei.value.code == -1
    P.close()
