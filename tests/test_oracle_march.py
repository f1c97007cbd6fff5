"""Pins of the oracle's iterative pieces: GMRES against a direct solve, and
the FFT march of eq. (5) (k-space history sum, GMRES per step) against the
march with the assembled AIM matrices and one LU factorisation."""
import numpy as np
import pytest

import workloads as W
from oracle import aim, excitation, geometry, kernels, march, physics as ph, zfill


def test_gmres_solves_a_dense_system():
    rng = np.random.default_rng(5)
    n = 60
    A = np.eye(n) * 4 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    d = 1.0 / np.diag(A)
    for restart in (5, 60):               # restarted and full
        x, its = march.gmres(lambda v: A @ v, b, d, np.zeros(n, complex), 1e-12, restart=restart)
        assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)
        assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-10 * np.linalg.norm(x)
        assert 1 <= its <= 200


def test_fft_march_equals_dense_lu_march():
    """Level-2 sphere, +-20 %, 14 steps (N_g = 4, so most steps carry the
    full history): the FFT march at GMRES tolerance 1e-13 against the LU
    march of the assembled Z^near_m + Z^FFT_m."""
    wl = W.SPHERE_L2
    xyz, tri, rwg = wl.mesh()
    s = geometry.Surface(xyz, tri, rwg)
    dt = ph.dt_from_beta(wl.beta, wl.f_bw)
    ng = ph.ng_from(ph.rmax_of(xyz), dt)
    A = aim.AIM(s, wl.grid, wl.near_lambda * ph.C0 / wl.f0, dt, wl.f0, ng)
    vals = A.near_values(lambda r, c, ms: zfill.assemble_pairs(
        s, r, c, [kernels.EnvelopeKernel(m, dt, wl.f0) for m in ms]))
    Z = np.stack([A.far_dense(m) for m in range(ng + 1)])
    for m in range(A.mn + 1):
        np.add.at(Z[m], (A.rows, A.cols), vals[m])
    kh, pp = wl.incidence()
    nt = 14
    V = excitation.excitation(s, nt, dt, kh, pp, wl.sigma, 4 * dt, wl.f0)[:, 0]
    ref = march.march_dense(Z, V[:, None, :])[:, 0]
    its = []
    I = march.march_fft(A, vals, V, 1e-13, restart=60, on_step=lambda l, k: its.append(k))
    assert len(its) == nt and min(its) >= 1
    assert np.linalg.norm(I - ref) <= 1e-10 * np.linalg.norm(ref)
