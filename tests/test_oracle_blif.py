"""Pins of the band-limited interpolatory basis and its causal
extrapolation (Sec. 3, Sec. 3.1.2; M = 3, N_samp = 3, N_omega = 6 for the
paper's ET runs):

* T(n) = delta_n0 (interpolatory) and T's derivatives against central
  differences;
* the window's power series equals Knab's sinh formula;
* shifted BLIFs reproduce exp(j Omega tau) for |Omega| <= 2 pi beta to the
  window's accuracy (about 1e-3 at M = 3, beta = 1/5), while the CPPIF of
  the same support does not at the band edge;
* with N_omega = N_samp the extrapolation is exact at its fit frequencies;
* folding the non-causal matrices reproduces the full sum over
  m = -(M-1)..N_g exactly for a current at a fit frequency (a wrong index
  or sign in the fold breaks it);
* the BLIF envelope kernels obey the approximate sum rule
  sum_m Z_m ~ j w_c Z_FD(f_c) (the BLIF's partition of unity holds to the
  window's accuracy);
* the AIM with a BLIF: its far-part paths agree and the pre-correction
  restores the folded exact entries.
"""
import math

import numpy as np
import pytest

from oracle import aim, blif, cppif, kernels, physics as ph, zfill
from oracle_cases import dense_z, sphere

FC = 300e6


def test_interpolatory_and_window_series():
    b = blif.Blif(3, 0.2)
    n = np.arange(-4, 5).astype(float)
    assert np.abs(b.T(n) - (n == 0)).max() <= 1e-15
    t = np.linspace(-2.9, 2.9, 23)
    w_ser = b._w(1.0 - t * t / 9.0, 0)
    assert np.abs(w_ser - b.window_closed_form(t)).max() <= 1e-14 * np.abs(w_ser).max()
    # support (-M, M]
    assert b.T(np.array([-3.0, -3.5, 3.2])).max() == 0.0


def test_derivatives_match_central_differences():
    b = blif.Blif(3, 0.2)
    t = np.array([0.37, -1.41, 2.3, 0.1, -0.05, 1.0])
    h = 1e-4
    for d in (1, 2, 3):
        fd = (b.T(t + h, d - 1) - b.T(t - h, d - 1)) / (2 * h)
        assert np.abs(fd - b.T(t, d)).max() <= 5e-7 * max(1.0, np.abs(b.T(t, d)).max()), d


def test_band_limited_reproduction():
    beta = 0.2
    b = blif.Blif(3, beta)
    tau = np.linspace(0.0, 1.0, 21)
    errs = []
    for x in (0.0, 0.5, 1.0):
        om = 2 * math.pi * beta * x
        s = sum(b.T(tau - n) * np.exp(1j * om * n) for n in range(-6, 7))
        errs.append(np.abs(s - np.exp(1j * om * tau)).max())
    assert max(errs) < 3e-3
    # the CPPIF (a causal cubic interpolant) is worse at the band edge
    om = 2 * math.pi * beta
    c = sum(cppif.T(tau - n) * np.exp(1j * om * n) for n in range(-6, 7))
    assert np.abs(c - np.exp(1j * om * tau)).max() > 3 * errs[-1]


def test_extrapolation_exact_at_its_fit_frequencies():
    beta = 0.2
    a = blif.extrapolation(beta, 3, 3, 3)
    wdt = 2 * math.pi * beta * np.linspace(-1, 1, 3)
    past = np.exp(-1j * np.outer(wdt, np.arange(3)))
    for k in (1, 2):
        assert np.abs(past @ a[k - 1] - np.exp(1j * wdt * k)).max() <= 1e-13
    # the paper's setting (N_omega = 2 N_samp) is a least-squares fit with real coefficients
    a6 = blif.extrapolation(beta, 3, 3, 6)
    assert a6.shape == (2, 3) and np.isrealobj(a6)


def test_fold_reproduces_the_full_sum_at_a_fit_frequency():
    rng = np.random.default_rng(7)
    M, ng, n = 3, 5, 6
    Z = {m: rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for m in range(-(M - 1), ng + 1)}
    beta = 0.2
    a = blif.extrapolation(beta, M, 3, 3)
    Zt = blif.fold(Z, a, ng)
    om = 2 * math.pi * beta           # a fit frequency: the extrapolation is exact there
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    l = 10
    I = {q: x * np.exp(1j * om * q) for q in range(l - ng - 2, l + M)}
    full = sum(Z[m] @ I[l - m] for m in range(-(M - 1), ng + 1))
    folded = sum(Zt[m] @ I[l - m] for m in range(ng + 1))
    assert np.abs(full - folded).max() <= 1e-12 * np.abs(full).max()


def _blif_problem(frac=0.2, beta=0.2):
    s = sphere()
    dt = beta / (frac * FC)
    b = blif.Blif(3, beta)
    ng = int(math.floor(ph.rmax_of(s.xyz) / (ph.C0 * dt) + b.M))
    return s, dt, b, ng


def test_blif_envelope_sum_rule():
    s, dt, b, ng = _blif_problem()
    ms = range(-(b.M - 1), ng + 1)
    Z = zfill.assemble_dense(s, [kernels.EnvelopeKernel(m, dt, FC, b) for m in ms])
    w = 2 * math.pi * FC
    ref = 1j * w * zfill.assemble_dense(s, [kernels.FDKernel(FC)])[0]
    e = np.abs(Z.sum(0) - ref).max() / np.abs(ref).max()
    # the BLIF's partition of unity holds to the window's accuracy, not exactly
    assert e < 2e-2
    # the CPPIF's is exact (its sum rule holds to rounding): the BLIF's error is the window's
    assert e > 1e-6


def test_blif_aim_paths_and_precorrection():
    s, dt, b, ng = _blif_problem()
    a = blif.extrapolation(b.beta, b.M, 3, 6)
    A = aim.AIM(s, 16, 0.3 * ph.C0 / FC, dt, FC, ng, basis=b, fold_a=a)
    assert A.mn <= ng and A.mlo == -2
    rng = np.random.default_rng(4)
    x = rng.standard_normal(s.ns) + 1j * rng.standard_normal(s.ns)
    for m in (0, 1, 3):
        d = A.far_matvec(m, x, direct=True)
        assert np.abs(A.far_matvec(m, x) - d).max() <= 1e-12 * np.abs(d).max()

    def exact(r, c, ms):
        return zfill.assemble_pairs(s, r, c, [kernels.EnvelopeKernel(m, dt, FC, b) for m in ms])

    vals = A.near_values(exact)
    rr, cc = A.rows[::13], A.cols[::13]
    ms = list(range(-(b.M - 1), A.mn + 1))
    z = exact(rr, cc, ms)
    zf = blif.fold({m: z[i] for i, m in enumerate(ms)}, a, A.mn)
    for m in range(A.mn + 1):
        got = vals[m][::13] + A.far_pairs(m, rr, cc)
        assert np.abs(got - zf[m]).max() <= 1e-12 * np.abs(zf[0]).max(), m
