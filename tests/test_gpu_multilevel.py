"""Multilevel time blocks of the delayed field (delay mode 1: the temporal
direction of the blocked space-time transforms that evaluate the right-hand
side of eq. (5), Sec. 4) against the FP64 oracle's direct history sum,
through the C ABI.

Lags 1..2 are summed at each step; lags [3 2^k, 6 2^k) form level k, whose
share of the next 3 2^k steps' sums is a temporal DFT convolution
(overlap-save) over the last block of history.  Two long-history problems:

* level-4 sphere (7680 RWG, 48^3 grid), N_g = 47, M_n = 13: levels of 3, 6,
  12 and 24 steps, the top one ending inside the history (lags 24..47);
* level-2 sphere (480 RWG, 16^3 grid), N_g = 95, M_n = 81: all five levels
  (the top one's 96-point transforms), the near history live over 81 lags;
* the same sphere with N_g = 150: two further 48-step segments (lags
  96..143 and 144..150) past the five levels.

The oracle sums every lag directly (near and far part) on sampled rows, so
each level's transform, its product with the lag segment's spectrum and
its accumulation are checked against the definition.  A march accumulates
the level sums step by step (the incremental passes, their ring of
per-step accumulators and its clearing), which the march tests compare
with the oracle-pinned direct sum of delay mode 0 on the same problem, also
after a resume from a saved state (the accumulators are rebuilt from the
ring) and for the adjoint march (conj(G))."""
import dataclasses
import functools
import sys

import numpy as np
import pytest

import workloads as W
from gpu_cases import gpu_problem, params_of, rel
from oracle import aim, excitation, geometry, kernels, mfie, zfill

pytestmark = pytest.mark.gpu

L4 = W.SPHERE_L4_NG47
L2 = W.SPHERE_L2_NG95
COLS = (0, 1)
F_CONTINUE_ON_NOCONV = 1


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def _with_engine(P, yz, xe):
    d = P.tuning()
    d["yz_engine"], d["x_engine"] = yz, xe
    P.set_tuning(d)
    assert (P.tuning()["yz_engine"], P.tuning()["x_engine"]) == (yz, xe)


@functools.lru_cache(maxsize=None)
def _oracle_rows(name, nrows, alpha=1.0):
    """(AIM, params, sampled rows, near selection, exact near values of those
    rows); alpha < 1: the CFIE."""
    wl = W.WORKLOADS[name]
    p = params_of(wl)
    s = geometry.Surface(p["xyz"], p["tri"], p["rwg"])
    A = aim.AIM(s, wl.grid, p["d_near"], p["dt"], wl.f0, p["ng"], alpha=alpha)
    rows = np.sort(W.rng(0, 7).choice(s.ns, nrows, replace=False))

    def exact(r, c, ms):
        if alpha != 1.0:
            return mfie.cfie_pairs(s, r, c, ms, p["dt"], wl.f0, alpha)
        return zfill.assemble_pairs(s, r, c, [kernels.EnvelopeKernel(m, p["dt"], wl.f0) for m in ms])

    sel, vals = A.near_values_rows(exact, rows)
    _say(f"oracle {name}: N_g {p['ng']}, M_n {A.mn}, rows {nrows}, near pairs {int(sel.sum())}, alpha {alpha}")
    return A, p, rows, sel, vals


@functools.lru_cache(maxsize=None)
def _delayed_ref(name, nrows, alpha=1.0):
    """History [N_g, 2, ns] (hist[m-1] = I_{l-m}) and the oracle's direct sum
    sum_{m=1}^{N_g} (Z^near_m + Z^FFT_m) hist[m-1] on the sampled rows."""
    A, p, rows, sel, vals = _oracle_rows(name, nrows, alpha)
    ng = p["ng"]
    hist = W.complex_normal(71, (ng, 2, A.surf.ns))
    ref = []
    for c in COLS:
        far = A.far_sum_rows([(m, A.spectra(hist[m - 1, c])) for m in range(1, ng + 1)], rows)
        near = sum(A.near_rows(sel, vals[m], hist[m - 1, c], rows) for m in range(1, min(A.mn, ng) + 1))
        ref.append(far + near)
    return hist, np.array(ref)


L2X = W.SPHERE_L2_NG150
CASES = [(L4.name, 48, 0, 1e-12), (L4.name, 48, 1, 1e-5), (L2.name, 48, 0, 1e-12), (L2.name, 48, 1, 1e-5),
         (L2X.name, 48, 0, 1e-12), (L2X.name, 48, 1, 1e-5)]


@pytest.mark.parametrize("engine", [(2, 1), (3, 1), (0, 0)], ids=["zlines", "lines", "planes"])
@pytest.mark.parametrize("name,nrows,prec,tol", CASES, ids=["L4ng47_fp64", "L4ng47_fp32", "L2ng95_fp64",
                                                             "L2ng95_fp32", "L2ng150_fp64", "L2ng150_fp32"])
def test_multilevel_delayed_field_matches_oracle(torch, name, nrows, prec, tol, engine):
    A, p, rows, sel, vals = _oracle_rows(name, nrows)
    hist, ref = _delayed_ref(name, nrows)
    P = gpu_problem(name, precision=prec, batch=2, nt=8)
    assert P.info["ng"] == p["ng"] and P.info["mn"] == A.mn
    assert P.delay_mode() == 1      # the default beyond the one-level time blocks' N_g <= 32
    _with_engine(P, *engine)
    P.set_delay_mode(1)
    assert P.delay_mode() == 1
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()[list(COLS)][:, rows]
    e = rel(b, ref)
    _say("multilevel delayed", name, "engine", engine, "fp32" if prec else "fp64", "rel", e)
    assert e <= tol
    # the direct sum of mode 0 on the same context
    P.set_delay_mode(0)
    b0 = P.delayed_field(_dev(torch, hist)).cpu().numpy()[list(COLS)][:, rows]
    _say("  mode 0 rel", rel(b0, ref))
    assert rel(b0, ref) <= tol
    P.close()


@pytest.mark.parametrize("engine", [(2, 1), (3, 1)], ids=["zlines", "lines"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)], ids=["fp64", "fp32"])
def test_multilevel_cfie_delayed_field_matches_oracle(torch, prec, tol, engine):
    """The CFIE (alpha = 0.5, Sec. 2.1): the EFIE and MFIE passes each sum
    their history with their own level tables and accumulators (N_g = 47,
    level-4 sphere)."""
    A, p, rows, sel, vals = _oracle_rows(L4.name, 48, 0.5)
    hist, ref = _delayed_ref(L4.name, 48, 0.5)
    P = gpu_problem(L4.name, precision=prec, batch=2, nt=8, alpha=0.5)
    _with_engine(P, *engine)
    P.set_delay_mode(1)
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()[list(COLS)][:, rows]
    e = rel(b, ref)
    _say("multilevel CFIE delayed", engine, "fp32" if prec else "fp64", "rel", e)
    assert e <= tol
    P.close()


def _excitation(name, nt, nb, seed):
    wl = W.WORKLOADS[name]
    p = params_of(wl)
    s = geometry.Surface(p["xyz"], p["tri"], p["rwg"])
    kh = W.unit_vectors(seed, 2, nb)
    pp = W.polarisations(seed, kh)
    return excitation.excitation(s, nt, p["dt"], kh, pp, wl.sigma, wl.td, wl.f0)


def _march(torch, V, mode, engine, prec=0, tol=1e-13, nt=None, alpha=1.0, name=L2.name):
    P = gpu_problem(name, precision=prec, tol=tol, batch=V.shape[1], nt=nt or V.shape[0],
                    flags=F_CONTINUE_ON_NOCONV, alpha=alpha)
    _with_engine(P, *engine)
    P.set_delay_mode(mode)
    I, st = P.march(_dev(torch, V))
    P.close()
    return I.cpu().numpy(), st


@pytest.mark.parametrize("engine", [(2, 1), (3, 1), (0, 0)], ids=["zlines", "lines", "planes"])
def test_multilevel_march_equals_direct_sum(torch, engine):
    """240 steps at N_g = 95 (the accumulator ring of 51 slots wraps four
    times; every level passes at least twice past the history's length)."""
    nt = 240
    V = _excitation(L2.name, nt, 2, 81)
    I1, st1 = _march(torch, V, 1, engine)
    I0, st0 = _march(torch, V, 0, engine)
    e = rel(I1, I0)
    _say("multilevel march", engine, "rel to direct", e, "iters", st1["total_iters"], st0["total_iters"])
    assert np.isfinite(I1).all()
    assert e <= 1e-10
    # FP32 with the multilevel sums against the FP64 direct march
    I32, _ = _march(torch, V, 1, engine, prec=1, tol=1e-7)
    e32 = rel(I32, I0)
    _say("  fp32 multilevel vs fp64 direct", e32)
    assert e32 <= 1e-4


def test_multilevel_past_lag_95_march_equals_direct_sum(torch):
    """N_g = 150: the five levels and two further 48-step segments (lags
    96..143 and 144..150) over a 250-step march."""
    nt = 250
    V = _excitation(L2X.name, nt, 1, 86)
    I1, _ = _march(torch, V, 1, (3, 1), name=L2X.name)
    I0, _ = _march(torch, V, 0, (3, 1), name=L2X.name)
    e = rel(I1, I0)
    _say("multilevel march N_g 150 rel to direct", e)
    assert np.isfinite(I1).all() and e <= 1e-10


def test_multilevel_cfie_march_equals_direct_sum(torch):
    """The CFIE march with multilevel sums in both passes against the CFIE
    march with the direct sum (N_g = 95, 150 steps)."""
    nt = 150
    V = _excitation(L2.name, nt, 1, 84)
    I1, _ = _march(torch, V, 1, (2, 1), alpha=0.5)
    I0, _ = _march(torch, V, 0, (2, 1), alpha=0.5)
    e = rel(I1, I0)
    _say("multilevel CFIE march rel to direct", e)
    assert np.isfinite(I1).all()
    assert e <= 1e-10


def test_multilevel_resume_and_adjoint(torch):
    """A march split at a step inside every level's block, continued on the
    same context (incremental passes) and from a saved state in a fresh
    context (accumulators rebuilt from the ring), equals the uninterrupted
    multilevel march bit for bit; the adjoint march with multilevel sums
    (conj(G)) equals the adjoint march with the direct sum."""
    nt, split = 120, 77
    V = _excitation(L2.name, nt, 1, 82)
    Vd = _dev(torch, V)
    kw = dict(precision=0, tol=1e-13, batch=1, nt=nt, flags=F_CONTINUE_ON_NOCONV)
    P = gpu_problem(L2.name, **kw)
    P.set_delay_mode(1)
    I_full, _ = P.march(Vd)
    I_full = I_full.cpu().numpy()
    I1, _ = P.march(Vd, nsteps=split)
    state = P.save_state()
    I1, _ = P.march_continue(Vd, I1, split, nt - split)
    _say("multilevel resume same context max|d|", float(np.abs(I1.cpu().numpy() - I_full).max()))
    np.testing.assert_array_equal(I1.cpu().numpy(), I_full)
    Q = gpu_problem(L2.name, **kw)
    Q.set_delay_mode(1)
    I2 = torch.zeros_like(Vd)
    I2[:split] = _dev(torch, I_full[:split])
    Q.load_state(state)
    I2, _ = Q.march_continue(Vd, I2, split, nt - split)
    _say("  loaded context max|d|", float(np.abs(I2.cpu().numpy() - I_full).max()))
    np.testing.assert_array_equal(I2.cpu().numpy(), I_full)
    Q.close()
    # adjoint march: multilevel against direct
    S = _dev(torch, W.complex_normal(83, (nt, 1, V.shape[2])))
    L1, _ = P.adjoint_march(S)
    P.set_delay_mode(0)
    L0, _ = P.adjoint_march(S)
    ea = rel(L1.cpu().numpy(), L0.cpu().numpy())
    _say("  adjoint multilevel vs direct", ea)
    assert ea <= 1e-10
    P.close()


@pytest.mark.parametrize("ng", [5, 11, 23])
def test_multilevel_few_levels(torch, ng):
    """N_g = 5, 11, 23: one, two and three levels, the top one inside the
    fused low-level pass (it starts the accumulator slots there); the
    delayed field against the oracle's direct sum on sampled rows (FP64) and
    a 50-step march (the pulse and its first crossing) against the direct
    sum.  Later steps are left out: at N_g = 5 the EFIE march's growing mode
    takes over (Sec. 3.1.1) and amplifies rounding alike for any change of
    summation order (two y/z engines of the direct sum differ by 1e-7 at
    step 89, as the multilevel and direct sums do)."""
    wl = dataclasses.replace(W.SPHERE_L2, name=f"sphere_L2_r0.5_300MHz_ng{ng}", ng=ng, nt=50)
    W.WORKLOADS[wl.name] = wl
    A, p, rows, sel, vals = _oracle_rows(wl.name, 48)
    hist, ref = _delayed_ref(wl.name, 48)
    P = gpu_problem(wl.name, precision=0, batch=2, nt=8)
    _with_engine(P, 2, 1)
    P.set_delay_mode(1)
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()[list(COLS)][:, rows]
    e = rel(b, ref)
    _say("multilevel delayed N_g", ng, "rel", e)
    assert e <= 1e-12
    P.close()
    V = _excitation(wl.name, 50, 2, 85)
    out = []
    for mode in (1, 0):
        Q = gpu_problem(wl.name, precision=0, tol=1e-13, batch=2, nt=50, flags=F_CONTINUE_ON_NOCONV)
        _with_engine(Q, 3, 1)
        Q.set_delay_mode(mode)
        I, _ = Q.march(_dev(torch, V))
        out.append(I.cpu().numpy())
        Q.close()
    em = rel(out[0], out[1])
    _say("  march rel to direct", em)
    assert np.isfinite(out[0]).all() and em <= 1e-10


@pytest.mark.parametrize("alpha", [1.0, 0.5], ids=["efie", "cfie"])
def test_multilevel_blif_delayed_field(torch, alpha):
    """The BLIF (Sec. 3, Sec. 3.1.2): its non-causal kernels are folded into
    Z_0..Z_2, the levels take the lags from 3 on (level-2 sphere, N_g = 4:
    one level, the top one in the fused pass), against the oracle's direct
    sum over every row, EFIE and CFIE."""
    from gpu_cases import oracle_aim, oracle_matvec
    name = W.SPHERE_L2.name
    s_, A, vals, p = oracle_aim(name, alpha, 1)
    ng = p["ng"]
    hist = W.complex_normal(72, (ng, 1, s_.ns))
    ref = sum(oracle_matvec(name, m, hist[m - 1], direct=False, alpha=alpha, basis=1) for m in range(1, ng + 1))
    P = gpu_problem(name, precision=0, alpha=alpha, basis=1)
    _with_engine(P, 2, 1)
    P.set_delay_mode(1)
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()
    e = rel(b, ref)
    _say("multilevel BLIF delayed, alpha", alpha, "N_g", ng, "rel", e)
    assert e <= 1e-12
    P.close()


def test_delay_mode_errors(torch):
    """Mode outside 0/1: EINVAL, the mode unchanged."""
    P = gpu_problem(W.SPHERE_L2.name, nt=4)
    with pytest.raises(Exception) as ei:
        P.set_delay_mode(2)
    assert ei.value.code == -1
    assert P.delay_mode() == 0
    P.close()
