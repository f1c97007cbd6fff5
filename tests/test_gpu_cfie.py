"""The combined-field equation (alpha = 0.5, the paper's spheres, Sec. 2.1
and Sec. 5.1) on the GPU against the FP64 oracle, through the C ABI.

The MFIE's far part runs as a second pass of the far pipeline (its curl
test projection and Green spectra in place of the EFIE's, the same
anterpolated currents and history ring), so every y/z and x engine, the
time blocks and the whole-step graphs take it.  Tolerances as for the EFIE:
FP64 operators <= 1e-12, FP32 <= 1e-5, marches <= 1e-10 of the peak
current against the LU-solved oracle march."""
import sys

import numpy as np
import pytest

import workloads as W
from gpu_cases import gpu_problem, oracle_aim, oracle_dense_aim, oracle_matvec, params_of, rel
from oracle import excitation, march, mfie

pytestmark = pytest.mark.gpu

L2 = W.SPHERE_L2.name
L3 = W.SPHERE_L3.name
A5 = 0.5
ENGINES = [(0, 0), (1, 1), (1, 0), (0, 1), (2, 1), (2, 0), (3, 0), (3, 1)]


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


def _with_engine(P, engine):
    d = P.tuning()
    d["yz_engine"], d["x_engine"] = engine
    P.set_tuning(d)
    assert (P.tuning()["yz_engine"], P.tuning()["x_engine"]) == engine


def _cfie_excitation(s, nt, dt, kh, pp, wl):
    inc = (s, nt, dt, kh, pp, wl.sigma, wl.td, wl.f0)
    return A5 * excitation.excitation(*inc) + (1 - A5) * mfie.excitation_h(*inc)


@pytest.mark.parametrize("name", [L2, L3])
def test_cfie_setup_matches_oracle(torch, name):
    _say("cfie setup", name)
    s, A, vals, p = oracle_aim(name, A5)
    P = gpu_problem(name, alpha=A5)
    assert P.info["mn"] == A.mn
    H = P.export("curl_lambda")
    assert np.abs(H[:, 3]).max() == 0.0
    assert np.abs(H[:, :3] - A.H).max() <= 1e-13 * np.abs(A.H).max()
    near = P.export("near")
    for m in range(A.mn + 1):
        assert np.abs(near[m] - vals[m]).max() <= 1e-12 * np.abs(vals[0]).max(), m
    P.close()


def test_cfie_excitation(torch):
    _say("cfie excitation")
    wl = W.SPHERE_L3
    p = params_of(wl)
    from oracle import geometry
    s = geometry.Surface(p["xyz"], p["tri"], p["rwg"])
    kh = W.unit_vectors(4, 2, 2)
    pp = W.polarisations(4, kh)
    P = gpu_problem(wl.name, batch=2, nt=30, alpha=A5)
    V = P.excitation(kh, pp, wl.sigma, wl.td).cpu().numpy()
    assert rel(V, _cfie_excitation(s, 30, p["dt"], kh, pp, wl)) <= 1e-13
    P.close()


@pytest.mark.parametrize("name,prec,tol", [(L2, 0, 1e-12), (L3, 0, 1e-12), (L3, 1, 1e-5)])
def test_cfie_apply_z_and_delayed_field(torch, name, prec, tol):
    _say("cfie apply_z / delayed", name, prec)
    s, A, vals, p = oracle_aim(name, A5)
    P = gpu_problem(name, precision=prec, alpha=A5)
    x = W.complex_normal(31, (1, s.ns))
    for m in range(p["ng"] + 1):
        y = P.apply_z(m, _dev(torch, x)).cpu().numpy()
        ref = oracle_matvec(name, m, x, direct=False, alpha=A5)
        assert rel(y, ref) <= tol, (m, rel(y, ref))
    hist = W.complex_normal(32, (p["ng"], 1, s.ns))
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()
    ref = sum(oracle_matvec(name, m, hist[m - 1], direct=False, alpha=A5) for m in range(1, p["ng"] + 1))
    assert rel(b, ref) <= tol, rel(b, ref)
    P.close()


@pytest.mark.parametrize("engine", ENGINES, ids=[f"yz{a}_x{b}" for a, b in ENGINES])
def test_cfie_engines(torch, engine):
    """Every y/z and x engine on the 16^3 grid (the register kernels' size)."""
    _say("cfie engine", engine)
    s, A, vals, p = oracle_aim(L2, A5)
    P = gpu_problem(L2, alpha=A5)
    _with_engine(P, engine)
    x = W.complex_normal(33, (1, s.ns))
    for m in (0, 1, p["ng"]):
        y = P.apply_z(m, _dev(torch, x)).cpu().numpy()
        ref = oracle_matvec(L2, m, x, direct=False, alpha=A5)
        assert rel(y, ref) <= 1e-12, (m, rel(y, ref))
    hist = W.complex_normal(34, (p["ng"], 1, s.ns))
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()
    ref = sum(oracle_matvec(L2, m, hist[m - 1], direct=False, alpha=A5) for m in range(1, p["ng"] + 1))
    assert rel(b, ref) <= 1e-12, rel(b, ref)
    P.close()


def test_cfie_march_matches_oracle_and_is_stable(torch):
    """The +-20 % level-2 sphere over its 200 steps: the EFIE march of this
    band grows (Sec. 3.1.1, parity is only checked over its first 30 steps),
    the CFIE march matches the oracle's LU march at every step and its
    current decays after the pulse."""
    wl = W.SPHERE_L2
    nt = wl.nt
    _say("cfie march", wl.name, nt)
    s, A, vals, p = oracle_aim(L2, A5)
    kh, pp = wl.incidence()
    V = _cfie_excitation(s, nt, p["dt"], kh, pp, wl)
    I_ref = march.march_dense(oracle_dense_aim(L2, A5), V)
    P = gpu_problem(L2, tol=1e-13, nt=nt, alpha=A5)
    I, st = P.march(_dev(torch, V))
    I = I.cpu().numpy()
    nrm = np.linalg.norm(I_ref[:, 0], axis=1)
    peak = nrm.max()
    _say("  iters", st["total_iters"], "rel", rel(I, I_ref), "last/peak", nrm[-1] / peak)
    for l in range(nt):
        assert np.linalg.norm(I[l] - I_ref[l]) <= 1e-10 * peak, l
    assert nrm[-1] < 1e-6 * peak
    assert st["unstable_step"] == -1
    P.close()


@pytest.mark.parametrize("engine", [(2, 1), (3, 1)], ids=["yz2_x1", "yz3_x1"])
def test_cfie_time_blocks_equal_the_plain_delayed_field(torch, engine):
    """Both passes keep block sums of the same block: a march with time
    blocks of 3 equals the one without (rounding only)."""
    wl = W.SPHERE_L2
    nt = 40
    _say("cfie time blocks", engine)
    s, A, vals, p = oracle_aim(L2, A5)
    kh, pp = wl.incidence()
    V = _cfie_excitation(s, nt, p["dt"], kh, pp, wl)
    out = {}
    for blk in (1, 3):
        P = gpu_problem(L2, tol=1e-13, nt=nt, alpha=A5)
        _with_engine(P, engine)
        d = P.tuning()
        d["delay_block"] = blk
        P.set_tuning(d)
        I, _ = P.march(_dev(torch, V))
        out[blk] = I.cpu().numpy()
        P.close()
    assert rel(out[3], out[1]) <= 1e-12


def test_cfie_step_graphs_equal_the_eager_march(torch):
    from paper_1408_7060_amd import _lib
    wl = W.SPHERE_L2
    nt = 40
    _say("cfie step graphs")
    s, A, vals, p = oracle_aim(L2, A5)
    kh, pp = wl.incidence()
    V = _cfie_excitation(s, nt, p["dt"], kh, pp, wl)
    out = {}
    for fl in (_lib.F_IMPLICIT_STOP, _lib.F_IMPLICIT_STOP | _lib.F_STEP_GRAPH):
        P = gpu_problem(L2, tol=1e-10, nt=nt, alpha=A5, flags=fl)
        _with_engine(P, (2, 1))
        I, st = P.march(_dev(torch, V))
        out[fl] = (I.cpu().numpy(), st)
        P.close()
    (Ie, _), (Ig, stg) = out.values()
    assert stg["graph_steps"] > 0
    assert np.array_equal(Ie, Ig)


def test_cfie_fp32_march_residual_check(torch):
    from paper_1408_7060_amd import _lib
    wl = W.SPHERE_L3
    nt = 40
    _say("cfie fp32 residual check")
    P = gpu_problem(L3, precision=1, tol=1e-6, nt=nt, alpha=A5, flags=_lib.F_RESIDUAL_CHECK)
    kh, pp = wl.incidence()
    V = P.excitation(kh, pp, wl.sigma, wl.td)
    I, st = P.march(V)
    _say("  checks", st["residual_checks"], "worst", st["max_residual64"])
    assert st["residual_checks"] >= 2
    assert st["max_residual64"] <= 1e-4
    P.close()


def test_cfie_adjoint_is_refused(torch):
    from paper_1408_7060_amd import EtaimError
    P = gpu_problem(L2, nt=8, alpha=A5)
    S = _dev(torch, W.complex_normal(35, (8, 1, P.ns)))
    with pytest.raises(EtaimError):
        P.adjoint_march(S)
    P.close()


def test_cfie_stability_of_the_level4_sphere_depends_on_the_time_step(torch):
    """The bench's level-4 sphere (7680 RWG, +-10 %), one direction, FP32.
    At the paper's oversampling beta = 1/5 the CFIE march decays after the
    pulse while the EFIE march's growing mode is flagged.  At the bench's
    N_g = 24 (beta = f_bw dt ~ 1/54, c dt = 9.3 cm, about one mesh edge)
    both grow: the CFIE's damping is lost at small time steps (the oracle's
    companion matrices of the level-2 sphere show the same, spectral radius
    0.87 at beta = 1/5 and 1.06-1.18 at 1/10-1/40)."""
    from paper_1408_7060_amd import Problem
    wl = W.SPHERE_L4_BATCH
    p = params_of(wl)
    kh, pp = wl.incidence()
    res = {}
    for beta, nt in ((0.2, 200), (None, wl.nt)):
        for alpha in (1.0, A5):
            kw = dict(fc=wl.f0, nt=nt, grid=wl.grid, d_near=p["d_near"], precision=1, batch=1, tol=1e-5,
                      restart=50, maxit=2000, alpha=alpha)
            if beta:
                kw.update(beta=beta, f_bw=wl.f_bw)
            else:
                kw["ng"] = wl.ng
            P = Problem(p["xyz"], p["tri"], p["rwg"], **kw)
            V = P.excitation(kh[:1], pp[:1], wl.sigma, wl.td)
            I, st = P.march(V)
            nrm = np.linalg.norm(I[:, 0].cpu().numpy(), axis=1)
            res[beta, alpha] = (st["unstable_step"], nrm[-1] / nrm.max())
            _say("level-4", "beta", beta, "ng", P.info["ng"], "alpha", alpha, "unstable step", st["unstable_step"],
                 "last/peak", nrm[-1] / nrm.max())
            P.close()
    assert res[0.2, A5][0] == -1 and res[0.2, A5][1] < 1e-3
    assert res[0.2, 1.0][0] >= 0
    assert res[None, 1.0][0] >= 0 and res[None, A5][0] >= 0
