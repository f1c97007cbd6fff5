"""Batched-GMRES schedules (calls through the C ABI): Arnoldi steps enqueued
several at a time behind the device-side gate, and Arnoldi steps replayed
from captured HIP graphs, give the same march as one host check per step.

Each graph march replays every captured step many times, with the
library's own eager work (cycle starts, delayed field, commit) and host
synchronisations between replays; every replayed march is compared with
the eager one."""
import sys

import numpy as np
import pytest

import workloads as W
from gpu_cases import gpu_problem, oracle_aim
from oracle import excitation

pytestmark = pytest.mark.gpu

F_CONTINUE_ON_NOCONV, F_GRAPH = 1, 4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _excitation(name, nt, nb, seed):
    wl = W.WORKLOADS[name]
    s, A, vals, p = oracle_aim(name)
    kh = W.unit_vectors(seed, nb, 3)
    pp = W.polarisations(seed, kh)
    return excitation.excitation(s, nt, p["dt"], kh, pp, wl.sigma, wl.td, wl.f0)


def _march(torch, name, V, adjoint=False, **kw):
    P = gpu_problem(name, nt=V.shape[0], batch=V.shape[1], **kw)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    I, st = (P.adjoint_march(Vd) if adjoint else P.march(Vd))
    out = I.cpu().numpy(), st["total_iters"], list(st["iters_per_step"])
    runs = [out]
    if kw["flags"] & F_GRAPH:
        # second march on the same context: pure replays of the captured steps
        I2, st2 = (P.adjoint_march(Vd) if adjoint else P.march(Vd))
        runs.append((I2.cpu().numpy(), st2["total_iters"], list(st2["iters_per_step"])))
    P.close()
    return runs


# restart 7 forces several GMRES cycles per step; B = 3 columns converge at
# different iterations, so the device-side masks and the gate both matter
CASES = [("fp64_L2", W.SPHERE_L2.name, 0, 1e-12), ("fp32_L3", W.SPHERE_L3.name, 1, 1e-6)]


@pytest.mark.parametrize("label,name,prec,tol", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("adjoint", [False, True], ids=["forward", "adjoint"])
def test_gated_and_graph_schedules_equal_eager(torch, label, name, prec, tol, adjoint):
    nt = 12
    V = _excitation(name, nt, 3, 11)
    common = dict(precision=prec, tol=tol, restart=7, adjoint=adjoint)
    plain = F_CONTINUE_ON_NOCONV
    _say("schedule", label, "adjoint" if adjoint else "forward")
    (I0, it0, per0), = _march(torch, name, V, flags=plain, **common)
    assert it0 > 0 and np.isfinite(I0).all()
    for kw in (dict(flags=plain, sync_every=5), dict(flags=plain | F_GRAPH, sync_every=1),
               dict(flags=plain | F_GRAPH, sync_every=4)):
        for r, (I, it, per) in enumerate(_march(torch, name, V, **common, **kw)):
            _say("  ", kw, "run", r, "iters", it, "vs", it0, "max|d|", float(np.abs(I - I0).max()))
            assert it == it0 and per == per0
            np.testing.assert_array_equal(I, I0)


# ---------------------------------------------------------------------------
# Autotuner and explicit settings

from gpu_cases import oracle_matvec, rel  # noqa: E402


def _plans(L, maxp):
    out = []

    def rec(n, cur):
        if n == 1:
            out.append(cur)
            return
        if len(cur) == maxp:
            return
        for r in (16, 12, 8, 6, 4, 3, 2):
            if n % r == 0:
                rec(n // r, cur + [r])
    rec(L, [])
    return out


@pytest.mark.parametrize("name", [W.SPHERE_L2.name, W.SPHERE_L3.name])
def test_every_radix_plan_matches_oracle(torch, name):
    """Each admissible plan of the padded length (every codelet 2..16 in
    every pass position) gives the oracle's matvec to FP64 rounding."""
    s, A, vals, p = oracle_aim(name)
    P = gpu_problem(name)
    base = P.tuning()
    L = P.info["padded"][0]
    x = W.complex_normal(21, (1, s.ns))
    ref = oracle_matvec(name, 1, x, direct=(name == W.SPHERE_L2.name))
    xd = torch.from_numpy(x).cuda()
    plans = _plans(L, 3)
    _say("plans of", L, len(plans))
    tried = 0
    for pl in plans:
        for axes in (("radix_x",), ("radix_y", "radix_z")):
            d = dict(base)
            for ax in axes:
                d[ax] = pl
            try:
                P.set_tuning(d)
            except Exception as e:  # plan does not fit the register staging
                assert getattr(e, "code", None) == -7, e
                continue
            y = P.apply_z(1, xd).cpu().numpy()
            e = rel(y, ref)
            assert e <= 1e-12, (pl, axes, e)
            tried += 1
    _say("  plans run", tried)
    assert tried >= len(plans)
    P.close()


def test_set_tuning_rejects_bad_settings(torch):
    P = gpu_problem(W.SPHERE_L2.name)
    base = P.tuning()
    for bad, code in ((dict(radix_x=[5, 6]), -1), (dict(radix_x=[16]), -1), (dict(interp_waves=5), -7),
                      (dict(gather_rows=0), -1), (dict(sync_every=1000), -7),
                      (dict(delay_block=0), -7), (dict(delay_block=9), -7)):
        d = dict(base)
        d.update(bad)
        with pytest.raises(Exception) as ei:
            P.set_tuning(d)
        assert ei.value.code == code, (bad, ei.value)
    assert P.tuning() == base
    P.close()


@pytest.mark.parametrize("name,prec,tol", [(W.SPHERE_L3.name, 1, 1e-5), (W.SPHERE_L2.name, 0, 1e-12)])
def test_autotune_keeps_the_operator_and_caches(torch, tmp_path, name, prec, tol):
    s, A, vals, p = oracle_aim(name)
    x = W.complex_normal(22, (1, s.ns))
    xd = torch.from_numpy(x).cuda()
    ref = oracle_matvec(name, 0, x, direct=(name == W.SPHERE_L2.name))
    cache = str(tmp_path / "tune.jsonl")
    solver = dict(precision=prec, tol=1e-6 if prec else 1e-12, flags=F_CONTINUE_ON_NOCONV)
    P = gpu_problem(name, **solver)
    t = P.autotune(budget_ms=3000, cache=cache)
    _say("tuned", name, t)
    assert t["apply_ms"] > 0 and t["solve_ms"] > 0
    assert rel(P.apply_z(0, xd).cpu().numpy(), ref) <= tol
    # the tuned march equals the untuned one (same operator, same schedule semantics)
    V = _excitation(name, 6, 1, 23)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    I1, _ = P.march(Vd)
    P.close()
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1
    P2 = gpu_problem(name, **solver)
    I0, _ = P2.march(Vd)
    t2 = P2.autotune(budget_ms=3000, cache=cache)   # cache hit: applied without timing
    assert {k: t2[k] for k in t2 if not k.endswith("_ms")} == {k: t[k] for k in t if not k.endswith("_ms")}
    assert t2["apply_ms"] == 0
    assert len(open(cache).read().strip().splitlines()) == 1
    assert rel(P2.apply_z(0, xd).cpu().numpy(), ref) <= tol
    P2.close()
    assert rel(I1.cpu().numpy(), I0.cpu().numpy()) <= (1e-4 if prec else 1e-10)


@pytest.mark.parametrize("name,prec,tol,bound", [(W.SPHERE_L2.name, 0, 1e-13, 1e-11),
                                                 (W.SPHERE_L3.name, 1, 1e-6, 1e-5)])
def test_initial_guess_order(torch, name, prec, tol, bound):
    """The extrapolated initial guess changes the march only within the
    GMRES tolerance; the adaptive order (the one that best predicted the
    previous step) takes at most a few percent more iterations than the
    previous solution as the guess, also where the envelope is coarsely
    sampled and extrapolation does not pay."""
    V = _excitation(name, 24, 2, 41)
    out = {}
    for order in (0, 1, 4):
        P = gpu_problem(name, precision=prec, tol=tol, nt=24, batch=2, flags=F_CONTINUE_ON_NOCONV)
        d = P.tuning()
        d["guess_order"] = order
        P.set_tuning(d)
        I, st = P.march(torch.from_numpy(np.ascontiguousarray(V)).cuda())
        out[order] = (I.cpu().numpy(), st["total_iters"])
        P.close()
        _say("guess order", order, "iterations", st["total_iters"])
    ref = out[1][0]
    for order in (0, 4):
        e = float(np.linalg.norm(out[order][0] - ref) / np.linalg.norm(ref))
        assert e <= bound, (order, e)
    assert out[4][1] <= 1.05 * out[1][1]


@pytest.mark.parametrize("adjoint", [False, True], ids=["forward", "adjoint"])
@pytest.mark.parametrize("name,prec,tol,bound", [(W.SPHERE_L2.name, 0, 1e-13, 1e-11),
                                                 (W.SPHERE_L3.name, 1, 1e-6, 1e-4)])
def test_preconditioners_agree(torch, name, prec, tol, bound, adjoint):
    """The near-zone sparse approximate inverse and the Jacobi diagonal give
    the same march within the GMRES tolerance; the approximate inverse needs
    fewer iterations."""
    V = _excitation(name, 16, 2, 43)
    out = {}
    for pc in (0, 1):
        P = gpu_problem(name, precision=prec, tol=tol, nt=16, batch=2, flags=F_CONTINUE_ON_NOCONV)
        d = P.tuning()
        d["precond"] = pc
        P.set_tuning(d)
        Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
        I, st = P.adjoint_march(Vd) if adjoint else P.march(Vd)
        out[pc] = (I.cpu().numpy(), st["total_iters"])
        P.close()
        _say("precond", pc, "iterations", st["total_iters"])
    e = float(np.linalg.norm(out[1][0] - out[0][0]) / np.linalg.norm(out[0][0]))
    assert e <= bound, e
    assert out[1][1] < out[0][1]


@pytest.mark.parametrize("name,prec,tol,bound", [(W.SPHERE_L2.name, 0, 1e-12, 1e-11),
                                                 (W.SPHERE_L3.name, 1, 1e-6, 1e-5)])
@pytest.mark.parametrize("adjoint", [False, True], ids=["forward", "adjoint"])
def test_implicit_stop(torch, name, prec, tol, bound, adjoint):
    """Stopping on the GMRES residual estimate (no confirming true residual)
    keeps the Arnoldi iterations of every step and the march within the
    tolerance of the confirmed one; every step's reported residual is the
    estimate, below the tolerance."""
    F_IMPLICIT_STOP = 8
    V = _excitation(name, 16, 3, 43)
    common = dict(precision=prec, tol=tol, adjoint=adjoint)
    (I0, it0, per0), = _march(torch, name, V, flags=F_CONTINUE_ON_NOCONV, **common)
    P = gpu_problem(name, nt=V.shape[0], batch=V.shape[1], flags=F_CONTINUE_ON_NOCONV | F_IMPLICIT_STOP,
                    precision=prec, tol=tol)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    I1, st = (P.adjoint_march(Vd) if adjoint else P.march(Vd))
    P.close()
    _say("implicit stop", name, "iters", st["total_iters"], "vs", it0, "max resid", st["max_rel_residual"])
    assert st["total_iters"] <= it0
    assert st["max_rel_residual"] <= tol
    assert rel(I1.cpu().numpy(), I0) <= bound


def test_profiling_mask(torch):
    """Tracing a subset of the kernel classes counts launches of those only
    and leaves the march bit for bit as untraced; tracing every class then
    counts the marker-timed classes too."""
    name = W.SPHERE_L2.name
    V = _excitation(name, 12, 2, 47)
    P = gpu_problem(name, nt=V.shape[0], batch=V.shape[1], flags=F_CONTINUE_ON_NOCONV)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    I0 = P.march(Vd)[0].cpu().numpy()
    some = ("yz_green", "yz_delayed")
    P.set_profiling(classes=some)
    I1 = P.march(Vd)[0].cpu().numpy()
    ks = P.kernel_stats()
    P.set_profiling(True)
    I2 = P.march(Vd)[0].cpu().numpy()
    ks2 = P.kernel_stats()
    P.set_profiling(False)
    P.close()
    _say("profiling mask", {n: v["launches"] for n, v in ks.items()}, {n: v["launches"] for n, v in ks2.items()})
    assert all(ks[n]["launches"] > 0 and ks[n]["ms"] > 0 for n in some)
    assert all(v["launches"] == 0 for n, v in ks.items() if n not in some)
    assert ks2["krylov"]["launches"] > 0 and ks2["anterp_x"]["launches"] > 0
    assert ks2["yz_green"]["launches"] == ks["yz_green"]["launches"]
    assert np.array_equal(I1, I0) and np.array_equal(I2, I0)


@pytest.mark.parametrize("xe", [1, 0], ids=["x_register", "x_lds"])
def test_profiling_on_the_line_engine(torch, xe):
    """Every class traced on a grid whose planes take the line-pass engine
    (level-3 sphere on a 72^3 grid: four-step lines of 144 points, the x
    stage from the anterpolated grid or the LDS gather): all event pairs
    resolve, every matvec class is counted, and the march is bit for bit
    the untraced one."""
    name = W.SPHERE_L3.name
    V = _excitation(name, 8, 1, 48)
    P = gpu_problem(name, nt=V.shape[0], batch=V.shape[1], flags=F_CONTINUE_ON_NOCONV, grid=72)
    P.set_tuning(dict(P.tuning(), x_engine=xe))
    assert (P.tuning()["yz_engine"], P.tuning()["x_engine"]) == (3, xe)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    I0 = P.march(Vd)[0].cpu().numpy()
    P.set_profiling(True)
    I1 = P.march(Vd)[0].cpu().numpy()
    ks = P.kernel_stats()
    P.set_profiling(False)
    P.close()
    _say("line engine profiling", {n: v["launches"] for n, v in ks.items()})
    for n in ("anterp_x", "yz_green", "fft_x_inv", "interp_near", "yz_delayed", "yz_commit", "krylov"):
        assert ks[n]["launches"] > 0 and ks[n]["ms"] > 0, n
    assert np.array_equal(I1, I0)
