"""Whole-step graphs of the forward march (ETAIM_F_STEP_GRAPH, tuning graph
= 2): every step from the fourth on (and after the first step of a call) is
one replayed HIP graph whose per-step values come from device descriptors,
several steps per host check; a step that does not converge within the
graph's Arnoldi steps stops the replays on the device and is completed
eagerly.  The currents, the per-step iteration counts and the FP64
residual checks equal the eager march's bit for bit, also when the march is
split and continued, and when replays halt (the first steps have a zero
excitation, so the graphs start with two Arnoldi steps, and the pulse that
follows needs more)."""
import sys

import numpy as np
import pytest

import workloads as W
from gpu_cases import gpu_problem, oracle_aim

pytestmark = pytest.mark.gpu

L2 = W.SPHERE_L2.name
F_CONTINUE_ON_NOCONV, F_IMPLICIT_STOP, F_RESIDUAL_CHECK = 1, 8, 16


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _excitation(nt, nb, zero_steps):
    from oracle import excitation
    wl = W.SPHERE_L2
    s, A, vals, p = oracle_aim(L2)
    kh = W.unit_vectors(81, 2, nb)
    pp = W.polarisations(81, kh)
    V = excitation.excitation(s, nt, p["dt"], kh, pp, wl.sigma, (zero_steps + 8) * p["dt"], wl.f0)
    V[:zero_steps] = 0.0
    return V


def _problem(prec, nt, nb, graph, tol):
    P = gpu_problem(L2, precision=prec, nt=nt, batch=nb, tol=tol,
                    flags=F_CONTINUE_ON_NOCONV | F_IMPLICIT_STOP | F_RESIDUAL_CHECK, sync_every=4)
    d = P.tuning()
    assert (d["yz_engine"], d["x_engine"]) == (2, 1)
    d["graph"] = graph
    P.set_tuning(d)
    assert P.tuning()["graph"] == graph
    return P


@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 1e-6)], ids=["fp64", "fp32"])
def test_step_graph_equals_eager(torch, prec, tol):
    nt, nb = 48, 2
    V = torch.from_numpy(np.ascontiguousarray(_excitation(nt, nb, 10))).cuda()
    out = {}
    for graph in (0, 2):
        P = _problem(prec, nt, nb, graph, tol)
        I, st = P.march(V)
        out[graph] = (I.cpu().numpy(), st)
        # split at 21 and continued (the continued call replays from its second step)
        I1, st1 = P.march(V, nsteps=21)
        I1, st2 = P.march_continue(V, I1, 21, nt - 21)
        out[graph, "split"] = (I1.cpu().numpy(), st1, st2)
        P.close()
    (Ie, se), (Ig, sg) = out[0], out[2]
    _say("step graph", "fp32" if prec else "fp64", "graph steps", sg["graph_steps"], "halts", sg["graph_halts"],
         "iterations", se["total_iters"], sg["total_iters"], "ms", se["ms_total"], sg["ms_total"])
    assert se["graph_steps"] == 0 and sg["graph_steps"] >= nt - 4 - sg["graph_halts"]
    assert sg["graph_halts"] >= 1                      # the pulse after the zero steps
    np.testing.assert_array_equal(Ig, Ie)
    assert list(sg["iters_per_step"]) == list(se["iters_per_step"])
    for k in ("total_iters", "max_iters", "steps_done", "residual_checks", "residual_worst_step",
              "max_residual64", "max_rel_residual", "unstable_step", "first_noconv_step"):
        assert sg[k] == se[k], k
    Is, s1, s2 = out[2, "split"]
    np.testing.assert_array_equal(Is, Ie)
    assert s2["graph_steps"] > 0
    assert list(s1["iters_per_step"][:21]) + list(s2["iters_per_step"][:nt - 21]) == list(se["iters_per_step"])
