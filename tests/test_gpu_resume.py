"""Checkpoint/resume of the forward march, through the C ABI: a march split
at step k and continued (on the same context, or after its state was saved
to host memory and loaded into a fresh context of the same problem) gives
the same currents as the uninterrupted march, bit for bit.  The split falls
inside a time block of the delayed field, so the continued march rebuilds
the block sums from the ring."""
import sys

import numpy as np
import pytest

import workloads as W
from gpu_cases import gpu_problem, oracle_aim
from oracle import excitation

pytestmark = pytest.mark.gpu

F_CONTINUE_ON_NOCONV = 1
L2 = W.SPHERE_L2.name


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _excitation(nt, nb, seed):
    wl = W.SPHERE_L2
    s, A, vals, p = oracle_aim(L2)
    kh = W.unit_vectors(seed, 2, nb)  # stream 2: directions
    pp = W.polarisations(seed, kh)
    return excitation.excitation(s, nt, p["dt"], kh, pp, wl.sigma, wl.td, wl.f0)


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-6)], ids=["fp64", "fp32"])
@pytest.mark.parametrize("split", [5, 8])
def test_resume_equals_uninterrupted(torch, prec, tol, split):
    nt = 16
    V = _excitation(nt, 2, 51)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    kw = dict(precision=prec, tol=tol, nt=nt, batch=2, flags=F_CONTINUE_ON_NOCONV, sync_every=4)
    P = gpu_problem(L2, **kw)
    I_full, _ = P.march(Vd)
    I_full = I_full.cpu().numpy()
    # the same context, interrupted at `split`
    I1, st1 = P.march(Vd, nsteps=split)
    state = P.save_state()
    I1, st2 = P.march_continue(Vd, I1, split, nt - split)
    assert st2["steps_done"] == nt - split and len(st2["iters_per_step"]) == nt - split
    _say("resume", "fp32" if prec else "fp64", "split", split, "same context max|d|",
         float(np.abs(I1.cpu().numpy() - I_full).max()))
    np.testing.assert_array_equal(I1.cpu().numpy(), I_full)
    # the history is now at step nt: continuing at another step is refused
    with pytest.raises(Exception) as ei:
        P.march_continue(Vd, I1, split, 1)
    assert ei.value.code == -1
    P.close()
    # a fresh context of the same problem, from the saved state
    Q = gpu_problem(L2, **kw)
    I2 = torch.zeros_like(Vd)
    I2[:split] = torch.from_numpy(np.ascontiguousarray(I_full[:split])).cuda()
    with pytest.raises(Exception) as ei:       # no history yet
        Q.march_continue(Vd, I2, split, nt - split)
    assert ei.value.code == -1
    Q.load_state(state)
    I2, _ = Q.march_continue(Vd, I2, split, nt - split)
    _say("  loaded context max|d|", float(np.abs(I2.cpu().numpy() - I_full).max()))
    np.testing.assert_array_equal(I2.cpu().numpy(), I_full)
    Q.close()


def test_state_of_another_problem_is_refused(torch):
    V = _excitation(8, 1, 52)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    P = gpu_problem(L2, precision=0, nt=8, batch=1, flags=F_CONTINUE_ON_NOCONV)
    with pytest.raises(Exception) as ei:       # nothing marched yet
        P.save_state()
    assert ei.value.code == -1
    P.march(Vd, nsteps=4)
    state = P.save_state()
    P.close()
    Q = gpu_problem(L2, precision=1, nt=8, batch=1, flags=F_CONTINUE_ON_NOCONV)
    with pytest.raises(Exception) as ei:       # FP32 rings: another size
        Q.load_state(state)
    assert ei.value.code == -1
    bad = state.copy()
    bad[:8] = 0
    R = gpu_problem(L2, precision=0, nt=8, batch=1, flags=F_CONTINUE_ON_NOCONV)
    with pytest.raises(Exception) as ei:       # not a state
        R.load_state(bad)
    assert ei.value.code == -1
    Q.close()
    R.close()


def test_engine_switch_invalidates_the_history(torch):
    """The LDS and register y/z engines lay the spectrum ring out
    differently: after a switch between them the history of the last march
    is not resumable (continue and save are refused), while a switch of the
    x stage only (same ring layout) keeps it."""
    nt = 10
    V = _excitation(nt, 1, 53)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    P = gpu_problem(L2, precision=0, nt=nt, batch=1, flags=F_CONTINUE_ON_NOCONV)
    t0 = P.tuning()
    assert t0["yz_engine"] != 0
    I, _ = P.march(Vd, nsteps=4)
    P.set_tuning(dict(t0, x_engine=1 - t0["x_engine"]))      # same ring layout
    I, _ = P.march_continue(Vd, I, 4, 2)
    P.set_tuning(dict(t0, yz_engine=0))
    for call in (lambda: P.march_continue(Vd, I, 6, 2), P.save_state):
        with pytest.raises(Exception) as ei:
            call()
        assert ei.value.code == -1
    P.close()


def test_state_with_a_corrupt_guess_order_is_refused(torch):
    """The carried initial-guess orders index a 6 x 6 coefficient table; a
    state whose orders lie outside 1..6 is refused before it is loaded."""
    V = _excitation(8, 1, 54)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    P = gpu_problem(L2, precision=0, nt=8, batch=1, flags=F_CONTINUE_ON_NOCONV)
    P.march(Vd, nsteps=5)
    state = P.save_state()
    # magic (8 bytes = int32 slots 0, 1), then version, prec, B, ns, ng, mn,
    # next_step, guess_p (slot 9), guess_dev, pnext (slot 11)
    hdr = state[:48].view(np.int32)
    for field, value in ((9, 7), (9, -1), (11, 0), (11, 7)):
        bad = state.copy()
        bad[:48].view(np.int32)[field] = value
        assert hdr[field] != value
        with pytest.raises(Exception) as ei:
            P.load_state(bad)
        assert ei.value.code == -1
    P.load_state(state)
    P.close()


def test_state_of_another_ring_layout_is_refused(torch):
    """A state saved with the register plane engine (ring slots by parity
    quadrants) loads into a context with the other register engine, not
    into one with the line-pass engine (plain slots); saved with the
    line-pass engine, it loads there and continues the march bit for bit."""
    nt = 10
    V = _excitation(nt, 1, 55)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    kw = dict(precision=0, nt=nt, batch=1, flags=F_CONTINUE_ON_NOCONV)
    P = gpu_problem(L2, **kw)
    t0 = P.tuning()
    assert t0["yz_engine"] == 2
    I, _ = P.march(Vd, nsteps=4)
    state = P.save_state()
    P.close()
    for yz, ok in ((1, True), (3, False), (0, False)):
        Q = gpu_problem(L2, **kw)
        Q.set_tuning(dict(Q.tuning(), yz_engine=yz))
        if ok:
            Q.load_state(state)
        else:
            with pytest.raises(Exception) as ei:
                Q.load_state(state)
            assert ei.value.code == -1
        Q.close()
    R = gpu_problem(L2, **kw)
    R.set_tuning(dict(R.tuning(), yz_engine=3))
    I_full, _ = R.march(Vd)
    I3, _ = R.march(Vd, nsteps=4)
    s3 = R.save_state()
    R.close()
    S = gpu_problem(L2, **kw)
    S.set_tuning(dict(S.tuning(), yz_engine=3))
    S.load_state(s3)
    I3, _ = S.march_continue(Vd, I3, 4, nt - 4)
    np.testing.assert_array_equal(I3.cpu().numpy(), I_full.cpu().numpy())
    S.close()
