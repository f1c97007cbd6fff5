"""The late-time growth detector of the march (flags, and with
ETAIM_F_FAIL_ON_UNSTABLE stops on, monotone growth of the current by more
than 10x over 32 steps that begin more than N_g steps after the
excitation's peak).  CPPIF envelope marching at +-20 % on the
level-2 sphere is unstable (companion spectral radius 1.41, Sec. 3.1.1):
its late-time growth is flagged.  The same march stopped while the pulse
still rises (the current grows with it) is not, nor is the stable
narrow-band march."""
import sys

import pytest

import workloads as W
from gpu_cases import gpu_problem

pytestmark = pytest.mark.gpu

F_CONTINUE_ON_NOCONV, F_FAIL_ON_UNSTABLE = 1, 2


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _march(wl, nt, td_steps=None, flags=F_CONTINUE_ON_NOCONV):
    P = gpu_problem(wl.name, precision=0, nt=nt, tol=1e-10, flags=flags)
    kh, pp = wl.incidence()
    td = wl.td if td_steps is None else td_steps * P.info["dt"]
    V = P.excitation(kh, pp, wl.sigma, td)
    try:
        I, st = P.march(V)
    finally:
        peak = td / P.info["dt"]
        P.close()
    return st, peak


def test_late_time_growth_is_flagged(torch):
    st, peak = _march(W.SPHERE_L2, 120)
    _say("L2 +-20 %: unstable_step", st["unstable_step"], "pulse peak at step", round(peak))
    assert st["unstable_step"] >= peak + 32 + 4     # N_g = 4 at level 2
    from paper_1408_7060_amd import EtaimError
    with pytest.raises(EtaimError) as ei:
        _march(W.SPHERE_L2, 120, flags=F_CONTINUE_ON_NOCONV | F_FAIL_ON_UNSTABLE)
    assert ei.value.code == -6


def test_growth_with_a_rising_pulse_is_not_flagged(torch):
    st, peak = _march(W.SPHERE_L2, 50, td_steps=60)
    _say("L2 +-20 %, pulse peak after the march: unstable_step", st["unstable_step"])
    assert st["unstable_step"] == -1


def test_stable_march_is_not_flagged(torch):
    st, _ = _march(W.SPHERE_L2_NARROW, 60)
    assert st["unstable_step"] == -1


def test_growth_under_a_decaying_pulse_is_flagged(torch):
    """The 250 MHz composite grows by about 1.27 per step from the start
    (CPPIF at +-5 %, Sec. 3.1.1); with the pulse peaking at step 10 the
    growth is flagged once 32 steps past the peak plus N_g (32) show it,
    while the excitation is still within a few e-folds of its peak."""
    st, peak = _march(W.COMPOSITE_SMALL, 110, td_steps=10)
    _say("composite 250 MHz: unstable_step", st["unstable_step"], "pulse peak at step", round(peak))
    assert peak + 32 + 32 <= st["unstable_step"] < 110
