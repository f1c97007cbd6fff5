"""The no-allocation excitation entry point against the allocating one,
through the C ABI: the same kernel on the same directions, so the vectors
agree bit for bit; two calls in a row on contexts of different batch (the
second smaller, so stale staging beyond its directions must not be read),
and the limit is enforced with a clear error."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W
from gpu_cases import gpu_problem

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


def _noalloc(P, kh, ph, sigma, td, V):
    from paper_1408_7060_amd import _lib
    lib = _lib.load()
    kh = np.ascontiguousarray(kh, dtype=np.float64)
    ph = np.ascontiguousarray(ph, dtype=np.float64)
    rc = lib.etaim_excitation_planewave_noalloc(P._h, len(kh), kh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), sigma, td,
                                                ctypes.c_void_p(V.data_ptr()))
    return rc, lib.etaim_last_error().decode()


def test_noalloc_excitation_equals_allocating_entry_point(torch):
    wl = W.SPHERE_L2
    dirs = W.unit_vectors(11, 2, 5)
    pols = W.polarisations(11, dirs)
    for batch, prec in ((5, 0), (2, 1)):
        _say("no-alloc excitation: batch", batch, "precision", prec)
        P = gpu_problem(wl.name, precision=prec, batch=batch, nt=12)
        kh, ph = dirs[:batch], pols[:batch]
        ref = P.excitation(kh, ph, wl.sigma, wl.td)
        V = torch.full_like(ref, float("nan"))
        rc, msg = _noalloc(P, kh, ph, wl.sigma, wl.td, V)
        assert rc == 0, msg
        torch.cuda.synchronize()
        assert torch.equal(V, ref)
        # the same staging reused with other directions (a reversed order)
        ref2 = P.excitation(kh[::-1].copy(), ph[::-1].copy(), wl.sigma, wl.td)
        rc, msg = _noalloc(P, kh[::-1], ph[::-1], wl.sigma, wl.td, V)
        assert rc == 0, msg
        assert torch.equal(V, ref2)
        # limits: more directions than the staging holds, and nb != batch
        big = np.tile(kh[:1], (4097, 1))
        rc, msg = _noalloc(P, big, big, wl.sigma, wl.td, V)
        assert rc == -1 and "4096" in msg, msg
        rc, msg = _noalloc(P, kh[:batch - 1], ph[:batch - 1], wl.sigma, wl.td, V)
        assert rc == -1, msg
        assert torch.equal(V, ref2)
        P.close()
