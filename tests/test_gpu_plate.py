"""The plate (Sec. 5.1; the EFIE, as the paper's plates) on the GPU against
the FP64 oracle, through the C ABI: a 1 m square PEC plate at 300 MHz
+-5 % (341 RWG on the interior edges of an open mesh) on a 16 x 16 x 8
grid, the plate in the z = 0 plane midway between two node planes.

* set-up: projection and pre-corrected near values;
* Z_m and the delayed field, FP64 <= 1e-12 and FP32 <= 1e-5, on the
  engines that take a grid with N_y != N_z (the LDS plane and the
  line-pass y/z engines, both x engines);
* the 80-step march against the oracle's LU march, <= 1e-10 of the peak
  current at every step; the march decays after the pulse (stable at
  this c dt)."""
import sys

import numpy as np
import pytest

import workloads as W
from gpu_cases import gpu_problem, oracle_aim, oracle_dense_aim, oracle_matvec, rel
from oracle import excitation, march

pytestmark = pytest.mark.gpu

WL = W.PLATE_1M
ENGINES = [(0, 0), (0, 1), (3, 0), (3, 1)]


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


def test_plate_setup_matches_oracle(torch):
    s, A, vals, p = oracle_aim(WL.name)
    P = gpu_problem(WL.name)
    assert (P.info["ng"], P.info["mn"], P.info["grid"]) == (p["ng"], A.mn, [16, 16, 8])
    lam = P.export("lambda")
    assert np.abs(lam - A.L).max() <= 1e-13 * np.abs(A.L).max()
    near = P.export("near")
    for m in range(A.mn + 1):
        assert np.abs(near[m] - vals[m]).max() <= 1e-12 * np.abs(vals[0]).max(), m
    P.close()


@pytest.mark.parametrize("engine", ENGINES, ids=[f"yz{a}_x{b}" for a, b in ENGINES])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)], ids=["fp64", "fp32"])
def test_plate_apply_z_and_delayed_field(torch, prec, tol, engine):
    _say("plate", prec, engine)
    s, A, vals, p = oracle_aim(WL.name)
    P = gpu_problem(WL.name, precision=prec)
    d = P.tuning()
    d["yz_engine"], d["x_engine"] = engine
    P.set_tuning(d)
    x = W.complex_normal(71, (1, s.ns))
    for m in (range(p["ng"] + 1) if prec == 0 else (0, 1)):
        y = P.apply_z(m, _dev(torch, x)).cpu().numpy()
        ref = oracle_matvec(WL.name, m, x, direct=False)
        assert rel(y, ref) <= tol, (m, rel(y, ref))
    hist = W.complex_normal(72, (p["ng"], 1, s.ns))
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()
    ref = sum(oracle_matvec(WL.name, m, hist[m - 1], direct=False) for m in range(1, p["ng"] + 1))
    assert rel(b, ref) <= tol, rel(b, ref)
    P.close()


def test_plate_march_matches_oracle(torch):
    nt = WL.nt
    s, A, vals, p = oracle_aim(WL.name)
    kh, pp = WL.incidence()
    V = excitation.excitation(s, nt, p["dt"], kh, pp, WL.sigma, WL.td, WL.f0)
    I_ref = march.march_dense(oracle_dense_aim(WL.name), V)
    P = gpu_problem(WL.name, tol=1e-13, nt=nt)
    I, st = P.march(_dev(torch, V))
    I = I.cpu().numpy()
    nrm = np.linalg.norm(I_ref[:, 0], axis=1)
    peak = nrm.max()
    _say("plate march iters", st["total_iters"], "rel", rel(I, I_ref), "last/peak", nrm[-1] / peak)
    for l in range(nt):
        assert np.linalg.norm(I[l] - I_ref[l]) <= 1e-10 * peak, l
    assert nrm[-1] < 1e-4 * peak and st["unstable_step"] == -1
    P.close()
