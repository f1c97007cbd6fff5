"""The y/z plane engines (LDS-staged radix passes over the padded plane,
register-resident parity quadrants, the same with the matvec plane
transform taking the z lines first, and separate y- and z-line passes over
a full-spectrum work array) against the FP64 oracle, through the C ABI.

At the level-4 sphere (48^3 grid, the size the bench marches) the oracle's
exact near-zone entries take minutes to assemble on the host, so the
operator is checked where the near zone is empty: Z_m for m > M_n is the
pure FFT (far) operator, and the delayed field of a history whose first M_n
samples are zero only sees those Z_m."""
import functools
import sys

import numpy as np
import pytest

import workloads as W
from gpu_cases import gpu_problem, oracle_aim, oracle_matvec, params_of, rel
from oracle import aim, geometry, physics as ph

pytestmark = pytest.mark.gpu

L2 = W.SPHERE_L2.name
L3 = W.SPHERE_L3.name
L4 = W.SPHERE_L4.name


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


@functools.lru_cache(maxsize=None)
def _oracle_far(name):
    wl = W.WORKLOADS[name]
    p = params_of(wl)
    s = geometry.Surface(p["xyz"], p["tri"], p["rwg"])
    return s, aim.AIM(s, wl.grid, p["d_near"], p["dt"], wl.f0, p["ng"]), p


def _with_engine(P, engine):
    """engine = (yz_engine, x_engine), or one value for both stages."""
    yz, xe = engine if isinstance(engine, tuple) else (engine, engine)
    d = P.tuning()
    d["yz_engine"], d["x_engine"] = yz, xe
    P.set_tuning(d)
    t = P.tuning()
    assert (t["yz_engine"], t["x_engine"]) == (yz, xe)


ENGINES = [(0, 0), (1, 1), (1, 0), (0, 1), (2, 1), (2, 0), (3, 0), (3, 1)]


@pytest.mark.parametrize("engine", ENGINES, ids=[f"yz{a}_x{b}" for a, b in ENGINES])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)], ids=["fp64", "fp32"])
def test_far_operator_level4(torch, prec, tol, engine):
    s, A, p = _oracle_far(L4)
    assert A.mn < p["ng"]
    P = gpu_problem(L4, precision=prec, batch=2, nt=8)
    assert P.info["mn"] == A.mn
    _with_engine(P, engine)
    x = W.complex_normal(31, (2, s.ns))
    for m in (A.mn + 1, (A.mn + p["ng"]) // 2, p["ng"]):
        y = P.apply_z(m, _dev(torch, x)).cpu().numpy()
        ref = np.array([A.far_matvec(m, xb) for xb in x])
        e = rel(y, ref)
        _say("L4 far", "fp32" if prec else "fp64", "engine", engine, "m", m, "rel", e)
        assert e <= tol, (m, e)
    P.close()


@pytest.mark.parametrize("engine,batch", [(0, 1), (1, 1), (1, 2), ((2, 1), 1), ((2, 1), 2)],
                         ids=["lds", "reg", "reg_pairs", "zlines", "zlines_b2"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)], ids=["fp64", "fp32"])
def test_delayed_field_level4(torch, prec, tol, engine, batch):
    """batch 2 runs the plane-pair delayed kernel in FP32 (two planes share
    each Green load); FP64 keeps one plane per block at this size."""
    s, A, p = _oracle_far(L4)
    ng = p["ng"]
    P = gpu_problem(L4, precision=prec, batch=batch, nt=8)
    _with_engine(P, engine)
    hist = W.complex_normal(32, (ng, batch, s.ns))
    hist[:A.mn] = 0.0
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()
    ref = np.array([sum(A.far_matvec(m, hist[m - 1, j]) for m in range(A.mn + 1, ng + 1)) for j in range(batch)])
    e = rel(b, ref)
    _say("L4 delayed", "fp32" if prec else "fp64", "engine", engine, "rel", e)
    assert e <= tol
    P.close()


@functools.lru_cache(maxsize=None)
def _oracle_far_grid(name, grid):
    wl = W.WORKLOADS[name]
    p = params_of(wl)
    s = geometry.Surface(p["xyz"], p["tri"], p["rwg"])
    return s, aim.AIM(s, grid, p["d_near"], p["dt"], wl.f0, p["ng"]), p


@pytest.mark.parametrize("engine", [(2, 1), (2, 0), (1, 1)], ids=["zlines", "zlines_xlds", "reg"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)], ids=["fp64", "fp32"])
def test_register_planes_grid24(torch, prec, tol, engine):
    """The register plane kernels at N = 24 (96-thread blocks: the matvec
    and commit kernels' second wave holds only odd-parity tasks): the level-3
    sphere on a 24^3 grid, far operator Z_m for m > M_n and the delayed field
    of a history whose first M_n samples are zero (commit + delayed sum),
    against the oracle."""
    s, A, p = _oracle_far_grid(L3, 24)
    ng = p["ng"]
    assert A.mn < ng
    P = gpu_problem(L3, precision=prec, batch=2, nt=8, grid=24)
    assert P.info["mn"] == A.mn
    _with_engine(P, engine)
    x = W.complex_normal(33, (2, s.ns))
    for m in range(A.mn + 1, ng + 1):
        y = P.apply_z(m, _dev(torch, x)).cpu().numpy()
        ref = np.array([A.far_matvec(m, xb) for xb in x])
        e = rel(y, ref)
        _say("grid24 far", "fp32" if prec else "fp64", "engine", engine, "m", m, "rel", e)
        assert e <= tol, (m, e)
    hist = W.complex_normal(34, (ng, 2, s.ns))
    hist[:A.mn] = 0.0
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()
    ref = np.array([sum(A.far_matvec(m, hist[m - 1, j]) for m in range(A.mn + 1, ng + 1)) for j in range(2)])
    e = rel(b, ref)
    _say("grid24 delayed", "fp32" if prec else "fp64", "engine", engine, "rel", e)
    assert e <= tol
    P.close()


@functools.lru_cache(maxsize=None)
def _delayed_ref_level4(batch):
    s, A, p = _oracle_far(L4)
    ng = p["ng"]
    hist = W.complex_normal(36, (ng, batch, s.ns))
    hist[:A.mn] = 0.0
    ref = np.array([sum(A.far_matvec(m, hist[m - 1, j]) for m in range(A.mn + 1, ng + 1)) for j in range(batch)])
    return hist, ref


@pytest.mark.parametrize("block", [1, 3, 5, 8])
@pytest.mark.parametrize("engine", [1, (2, 1), (3, 1)], ids=["reg", "zlines", "lines"])
@pytest.mark.parametrize("prec,tol,batch", [(0, 1e-12, 1), (1, 1e-5, 2)], ids=["fp64", "fp32_b2"])
def test_delayed_time_blocks_level4(torch, prec, tol, batch, engine, block):
    """The register and line-pass engines sum, in time blocks of that many steps, the
    history older than a block once at its first step and the block's own
    steps at every step; the delayed field at step N_g then stands at block
    position (N_g - 1) mod block (7 of 8 at block 8: seven own steps, the
    rest from the block pass), which the oracle's direct sum checks."""
    s, A, p = _oracle_far(L4)
    hist, ref = _delayed_ref_level4(batch)
    P = gpu_problem(L4, precision=prec, batch=batch, nt=8)
    _with_engine(P, engine)
    d = P.tuning()
    d["delay_block"] = block
    P.set_tuning(d)
    assert P.tuning()["delay_block"] == block
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()
    e = rel(b, ref)
    _say("L4 delayed blocks", block, "engine", engine, "fp32" if prec else "fp64", "rel", e)
    assert e <= tol
    P.close()


@pytest.mark.parametrize("engine", [(2, 1), (3, 1)], ids=["zlines", "lines"])
def test_time_blocks_give_the_same_march(torch, engine):
    """Marches with the history sum in time blocks of 2 and 3 steps (N_g = 4
    at level 2) against the direct sum at every step."""
    wl = W.SPHERE_L2
    s, A, vals, p = oracle_aim(L2)
    assert p["ng"] == 4
    from oracle import excitation
    kh = W.unit_vectors(37, 2, 3)
    pp = W.polarisations(37, kh)
    V = excitation.excitation(s, 24, p["dt"], kh, pp, wl.sigma, wl.td, wl.f0)
    out = []
    for block in (1, 2, 3):
        P = gpu_problem(L2, nt=24, batch=2, tol=1e-13)
        _with_engine(P, engine)
        d = P.tuning()
        d["delay_block"] = block
        P.set_tuning(d)
        I, _ = P.march(_dev(torch, V))
        out.append(I.cpu().numpy())
        P.close()
    for o in out[1:]:
        _say("L2 march blocks rel", rel(o, out[0]))
        assert rel(o, out[0]) <= 1e-11


@pytest.mark.parametrize("engine", ENGINES, ids=[f"yz{a}_x{b}" for a, b in ENGINES])
def test_engines_full_operator_level2(torch, engine):
    """Every Z_m (near + far) and the delayed field at the 16^3 grid."""
    s, A, vals, p = oracle_aim(L2)
    P = gpu_problem(L2)
    _with_engine(P, engine)
    x = W.complex_normal(33, (2, s.ns))
    for m in range(p["ng"] + 1):
        y = P.apply_z(m, _dev(torch, x[:1])).cpu().numpy()
        ref = oracle_matvec(L2, m, x[:1], direct=True)
        assert rel(y, ref) <= 1e-12, (m, rel(y, ref))
    hist = W.complex_normal(34, (p["ng"], 1, s.ns))
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()
    ref = sum(oracle_matvec(L2, m, hist[m - 1], direct=True) for m in range(1, p["ng"] + 1))
    assert rel(b, ref) <= 1e-12
    P.close()


def test_engines_give_the_same_march(torch):
    wl = W.SPHERE_L2
    s, A, vals, p = oracle_aim(L2)
    from oracle import excitation
    kh = W.unit_vectors(35, 2, 3)
    pp = W.polarisations(35, kh)
    V = excitation.excitation(s, 16, p["dt"], kh, pp, wl.sigma, wl.td, wl.f0)
    out = []
    for engine in ENGINES:
        P = gpu_problem(L2, nt=16, batch=2, tol=1e-13)
        _with_engine(P, engine)
        I, _ = P.march(_dev(torch, V))
        out.append(I.cpu().numpy())
        P.close()
    for o in out[1:]:
        assert rel(o, out[0]) <= 1e-11


@pytest.mark.parametrize("batch", [1, 3])
def test_interp_tiles_full_operator_level2(torch, batch):
    """The grid-tile interpolation engine (a block per tile and column group,
    the tile's potentials staged in LDS): every Z_m (near + far) and the
    delayed field at the 16^3 grid against the oracle, FP64; batch 3 leaves
    the last column group partial."""
    s, A, vals, p = oracle_aim(L2)
    P = gpu_problem(L2, batch=batch)
    d = P.tuning()
    d["interp_engine"] = 1
    P.set_tuning(d)
    assert P.tuning()["interp_engine"] == 1
    x = W.complex_normal(38, (batch, s.ns))
    for m in range(p["ng"] + 1):
        y = P.apply_z(m, _dev(torch, x)).cpu().numpy()
        ref = oracle_matvec(L2, m, x, direct=True)
        assert rel(y, ref) <= 1e-12, (m, rel(y, ref))
    hist = W.complex_normal(39, (p["ng"], batch, s.ns))
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()
    ref = np.array([sum(oracle_matvec(L2, m, hist[m - 1, j:j + 1], direct=True)[0] for m in range(1, p["ng"] + 1))
                    for j in range(batch)])
    e = rel(b, ref)
    _say("L2 tiles batch", batch, "delayed rel", e)
    assert e <= 1e-12
    P.close()


@pytest.mark.parametrize("prec,grid,tol,xe", [(0, 54, 1e-12, None), (1, 72, 1e-5, None), (0, 72, 1e-12, None),
                                              (1, 72, 1e-5, 0)],
                         ids=["fp64_54", "fp32_72", "fp64_72", "fp32_72_xlds"])
def test_line_engine_where_planes_do_not_fit(torch, prec, grid, tol, xe):
    """A padded (y, z) plane larger than the LDS (108^2 FP64 = 186 KB, 144^2
    FP32 = 166 KB) puts the y/z stage on the line-pass engine by itself: the
    level-3 sphere on that grid, far operator Z_m for m > M_n and the
    delayed field of a history whose first M_n samples are zero, against
    the oracle.  Line length 108 runs the LDS passes; 144 = 12 x 12 the
    four-step register lines, with the anterpolated grid transformed by
    them (the default x stage there) or the LDS gather (xlds)."""
    s, A, p = _oracle_far_grid(L3, grid)
    ng = p["ng"]
    assert A.mn < ng
    P = gpu_problem(L3, precision=prec, batch=2, nt=8, grid=grid)
    assert P.tuning()["yz_engine"] == 3 and P.info["mn"] == A.mn
    assert P.tuning()["x_engine"] == (0 if grid == 54 else 1)
    if xe is not None:
        P.set_tuning(dict(P.tuning(), x_engine=xe))
        assert P.tuning()["x_engine"] == xe
    x = W.complex_normal(40, (2, s.ns))
    for m in range(A.mn + 1, ng + 1):
        y = P.apply_z(m, _dev(torch, x)).cpu().numpy()
        ref = np.array([A.far_matvec(m, xb) for xb in x])
        e = rel(y, ref)
        _say("line engine", grid, "fp32" if prec else "fp64", "m", m, "rel", e)
        assert e <= tol, (m, e)
    hist = W.complex_normal(41, (ng, 2, s.ns))
    hist[:A.mn] = 0.0
    b = P.delayed_field(_dev(torch, hist)).cpu().numpy()
    ref = np.array([sum(A.far_matvec(m, hist[m - 1, j]) for m in range(A.mn + 1, ng + 1)) for j in range(2)])
    e = rel(b, ref)
    _say("line engine", grid, "delayed rel", e)
    assert e <= tol
    P.close()
