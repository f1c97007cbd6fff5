"""C-ABI checks that need no GPU: every declared entry point is exported,
and invalid inputs are rejected (EINVAL/EUNSUPPORTED) before device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "etaim.h")


def _lib():
    from paper_1408_7060_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1408_7060_amd import build
        build.build(verbose=False)
    return _lib


def test_every_declared_symbol_is_exported():
    L = _lib()
    lib = L.load()
    decl = set(re.findall(r"\b(etaim_[a-z_]+)\s*\(", open(HEADER).read()))
    assert decl, "no declarations found"
    assert decl == set(L.SIGNATURES), decl ^ set(L.SIGNATURES)
    for name in decl:
        assert hasattr(lib, name)


def _create(xyz, tri, rwg, **kw):
    L = _lib()
    lib = L.load()
    xyz = np.ascontiguousarray(xyz, np.float64)
    tri = np.ascontiguousarray(tri, np.int32)
    rwg = np.ascontiguousarray(rwg, np.int32)
    mesh = L.Mesh(len(xyz), xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(tri),
                  tri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    r = L.Rwg(len(rwg), rwg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    args = dict(fc=3e8, beta=0.2, f_bw=6e7, nt_steps=10, order=3, grid=(16, 16, 16), d_near=0.3, ng=0,
                precision=0, batch=1, tol=1e-6, restart=20, maxit=100, flags=0)
    args.update(kw)
    g = args.pop("grid")
    p = L.Params(grid=(ctypes.c_int32 * 3)(*g), **args)
    h = ctypes.c_void_p()
    rc = lib.etaim_create(ctypes.byref(h), ctypes.byref(mesh), ctypes.byref(r), ctypes.byref(p), None)
    return rc, lib.etaim_last_error().decode()


def _sphere():
    xyz, tri = W.icosphere(2, 0.5)
    return xyz, tri, W.rwg_table(tri)


def test_rejects_null_arguments():
    lib = _lib().load()
    h = ctypes.c_void_p()
    assert lib.etaim_create(ctypes.byref(h), None, None, None, None) == _lib().EINVAL
    assert lib.etaim_describe(None, None) == _lib().EINVAL
    assert lib.etaim_march(None, None, None, 0, None) == _lib().EINVAL
    t = _lib().Tuning()
    assert lib.etaim_autotune(None, 100, None, ctypes.byref(t)) == _lib().EINVAL
    assert lib.etaim_get_tuning(None, ctypes.byref(t)) == _lib().EINVAL
    assert lib.etaim_set_tuning(None, ctypes.byref(t)) == _lib().EINVAL
    assert lib.etaim_march_continue(None, None, None, 1, 1, None) == _lib().EINVAL
    n = ctypes.c_size_t(0)
    assert lib.etaim_state_size(None, ctypes.byref(n)) == _lib().EINVAL
    assert lib.etaim_state_save(None, None, 0) == _lib().EINVAL
    assert lib.etaim_state_load(None, None, 0) == _lib().EINVAL
    assert lib.etaim_set_profiling(None, 1) == _lib().EINVAL
    assert lib.etaim_set_profiling_mask(None, 1) == _lib().EINVAL
    lib.etaim_destroy(None)


@pytest.mark.parametrize("kw,code", [
    (dict(order=4), -7),                 # only CPPIF Q = 3
    (dict(grid=(10, 10, 10)), -7),       # padded length 20 has a factor 5
    (dict(grid=(6, 16, 16)), -1),        # grid too small
    (dict(grid=(8, 8, 8)), -1),          # stencils leave the 8^3 grid? (h = E/4 puts them inside) or pass
    (dict(fc=-1.0), -1),
    (dict(nt_steps=0), -1),
    (dict(tol=0.0), -1),
    (dict(restart=0), -1),
    (dict(beta=0.0), -1),                # dt and ng both derived needs beta
    (dict(sync_every=-1), -1),
    (dict(sync_every=61), -1),           # more Arnoldi steps per check than the restart length
])
def test_rejects_bad_parameters(kw, code):
    rc, msg = _create(*_sphere(), **kw)
    if kw == dict(grid=(8, 8, 8)):
        # an 8^3 grid is valid geometry-wise; creation then needs a GPU
        assert rc in (-1, -3), msg
        return
    assert rc == code, msg
    assert msg


def test_rejects_bad_mesh():
    xyz, tri, rwg = _sphere()
    bad = rwg.copy()
    bad[0, [0, 1]] = bad[0, [1, 0]]          # T+/T- swapped: orientation violated
    rc, msg = _create(xyz, tri, bad)
    assert rc == -1 and "orientation" in msg
    bad = rwg.copy()
    bad[3, 2] = len(xyz) + 5                 # vertex out of range
    assert _create(xyz, tri, bad)[0] == -1
    tri2 = tri.copy()
    tri2[0, 1] = tri2[0, 0]                  # degenerate triangle
    assert _create(xyz, tri2, rwg)[0] == -1
    xyz2 = xyz.copy()
    xyz2[0, 0] = np.nan
    assert _create(xyz2, tri, rwg)[0] == -1


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1408_7060_amd import _lib as L
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_LIB", None)
    with pytest.raises(ImportError):
        L.load()


def test_db_error_matches_the_oracle():
    """eq. (2) in the library (host code) against the oracle's, on random
    patterns spanning 100 dB, with values below the threshold on both sides."""
    from oracle import mie
    from paper_1408_7060_amd import db_error
    rng = np.random.default_rng(7)
    TH, PH, d, th = mie.sphere_grid(19, 36)
    ref = 10.0 ** rng.uniform(-10, 0, TH.shape)
    sig = ref * 10.0 ** rng.normal(0, 0.05, TH.shape)
    sig[3, 5] = 0.0
    for floor in (80.0, 30.0):
        e = db_error(sig, ref, np.sin(TH), floor)
        assert e == pytest.approx(mie.db_error(sig, ref, TH, floor), rel=1e-12)
    assert db_error(ref, ref, np.sin(TH)) == 0.0
    lib = _lib().load()
    assert lib.etaim_db_error(0, None, None, None, 80.0, None) == _lib().EINVAL
    assert lib.etaim_rcs(None, 1, None, 1, None, 1.0, None, None) == _lib().EINVAL

