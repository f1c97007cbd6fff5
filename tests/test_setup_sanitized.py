"""The library's host set-up (geometry, derived parameters, projection,
near zone, exact near entries, sparse approximate inverse; plus the
rejection of invalid meshes) built for the CPU with the address and
undefined-behaviour sanitizers and run on the level-2 sphere: it must end
cleanly (any sanitizer report aborts the run) and reproduce the near-zone
size and depth the oracle derives."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


_ENV = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
            UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    """The sanitized driver and the level-2 sphere's input file."""
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    tmp = tmp_path_factory.mktemp("setup")
    exe = tmp / "setup_san"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "native", "setup_driver.cpp"),
           os.path.join(ROOT, "paper_1408_7060_amd", "csrc", "setup.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    wl = W.SPHERE_L2
    xyz, tri, rwg = wl.mesh()
    d_near = wl.near_lambda * 299_792_458.0 / wl.f0
    mesh = tmp / "mesh.bin"
    with open(mesh, "wb") as f:
        np.array([len(xyz), len(tri), len(rwg)], dtype="<i4").tofile(f)
        np.ascontiguousarray(xyz, dtype="<f8").tofile(f)
        np.ascontiguousarray(tri, dtype="<i4").tofile(f)
        np.ascontiguousarray(rwg, dtype="<i4").tofile(f)
        np.array([wl.f0, wl.beta, wl.f_bw, d_near], dtype="<f8").tofile(f)
        np.array([wl.grid], dtype="<i4").tofile(f)
    return exe, mesh, tmp


def test_host_setup_under_asan_and_ubsan(driver):
    exe, mesh, tmp = driver
    wl = W.SPHERE_L2
    xyz, tri, rwg = wl.mesh()
    d_near = wl.near_lambda * 299_792_458.0 / wl.f0
    r = subprocess.run([str(exe), str(mesh)], capture_output=True, text=True, env=_ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    f = r.stdout.split()
    vals = dict(zip(f[0::2], f[1::2]))
    from oracle import aim, geometry, physics as ph
    s = geometry.Surface(xyz, tri, rwg)
    dt = ph.dt_from_beta(wl.beta, wl.f_bw)
    A = aim.AIM(s, wl.grid, d_near, dt, wl.f0, ph.ng_from(ph.rmax_of(xyz), dt))
    assert int(vals["ns"]) == s.ns and int(vals["nnz"]) == len(A.rows)
    assert int(vals["mn"]) == A.mn and int(vals["ng"]) == A.ng
    assert int(vals["rejected"]) == 4


def test_host_cfie_setup_matches_the_oracle(driver):
    """The CFIE's host set-up (alpha = 0.5), sanitized: the exact near-zone
    entries alpha Z^E + (1 - alpha) eta Z^H of every near pair and the
    MFIE's curl test projection equal the oracle's (rounding only)."""
    exe, mesh, tmp = driver
    out = tmp / "cfie.bin"
    r = subprocess.run([str(exe), str(mesh), "0.5", str(out)], capture_output=True, text=True, env=_ENV,
                       timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    from oracle import aim, geometry, mfie, physics as ph
    wl = W.SPHERE_L2
    xyz, tri, rwg = wl.mesh()
    s = geometry.Surface(xyz, tri, rwg)
    d_near = wl.near_lambda * 299_792_458.0 / wl.f0
    dt = ph.dt_from_beta(wl.beta, wl.f_bw)
    A = aim.AIM(s, wl.grid, d_near, dt, wl.f0, ph.ng_from(ph.rmax_of(xyz), dt), alpha=0.5)
    with open(out, "rb") as f:
        nnz, mn = np.fromfile(f, "<i4", 2)
        rowptr = np.fromfile(f, "<i4", s.ns + 1)
        col = np.fromfile(f, "<i4", nnz)
        near = np.fromfile(f, "<c16", nnz * (mn + 1)).reshape(nnz, mn + 1)
        lamH = np.fromfile(f, "<f8", s.ns * 256).reshape(s.ns, 4, 64)
    rows = np.repeat(np.arange(s.ns), np.diff(rowptr))
    assert mn == A.mn and np.array_equal(rows, A.rows) and np.array_equal(col, A.cols)
    assert np.abs(lamH[:, 3]).max() == 0.0
    assert np.abs(lamH[:, :3] - A.H).max() <= 1e-13 * np.abs(A.H).max()
    ref = mfie.cfie_pairs(s, A.rows, A.cols, list(range(mn + 1)), dt, wl.f0, 0.5)
    assert np.abs(near.T - ref).max() <= 1e-12 * np.abs(ref).max()


def test_host_blif_setup_matches_the_oracle(driver):
    """The BLIF basis (M = 3, extrapolation from 3 samples fitted at 6
    frequencies) in the host set-up, sanitized: the folded exact near-zone
    entries of every near pair equal the oracle's (the window series, the
    non-causal kernels, the least-squares extrapolation and the fold)."""
    exe, mesh, tmp = driver
    out = tmp / "blif.bin"
    r = subprocess.run([str(exe), str(mesh), "1.0", str(out), "blif"], capture_output=True, text=True, env=_ENV,
                       timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    from oracle import aim, blif, geometry, kernels, physics as ph, zfill
    wl = W.SPHERE_L2
    xyz, tri, rwg = wl.mesh()
    s = geometry.Surface(xyz, tri, rwg)
    d_near = wl.near_lambda * 299_792_458.0 / wl.f0
    dt = ph.dt_from_beta(wl.beta, wl.f_bw)
    b = blif.Blif(3, wl.f_bw * dt)
    a = blif.extrapolation(b.beta, 3, 3, 6)
    ng = int(np.floor(ph.rmax_of(xyz) / (ph.C0 * dt) + 3))
    A = aim.AIM(s, wl.grid, d_near, dt, wl.f0, ng, basis=b, fold_a=a)
    with open(out, "rb") as f:
        nnz, mn = np.fromfile(f, "<i4", 2)
        rowptr = np.fromfile(f, "<i4", s.ns + 1)
        col = np.fromfile(f, "<i4", nnz)
        near = np.fromfile(f, "<c16", nnz * (mn + 1)).reshape(nnz, mn + 1)
    assert mn == A.mn
    ref = A._exact(lambda rr, cc, ms: zfill.assemble_pairs(
        s, rr, cc, [kernels.EnvelopeKernel(m, dt, wl.f0, b) for m in ms]), A.rows, A.cols)
    assert np.abs(near.T - ref).max() <= 1e-12 * np.abs(ref).max()
