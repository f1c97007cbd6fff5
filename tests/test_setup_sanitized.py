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


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_setup_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "setup_san"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "native", "setup_driver.cpp"),
           os.path.join(ROOT, "paper_1408_7060_amd", "csrc", "setup.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    wl = W.SPHERE_L2
    xyz, tri, rwg = wl.mesh()
    d_near = wl.near_lambda * 299_792_458.0 / wl.f0
    mesh = tmp_path / "mesh.bin"
    with open(mesh, "wb") as f:
        np.array([len(xyz), len(tri), len(rwg)], dtype="<i4").tofile(f)
        np.ascontiguousarray(xyz, dtype="<f8").tofile(f)
        np.ascontiguousarray(tri, dtype="<i4").tofile(f)
        np.ascontiguousarray(rwg, dtype="<i4").tofile(f)
        np.array([wl.f0, wl.beta, wl.f_bw, d_near], dtype="<f8").tofile(f)
        np.array([wl.grid], dtype="<i4").tofile(f)
    env = dict(os.environ, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), str(mesh)], capture_output=True, text=True, env=env, timeout=600)
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
