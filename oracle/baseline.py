"""Timed CPU baseline of the marching hot path (oracle; test infrastructure
only): the oracle's FFT march of eq. (5) (``march.march_fft``) on the host
cores, for one incidence direction of a workload, over as many steps as fit
a time budget.

Run as ``python -m oracle.baseline --workload NAME``; prints one JSON line.
It is meant to run in a process that has not touched a GPU: the exact
near-zone entries (the set-up, not timed) are computed by a pool of forked
workers.  Thread counts: the 3-D transforms use scipy.fft with one worker
per core of the process's CPU set (at most --max-cores), the BLAS the same.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import aim, excitation, geometry, kernels, march, physics as ph, zfill  # noqa: E402

_JOB = {}


def _near_chunk(bounds):
    """Pre-corrected near values of the pairs [a, b) (a pool worker)."""
    a, b = bounds
    A, s, dt, fc = _JOB["A"], _JOB["s"], _JOB["dt"], _JOB["fc"]
    r, c = A.rows[a:b], A.cols[a:b]
    ms = list(range(A.mn + 1))
    exact = zfill.assemble_pairs(s, r, c, [kernels.EnvelopeKernel(m, dt, fc) for m in ms])
    return exact - A.far_pairs(ms, r, c)


def near_values_parallel(A, s, dt: float, fc: float, workers: int) -> np.ndarray:
    """A.near_values for the exact entries of zfill, with the pairs split
    over a pool of forked workers (same values, concatenated in order)."""
    _JOB.update(A=A, s=s, dt=dt, fc=fc)
    nnz = len(A.rows)
    step = max(1, min(4096, math.ceil(nnz / (4 * workers))))
    chunks = [(a, min(a + step, nnz)) for a in range(0, nnz, step)]
    if workers <= 1:
        parts = [_near_chunk(ch) for ch in chunks]
    else:
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_near_chunk, chunks)
    return np.concatenate(parts, axis=1)


class _Budget(Exception):
    pass


def _host() -> dict:
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "ram_GiB": ram}


def main(argv=None):
    import scipy
    import workloads as W

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="sphere_L4_r1_600MHz_32dir")
    ap.add_argument("--budget", type=float, default=25.0, help="seconds of timed marching")
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--max-cores", type=int, default=16)
    args = ap.parse_args(argv)
    cores = max(1, min(len(os.sched_getaffinity(0)), args.max_cores))
    aim.FFT_WORKERS = cores
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(cores)
    except ImportError:
        pass
    wl = W.WORKLOADS[args.workload]
    t0 = time.perf_counter()
    xyz, tri, rwg = wl.mesh()
    s = geometry.Surface(xyz, tri, rwg)
    rmax = ph.rmax_of(xyz)
    dt = ph.dt_from_ng(rmax, wl.ng) if wl.ng else ph.dt_from_beta(wl.beta, wl.f_bw)
    ng = wl.ng or ph.ng_from(rmax, dt)
    A = aim.AIM(s, wl.grid, wl.near_lambda * ph.C0 / wl.f0, dt, wl.f0, ng)
    vals = near_values_parallel(A, s, dt, wl.f0, cores)
    kh, pp = wl.incidence()
    nmax = 64
    V = excitation.excitation(s, nmax, dt, kh[:1], pp[:1], wl.sigma, wl.td, wl.f0)[:, 0]
    setup_s = time.perf_counter() - t0
    times, iters = [], []
    t_start = time.perf_counter()

    def on_step(l, its):
        times.append(time.perf_counter())
        iters.append(its)
        if times[-1] - t_start > args.budget:
            raise _Budget

    try:
        march.march_fft(A, vals, V, args.tol, restart=50, maxit=1000, nsteps=nmax, on_step=on_step)
    except _Budget:
        pass
    n = len(times)
    wall = times[-1] - t_start
    per_dir = n / wall
    out = {"value": per_dir / wl.batch, "unit": "time-steps/s", "cores": cores, "kind": "oracle",
           "direction_steps_per_s": per_dir, "steps": n, "seconds": wall,
           "gmres_iters_per_step": float(np.mean(iters)), "setup_s": setup_s,
           "sample": (f"oracle FFT march of eq. (5) (numpy/scipy FP64: k-space history sum, right-Jacobi "
                      f"GMRES tol {args.tol:g}, exact near-zone entries), direction 0 of {wl.name}, steps "
                      f"0..{n - 1} (history terms 0..{min(n - 1, ng)} of N_g = {ng}), {wall:.1f} s; the "
                      f"{wl.batch}-direction job priced as {wl.batch} such marches"),
           **_host(), "numpy": np.__version__, "scipy": scipy.__version__}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
