"""Benchmark of the ET-AIM marching hot path on one MI355X.

Workload (default): level-4 icosphere of radius 1 m (7680 RWG), 32 seeded
incidence directions with random polarisation, f0 = 600 MHz +-10 %,
48^3 grid padded to 96^3, N_g = 24, near zone 0.3 lambda, FP32 grid
arithmetic with FP64 GMRES (tol 1e-5), all 32 directions batched.

Before timing, the library's autotuner picks the FFT radix plans, launch
shapes and GMRES schedule for this problem (--tune-ms budget, untimed).

A "step" is one time step of the batched march: delayed field (k-space
temporal sum over the history + inverse FFT + interpolation + near history),
the GMRES solve (one AIM matvec per iteration) and the commit (anterpolation
+ forward FFT into the history ring).  The timed window is K = --steps steps
of the march, steps first .. first + K - 1, reached by marching the steps
before it untimed (at least --warmup of them): by default the window is
centred on the peak of the pulse (t_d / dt) and starts no earlier than
N_g + 8, so that every timed step sums all N_g history terms.  The timed
region is one etaim_march_continue call bracketed by
torch.cuda.synchronize(); it holds no ring reset.  Inputs (excitation) are
resident in HBM before timing.  The 40 (or K) steps just before the window
are marched with every kernel class traced, untimed, for the per-class
table; inside the timed region only the roofline kernel and the
delayed-field kernels are traced (their events ride on the dispatch).

Printed: one JSON line with the metric, the roofline record of the dominant
kernel class (algorithmic bytes or flops / device time, HIP events on the
library's stream over the timed region), the plain FP64 GPU path on the
first direction over the same window, the FP32-vs-FP64 error there, and the
CPU oracle baseline (the oracle's FFT march on the host cores, run as a
child process).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# published FP32 vector peak of the MI355X: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops (FMA) x 2 (packed FP32) x 2.4 GHz = 157.3 TFLOP/s
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2 * 2.4e9 / 1e12
# the rate without packed FP32 instructions, which the build disables: the
# issue ceiling of this code, reported beside the fraction of the peak
ALU_ISSUE_TFLOPS = ALU_PEAK_TFLOPS / 2
CSRC = os.path.join(ROOT, "paper_1408_7060_amd", "csrc")
FFT_CLASSES = ("anterp_x", "yz_green", "fft_x_inv", "interp_near", "yz_delayed", "yz_commit", "ring_far")
# traced inside the timed region: the roofline kernel and the delayed-field
# stream (single-kernel classes, whose HIP events ride on the dispatch itself)
TIMED_CLASSES = ("yz_green", "yz_delayed", "ring_far")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problem(wl, precision, batch, nt, tol, flags=1, sync_every=1, alpha=1.0, basis=0):
    import workloads as W  # noqa: F401
    from paper_1408_7060_amd import Problem
    xyz, tri, rwg = wl.mesh()
    d_near = wl.near_lambda * 299_792_458.0 / wl.f0
    kw = dict(fc=wl.f0, nt=nt, grid=wl.grid, d_near=d_near, precision=precision, batch=batch, tol=tol,
              restart=50, maxit=2000, flags=flags, sync_every=sync_every, alpha=alpha, basis=basis)
    if wl.ng:
        kw["ng"] = wl.ng
        kw["f_bw"] = wl.f_bw
    else:
        kw.update(beta=wl.beta, f_bw=wl.f_bw)
    return Problem(xyz, tri, rwg, **kw)


def cpu_baseline(wl, budget_s=25.0):
    """The oracle's FFT march of eq. (5) (numpy/scipy FP64, exact near-zone
    entries, right-Jacobi GMRES) on the host cores for one direction, run as
    a child process that never touches the GPU (its set-up forks a worker
    pool); returns its JSON record."""
    import subprocess
    cmd = [sys.executable, "-m", "oracle.baseline", "--workload", wl.name, "--budget", str(budget_s)]
    r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"cpu baseline failed ({r.returncode}): {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def step_err(a, b) -> float:
    """Largest per-step error ||a_l - b_l|| relative to the peak step norm of b."""
    nb = np.linalg.norm(b.reshape(len(b), -1), axis=1)
    return float(np.max(np.linalg.norm((a - b).reshape(len(b), -1), axis=1)) / max(nb.max(), 1e-300))


def stream_copy_gbps(torch, mib: int = 1024, reps: int = 5) -> float:
    """Device-to-device copy rate (read + write bytes / time) of a plain copy."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    rate = 2.0 * n * 4 * reps / (time.perf_counter() - t) / 1e9
    del src, dst
    return rate


def fft_flops(n: int) -> float:
    """Conventional flop count of an n-point complex FFT."""
    return 5.0 * n * math.log2(n)


def class_flops(cls: str, info: dict, batch: int):
    """Algorithmic flops of one launch of the y/z matvec stage split into
    parity halves (N_y = N_z = N, padded 2N): per (bc, kx) plane, 12 N
    transforms of N points (2N + 4N forward, 4N + 2N inverse: the zero half
    of the input and the discarded half of the output are pruned), the Green
    multiply (6 flops per point of the 4 N^2-point spectrum) and the parity
    twiddles (5 N^2 complex products, 3 N^2 additions).  Both register
    engines do this work (in the z-lines-first order the twiddles are N^2
    products more).  None for the other classes."""
    if cls != "yz_green":
        return None
    n = info["grid"][1]
    planes = 4 * batch * info["padded"][0]
    per_plane = (2 * n + 8 * n + 2 * n) * fft_flops(n) + 4 * n * n * 6 + 5 * n * n * 6 + 3 * n * n * 2
    return planes * per_plane


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()


def hbm_traffic(workload: str, kernel: str):
    """Measured HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE,
    calibrated on a plain copy), from profiles/hbm_traffic_<workload>.json;
    None if absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    k = rec.get("kernels", {}).get(kernel)
    if k is None or rec.get("source_sha256") != kernel_source_hash():
        return None
    return k["bytes_per_launch"]


def derived_dt(wl, xyz) -> float:
    """The time step the library derives for the workload: with N_g given,
    dt = R_max / (c (N_g - Q + 1/2)), R_max the largest vertex distance
    (a farthest pair lies on the convex hull); otherwise dt = beta / f_bw."""
    if not wl.ng:
        return wl.beta / wl.f_bw
    from scipy.spatial import ConvexHull
    h = xyz[ConvexHull(xyz).vertices]
    d = max(float(np.sqrt(((h[i:i + 256, None, :] - h[None, :, :]) ** 2).sum(-1)).max())
            for i in range(0, len(h), 256))
    return d / (299_792_458.0 * (wl.ng - 3 + 0.5))


def window(wl, dt: float, ng: int, K: int, warmup: int, first: int):
    """(first timed step, traced steps before it, pulse-peak step).  Default:
    centred on the pulse peak t_d / dt, no earlier than N_g + 8 plus the
    traced pass (every timed and traced step has N_g live history terms),
    and after at least `warmup` untimed steps."""
    peak = int(round(wl.td / dt))
    kt = min(K, 40)
    if first < 0:
        first = max(warmup, ng + 8 + kt, peak - K // 2)
    if first < kt + 1:
        raise SystemExit(f"--first must be at least {kt + 1}")
    return first, kt, peak


def roofline_record(dom, d, info, batch, traffic):
    avg_ms = d["ms"] / d["launches"]
    bytes_launch = d["bytes"] / d["launches"]
    hbm_gbs = bytes_launch / (avg_ms / 1e3) / 1e9
    flops = class_flops(dom, info, batch)
    if flops is not None and flops / (avg_ms / 1e3) / 1e12 / ALU_PEAK_TFLOPS > hbm_gbs / HBM_PEAK_GBS:
        # the FFT work, not the bytes, bounds this kernel: roofline against the FP32 vector issue rate
        achieved = flops / (avg_ms / 1e3) / 1e12
        return {"bound": "alu", "achieved": round(achieved, 2), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / ALU_PEAK_TFLOPS, 4), "traffic": traffic, "kernel": dom,
                "frac_of_unpacked_issue_rate": round(achieved / ALU_ISSUE_TFLOPS, 4), "flops_per_launch": flops, "bytes_per_launch": bytes_launch, "avg_launch_ms": avg_ms,
                "launches": d["launches"], "hbm_GBps": round(hbm_gbs, 1),
                "hbm_frac": round(hbm_gbs / HBM_PEAK_GBS, 4)}
    return {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(hbm_gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
            "bytes_per_launch": bytes_launch, "avg_launch_ms": avg_ms, "launches": d["launches"]}


def sweep(torch, W, FP64, alpha=1.0, basis=0, plates=False):
    """The ET-AIM size and bandwidth sweep of spheres, or of square plates
    (the trends of the paper's Figs. 2-3 without the comparison methods):
    every size at chi = 3 and 100, every chi at the smallest and a middle
    size; per
    point the whole march of one incidence along -z in FP64 (GMRES tol 1e-6,
    near-zone approximate inverse), its right-hand-side, solve and commit
    time per step, iterations per step, N_t, N_g and M_n."""
    from paper_1408_7060_amd._lib import F_CONTINUE_ON_NOCONV
    if plates:
        pts = [(size, g, chi) for (size, g) in W.PLATE_SWEEP_SIZES for chi in (3, 100)]
        pts += [(size, g, chi) for (size, g) in (W.PLATE_SWEEP_SIZES[0], W.PLATE_SWEEP_SIZES[2]) for chi in (10, 30)]
        mk = W.plate_sweep_workload
    else:
        pts = [(L, a, g, chi) for (L, a, g) in W.SWEEP_SIZES for chi in (3, 100)]
        pts += [(L, a, g, chi) for (L, a, g) in (W.SWEEP_SIZES[0], W.SWEEP_SIZES[2]) for chi in (10, 30)]
        mk = W.sweep_workload
    torch.cuda.set_device(0)
    for pt in pts:
        chi = pt[-1]
        wl = mk(*pt)
        g = wl.grid
        t = time.perf_counter()
        P = make_problem(wl, FP64, 1, wl.nt, 1e-6, flags=F_CONTINUE_ON_NOCONV, alpha=alpha, basis=basis)
        setup_s = time.perf_counter() - t
        kh, pp = wl.incidence()
        V = P.excitation(kh, pp, wl.sigma, wl.td)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = P.march(V)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        nt = st["steps_done"]
        rec = {"point": wl.name, "formulation": "EFIE" if alpha == 1.0 else f"CFIE alpha={alpha}",
               "basis": "BLIF M=3" if basis else "CPPIF Q=3",
               "ns": P.ns, "chi": chi, "f_c_MHz": round(wl.f0 / 1e6, 1),
               "f_bw_MHz": round(wl.f_bw / 1e6, 2), "grid": g, "ng": P.info["ng"], "mn": P.info["mn"],
               "nnz": P.info["nnz"], "nt": nt, "gmres_iters_per_step": round(st["total_iters"] / max(nt, 1), 2),
               "ms_rhs_per_step": round(st["ms_rhs"] / max(nt, 1), 3),
               "ms_solve_per_step": round(st["ms_solve"] / max(nt, 1), 3),
               "ms_commit_per_step": round(st["ms_commit"] / max(nt, 1), 3),
               "march_s": round(wall, 3), "setup_s": round(setup_s, 2),
               "unstable_step": st["unstable_step"] if st["unstable_step"] >= 0 else None,
               "first_noconv_step": st["first_noconv_step"] if st["first_noconv_step"] >= 0 else None}
        P.close()
        del V
        torch.cuda.empty_cache()
        print(json.dumps(rec), flush=True)


def delay_point(torch, W, FP32, ng, K=96):
    """The delayed field of the 32-direction level-4 sphere (FP32, B = 32,
    z-lines-first plane kernels, register x lines) with the time step shrunk
    so that the history holds ng steps, marched with delay mode 0 (the
    k-space temporal sum: in time blocks of 7 steps where N_g <= 32, else
    over all N_g stored spectra at every step) and mode 1 (multilevel time
    blocks).  K steps are timed after N_g + 104 untimed ones (every level has
    passed at least twice; K = 96 is two passes of the 48-step level); per
    mode the right-hand-side (delayed field) time per step from the march's
    phase events, the HBM bytes per step and rate of the delayed-field
    kernels (the per-step sum and the time-block or level passes) from their
    traced launches, GMRES iterations and the whole step.  Returns the two
    records."""
    import dataclasses
    from paper_1408_7060_amd._lib import F_CONTINUE_ON_NOCONV, F_IMPLICIT_STOP
    base = W.SPHERE_L4_BATCH
    wl = dataclasses.replace(base, name=f"{base.name}_ng{ng}", ng=ng)
    first = ng + 104
    nt = first + K
    t = time.perf_counter()
    P = make_problem(wl, FP32, wl.batch, nt, 1e-5, flags=F_CONTINUE_ON_NOCONV | F_IMPLICIT_STOP, sync_every=4)
    setup_s = time.perf_counter() - t
    kh, pp = wl.incidence()
    V = P.excitation(kh, pp, wl.sigma, wl.td)
    recs = []
    for mode in (0, 1):
        d = P.tuning()
        d.update(yz_engine=2, x_engine=1, delay_block=7)
        P.set_tuning(d)
        P.set_delay_mode(mode)
        P.set_profiling(False)
        I, _ = P.march(V, nsteps=first)
        P.set_profiling(True, classes=["yz_delayed", "ring_far"])
        torch.cuda.synchronize()
        t = time.perf_counter()
        I, st = P.march_continue(V, I, first, K)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        ks = P.kernel_stats()
        P.set_profiling(False)
        dms = sum(ks[c]["ms"] for c in ("yz_delayed", "ring_far"))
        dby = sum(ks[c]["bytes"] for c in ("yz_delayed", "ring_far"))
        recs.append({"point": wl.name, "ng": P.info["ng"], "mn": P.info["mn"], "batch": wl.batch,
                     "delay_mode": mode,
                     "delay": ("multilevel time blocks" if mode else
                               ("time blocks of 7" if ng <= 32 else "direct sum over N_g")),
                     "window": [first, nt - 1], "ms_per_step": round(1e3 * wall / K, 3),
                     "time_steps_per_s": round(K / wall, 2),
                     "ms_rhs_per_step": round(st["ms_rhs"] / K, 3),
                     "delayed_kernels_ms_per_step": round(dms / K, 3),
                     "delayed_GB_per_step": round(dby / K / 1e9, 2),
                     "delayed_GBps": round(dby / (dms / 1e3) / 1e9, 1) if dms > 0 else None,
                     "gmres_iters_per_step": round(st["total_iters"] / K, 2), "setup_s": round(setup_s, 1)})
        del I
    P.close()
    del V
    torch.cuda.empty_cache()
    return recs


def plate_history(torch, W, FP64, sizes=((16.0, 192),), chi=3.0):
    """The plate sweep's recipe beyond its largest size: a 16 m plate at
    chi = 3 (N_g above the one-level time blocks' 32), its whole march in
    FP64 (the default engines) with the delayed field as the direct sum
    (delay mode 0) and with multilevel time blocks (mode 1); per mode the
    right-hand-side, solve and march time, iterations, N_g and N_t."""
    from paper_1408_7060_amd._lib import F_CONTINUE_ON_NOCONV
    torch.cuda.set_device(0)
    for size, g in sizes:
        wl = W.plate_sweep_workload(size, g, chi)
        t = time.perf_counter()
        P = make_problem(wl, FP64, 1, wl.nt, 1e-6, flags=F_CONTINUE_ON_NOCONV)
        setup_s = time.perf_counter() - t
        kh, pp = wl.incidence()
        V = P.excitation(kh, pp, wl.sigma, wl.td)
        out = {}
        for mode in (0, 1):
            P.set_delay_mode(mode)
            torch.cuda.synchronize()
            t = time.perf_counter()
            I, st = P.march(V)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t
            out[mode] = I.cpu().numpy()
            nt = st["steps_done"]
            print(json.dumps({"point": wl.name, "ns": P.ns, "chi": chi, "grid": wl.grid, "ng": P.info["ng"],
                              "mn": P.info["mn"], "nt": nt, "delay_mode": mode,
                              "delay": "multilevel time blocks" if mode else "direct sum over N_g",
                              "gmres_iters_per_step": round(st["total_iters"] / max(nt, 1), 2),
                              "ms_rhs_per_step": round(st["ms_rhs"] / max(nt, 1), 3),
                              "ms_solve_per_step": round(st["ms_solve"] / max(nt, 1), 3),
                              "march_s": round(wall, 3), "setup_s": round(setup_s, 1)}), flush=True)
            del I
        d = out[1] - out[0]
        print(json.dumps({"point": wl.name, "multilevel_vs_direct_rel_l2":
                          float(np.linalg.norm(d) / np.linalg.norm(out[0]))}), flush=True)
        P.close()
        del V
        torch.cuda.empty_cache()


def delay_sweep(torch, W, FP32, ngs=(24, 47, 95, 150)):
    """delay_point at N_g = 24, 47, 95 and 150, one JSON line per point and mode."""
    torch.cuda.set_device(0)
    for ng in ngs:
        for rec in delay_point(torch, W, FP32, ng):
            print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="timed steps (default 100, centred on the pulse peak inside the configured march)")
    ap.add_argument("--warmup", type=int, default=5, help="at least this many untimed steps before the window")
    ap.add_argument("--first", type=int, default=-1,
                    help="first timed step (default: the window is centred on the pulse peak)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--workload", default="batch", choices=["batch", "single", "composite"],
                    help="batch: level-4 sphere, 32 directions; single: one direction; composite: six boxes "
                         "and cylinders, 200 634 RWG, 384^3 padded grid (default 100 timed steps; no CPU "
                         "baseline or whole-step graphs at that size)")
    ap.add_argument("--sync-every", type=int, default=4,
                    help="Arnoldi steps enqueued per host convergence check")
    ap.add_argument("--graph", action="store_true",
                    help="also time the window with Arnoldi steps replayed from HIP graphs (profiling off)")
    ap.add_argument("--no-step-graph", action="store_true",
                    help="skip timing the window with whole time steps replayed from HIP graphs")
    ap.add_argument("--tune-ms", type=int, default=4000,
                    help="autotuner budget before timing (0: keep the library's default shapes)")
    ap.add_argument("--true-residual", action="store_true",
                    help="confirm each step's convergence with a recomputed true residual (one operator "
                         "application more per step) instead of stopping on the GMRES residual estimate")
    ap.add_argument("--no-multilevel", action="store_true",
                    help="skip the multilevel-time-block sub-record (the 32-direction sphere at N_g = 95)")
    ap.add_argument("--plate-history", action="store_true",
                    help="a 16 m plate at chi = 3 (N_g > 32), marched with the direct history sum and with "
                         "multilevel time blocks")
    ap.add_argument("--delay-sweep", action="store_true",
                    help="the delayed field of the 32-direction sphere at N_g = 24, 47, 95, 150 with the k-space temporal "
                         "sum and with multilevel time blocks")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the bench: the sphere size and bandwidth sweep (ET-AIM only, FP64), one JSON "
                         "line per point")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="first copy this many MiB device-to-device (counter calibration)")
    ap.add_argument("--plates", action="store_true",
                    help="--sweep only: square plates of 1-8 m (the EFIE, as the paper's plates) instead of spheres")
    ap.add_argument("--blif", action="store_true",
                    help="--sweep only: the band-limited interpolatory basis (M = 3, extrapolation from 3 samples "
                         "fitted at 6 frequencies) instead of the CPPIF")
    ap.add_argument("--no-cfie", action="store_true",
                    help="skip the CFIE (alpha = 0.5) march of the same window that the EFIE bench adds")
    ap.add_argument("--alpha", type=float, default=1.0,
                    help="1: the EFIE the workloads state; below 1: the CFIE with this alpha (the paper's spheres: "
                         "0.5); the CPU baseline runs for the EFIE only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is design-only"}))
        sys.exit(2)
    import torch
    import workloads as W
    from paper_1408_7060_amd import FP32, FP64
    if args.delay_sweep:
        return delay_sweep(torch, W, FP32)
    if args.plate_history:
        return plate_history(torch, W, FP64)
    if args.sweep:
        return sweep(torch, W, FP64, args.alpha, 1 if args.blif else 0, args.plates)
    from paper_1408_7060_amd._lib import F_CONTINUE_ON_NOCONV, F_GRAPH, F_IMPLICIT_STOP, F_RESIDUAL_CHECK
    # the FP64 residual check of eq. (5) every 16 steps is part of the precision form
    fl = F_CONTINUE_ON_NOCONV | F_RESIDUAL_CHECK | (0 if args.true_residual else F_IMPLICIT_STOP)

    wl = {"batch": W.SPHERE_L4_BATCH, "single": W.SPHERE_L4, "composite": W.COMPOSITE}[args.workload]
    large = wl is W.COMPOSITE
    if large:
        # the oracle's set-up (13.7 M exact near-zone entries) does not fit a
        # CPU leg of minutes; whole-step graphs need the register plane kernels
        args.no_cpu = True
        args.no_step_graph = True
    alpha = args.alpha
    if alpha != 1.0:
        args.no_cpu = True
    K = args.steps
    xyz, _, _ = wl.mesh()
    dt = derived_dt(wl, xyz)
    ng = wl.ng   # every bench workload states N_g
    first, kt, peak = window(wl, dt, ng, K, args.warmup, args.first)
    nt = first + K
    if nt > wl.nt:
        # past the configured length the growing mode of the CPPIF envelope march can overflow FP32
        log(f"[bench] note: the window ends at step {nt - 1}, past the workload's {wl.nt} steps")
    torch.cuda.set_device(0)
    if args.calib_copy:
        n = args.calib_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy} MiB done")
        del src, dst
    log(f"[bench] set-up {wl.name}: B={wl.batch}, timed steps {first}..{nt - 1} (pulse peak at step {peak})")
    t = time.perf_counter()
    P = make_problem(wl, FP32, wl.batch, nt, 1e-5, flags=fl, sync_every=args.sync_every, alpha=alpha)
    log(f"[bench] set-up {time.perf_counter() - t:.1f} s, info {P.info}")
    if abs(P.info["dt"] - dt) > 1e-9 * dt or P.info["ng"] != ng:
        raise SystemExit(f"window derived for dt {dt}, N_g {ng}; the library derived {P.info['dt']}, {P.info['ng']}")
    tuning = None
    if args.tune_ms:
        t = time.perf_counter()
        tuning = P.autotune(budget_ms=args.tune_ms)
        log(f"[bench] autotune {time.perf_counter() - t:.1f} s: {tuning}")
    kh, pp = wl.incidence()
    V = P.excitation(kh, pp, wl.sigma, wl.td)
    I32 = P.empty(nt, wl.batch, P.ns)
    # untimed: steps 0 .. first - kt - 1, then steps first - kt .. first - 1 with
    # every kernel class traced (event markers between launches cost stream time)
    _, st_w = P.march(V, out=I32, nsteps=first - kt)
    P.set_profiling(True)
    _, st_t = P.march_continue(V, I32, first - kt, kt)
    ks = P.kernel_stats()
    log(f"[bench] untimed steps 0..{first - 1} done ({(st_w['total_iters'] + st_t['total_iters']) / first:.2f} "
        f"GMRES it/step)")
    # timed: steps first .. first + K - 1; only the single-kernel classes of the
    # roofline record are traced (their events ride on the dispatch)
    P.set_profiling(classes=TIMED_CLASSES)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = P.march_continue(V, I32, first, K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt_stats = P.kernel_stats()
    P.set_profiling(False)
    wall = t1 - t0
    steps_s = K / wall
    iters = st["total_iters"] / max(K, 1)
    unstable = [x["unstable_step"] for x in (st_w, st_t, st) if x["unstable_step"] >= 0]
    log(f"[bench] timed {K} steps in {wall:.3f} s: {steps_s:.2f} steps/s, {iters:.2f} GMRES it/step, "
        f"phase ms rhs {st['ms_rhs']:.0f} solve {st['ms_solve']:.0f} commit {st['ms_commit']:.0f}")
    for name, v in ks.items():
        if v["launches"]:
            log(f"[bench]   {name:12s} {v['ms']:9.1f} ms {v['launches']:7d} launches "
                f"{v['bytes'] / max(v['ms'], 1e-9) / 1e6:8.1f} GB/s")
    dom = max(FFT_CLASSES, key=lambda n: ks[n]["ms"])
    d = kt_stats[dom] if dom in TIMED_CLASSES else ks[dom]
    roof = roofline_record(dom, d, P.info, wl.batch, hbm_traffic(wl.name, dom))
    roof["timed_in"] = "timed window" if dom in TIMED_CLASSES else "traced pass before the window"
    # one AIM matvec = the four matvec classes once each (launch averages)
    per_matvec_ms = sum(ks[n]["ms"] / ks[n]["launches"] for n in ("anterp_x", "yz_green", "fft_x_inv", "interp_near"))
    copy_gbps = stream_copy_gbps(torch)
    roof["frac_of_stream_copy"] = round((roof["achieved"] if roof["bound"] == "hbm" else roof["hbm_GBps"])
                                        / copy_gbps, 4)
    # the HBM-bound stage: the delayed field streams the history (the time-block
    # pass over the ring plus the per-step sum of the block's own steps)
    dl_b = kt_stats["yz_delayed"]["bytes"] + kt_stats["ring_far"]["bytes"]
    dl_ms = kt_stats["yz_delayed"]["ms"] + kt_stats["ring_far"]["ms"]
    dl_gbs = dl_b / max(dl_ms, 1e-9) / 1e6
    hbm_stream = {"kernels": ["ring_far", "yz_delayed"], "GBps": round(dl_gbs, 1),
                  "frac": round(dl_gbs / HBM_PEAK_GBS, 4), "frac_of_stream_copy": round(dl_gbs / copy_gbps, 4),
                  "ms_per_step": round(dl_ms / max(K, 1), 3),
                  "launches": {n: kt_stats[n]["launches"] for n in ("ring_far", "yz_delayed")},
                  "traffic": {n: hbm_traffic(wl.name, n) for n in ("ring_far", "yz_delayed")}}
    out = {"metric": "ET-AIM time-steps/s & FFT-matvec HBM GB/s, FP32 batched vs FP64, 1 MI355X",
           "value": round(steps_s, 4), "unit": "time-steps/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
           "ms_per_step": round(1e3 * wall / K, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32 (grid/FFT/near) + fp64 (GMRES)", "data": "synthetic",
           "config": {"workload": wl.name, "ns": P.ns, "batch": wl.batch, "grid": wl.grid,
                      "sync_every": args.sync_every,
                      "gmres_stop": "true_residual" if args.true_residual else "residual_estimate",
                      "padded": 2 * wl.grid, "ng": P.info["ng"], "mn": P.info["mn"], "nt": nt, "tol": 1e-5,
                      "formulation": "EFIE" if alpha == 1.0 else f"CFIE alpha={alpha}",
                      "parallelism": "1 GPU"},
           "window": {"first_step": first, "last_step": nt - 1, "untimed_steps_before": first,
                      "pulse_peak_step": peak, "history_terms_per_step": ng},
           "unstable_step": min(unstable) if unstable else None,
           "fp64_residual_check": {
               "column": 0, "every_steps": 16, "checks_in_window": st["residual_checks"],
               "max_rel_residual": st["max_residual64"], "worst_step": st["residual_worst_step"],
               "max_rel_residual_before_window": max(st_w["max_residual64"], st_t["max_residual64"])},
           "direction_steps_per_s": round(steps_s * wl.batch, 3),
           "gmres_iters_per_step": round(iters, 2),
           "roofline": roof,
           "hbm_stream": hbm_stream,
           "matvecs_per_s": round(1e3 / per_matvec_ms, 2),
           "column_matvecs_per_s": round(1e3 * wl.batch / per_matvec_ms, 1),
           "stream_copy_GBps": round(copy_gbps, 1),
           "tuning": tuning,
           "kernels": {n: {"ms": round(v["ms"], 2), "launches": v["launches"],
                           "GBps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)} for n, v in ks.items()
                       if v["launches"]},
           "kernels_from": f"steps {first - kt}..{first - 1}, every class traced"}
    I32_0 = I32[:, 0].cpu().numpy()
    # the current's growth over the window (direction 0): a stable march
    # follows the pulse; the CPPIF growing mode multiplies it every step
    n0, n1 = (float(np.linalg.norm(I32_0[q])) for q in (first, nt - 1))
    out["current_growth_per_step_dir0"] = round((n1 / n0) ** (1.0 / max(K - 1, 1)), 4) if n0 > 0 else None
    P.close()
    del I32
    if args.graph or (tuning and tuning["graph"]):
        Pg = make_problem(wl, FP32, wl.batch, nt, 1e-5, flags=fl | F_GRAPH, sync_every=args.sync_every,
                          alpha=alpha)
        if tuning:
            Pg.set_tuning(dict(tuning, graph=1))
        Ig = Pg.empty(nt, wl.batch, Pg.ns)
        Pg.march(V, out=Ig, nsteps=first)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        _, stg = Pg.march_continue(V, Ig, first, K)
        torch.cuda.synchronize()
        wg = time.perf_counter() - g0
        out["graph"] = {"time_steps_per_s": round(K / wg, 4), "gmres_iters_per_step": round(stg["total_iters"] / K, 2),
                        "max_abs_diff_vs_eager": float(np.abs(Ig[:, 0].cpu().numpy() - I32_0).max())}
        log(f"[bench] graph replay: {K / wg:.2f} steps/s")
        Pg.close()
        del Ig
    if not args.no_step_graph:
        # the same window with every step replayed from a captured whole-step graph
        # (delayed field, device-gated GMRES cycle, commit; several steps per host check)
        Ps = make_problem(wl, FP32, wl.batch, nt, 1e-5, flags=fl, sync_every=args.sync_every, alpha=alpha)
        if tuning:
            Ps.set_tuning(dict(tuning, graph=2))
        else:
            Ps.set_tuning(dict(Ps.tuning(), graph=2))
        Is = Ps.empty(nt, wl.batch, Ps.ns)
        Ps.march(V, out=Is, nsteps=first)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        _, sts = Ps.march_continue(V, Is, first, K)
        torch.cuda.synchronize()
        wsg = time.perf_counter() - g0
        out["step_graph"] = {"time_steps_per_s": round(K / wsg, 4), "ms_per_step": round(1e3 * wsg / K, 3),
                             "gmres_iters_per_step": round(sts["total_iters"] / K, 2),
                             "replayed_steps": sts["graph_steps"], "halts": sts["graph_halts"],
                             "bit_identical_to_eager": bool(np.array_equal(Is[:, 0].cpu().numpy(), I32_0))}
        log(f"[bench] whole-step graphs: {K / wsg:.2f} steps/s ({sts['graph_steps']} replayed, "
            f"{sts['graph_halts']} halts)")
        Ps.close()
        del Is
    del V
    torch.cuda.empty_cache()
    win = slice(first, nt)
    if not args.no_fp64:
        P64 = make_problem(wl, FP64, 1, nt, 1e-5, flags=fl, alpha=alpha)
        if tuning:
            P64.autotune(budget_ms=max(args.tune_ms // 2, 1))
        V64 = P64.excitation(kh[:1], pp[:1], wl.sigma, wl.td)
        I64 = P64.empty(nt, 1, P64.ns)
        P64.march(V64, out=I64, nsteps=first)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        _, st64 = P64.march_continue(V64, I64, first, K)
        torch.cuda.synchronize()
        w64 = time.perf_counter() - s0
        I64_0 = I64[:, 0].cpu().numpy()
        err = float(np.linalg.norm(I32_0[win] - I64_0[win]) / np.linalg.norm(I64_0[win]))
        out["fp64_plain"] = {"direction_steps_per_s": round(K / w64, 3), "time_steps_per_s": round(K / w64, 3),
                             "gmres_iters_per_step": round(st64["total_iters"] / K, 2)}
        out["fp32_batched_over_fp64_plain"] = round(steps_s * wl.batch / (K / w64), 2)
        out["fp32_rel_l2_vs_fp64_dir0"] = err
        out["fp32_max_step_err_vs_fp64_dir0"] = step_err(I32_0[win], I64_0[win])
        out["fp32_rel_l2_vs_fp64_dir0_steps_0_to_last"] = float(np.linalg.norm(I32_0 - I64_0) / np.linalg.norm(I64_0))
        log(f"[bench] fp64 plain: {K / w64:.2f} steps/s; fp32 batch vs fp64 rel L2 over the window {err:.2e}")
        P64.close()
        del I64
    if not args.no_fp64 and not large:
        # precision error apart from the GMRES tolerance: FP32 at tol 1e-7 against
        # FP64 at tol 1e-12, direction 0, over the same window
        res = {}
        for prec, tol in ((FP64, 1e-12), (FP32, 1e-7)):
            Pt = make_problem(wl, prec, 1, nt, tol, flags=fl, alpha=alpha)
            It, _ = Pt.march(V64, nsteps=nt)
            res[prec] = It[:, 0].cpu().numpy()
            Pt.close()
            del It
        out["fp32_precision_error_dir0"] = {
            "steps": [first, nt - 1], "tol_fp32": 1e-7, "tol_fp64": 1e-12,
            "rel_l2": float(np.linalg.norm(res[FP32][win] - res[FP64][win]) / np.linalg.norm(res[FP64][win])),
            "max_step_err": step_err(res[FP32][win], res[FP64][win])}
        log(f"[bench] precision error (tol 1e-7 vs 1e-12, steps {first}..{nt - 1}): "
            f"{out['fp32_precision_error_dir0']['rel_l2']:.2e}")
        del V64
    if alpha == 1.0 and not large and not args.no_cfie:
        # the paper's sphere formulation (Sec. 2.1, Sec. 5.1: CFIE, alpha = 0.5)
        # on the same workload, setting and window
        Pc = make_problem(wl, FP32, wl.batch, nt, 1e-5, flags=fl, sync_every=args.sync_every, alpha=0.5)
        if tuning:
            Pc.set_tuning(tuning)
        Vc = Pc.excitation(kh, pp, wl.sigma, wl.td)
        Ic = Pc.empty(nt, wl.batch, Pc.ns)
        _, stc0 = Pc.march(Vc, out=Ic, nsteps=first)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        _, stc = Pc.march_continue(Vc, Ic, first, K)
        torch.cuda.synchronize()
        wc = time.perf_counter() - c0
        nc = np.linalg.norm(Ic[:, 0].cpu().numpy(), axis=1)
        uc = [x["unstable_step"] for x in (stc0, stc) if x["unstable_step"] >= 0]
        out["cfie"] = {"alpha": 0.5, "time_steps_per_s": round(K / wc, 4), "ms_per_step": round(1e3 * wc / K, 3),
                       "gmres_iters_per_step": round(stc["total_iters"] / K, 2),
                       "unstable_step": min(uc) if uc else None,
                       "current_growth_per_step_dir0": round((nc[nt - 1] / nc[first]) ** (1.0 / max(K - 1, 1)), 4)
                       if nc[first] > 0 else None,
                       "fp64_residual_check_max": stc["max_residual64"]}
        log(f"[bench] CFIE alpha 0.5: {K / wc:.2f} steps/s, {stc['total_iters'] / K:.2f} GMRES it/step")
        Pc.close()
        del Ic, Vc
    if alpha == 1.0 and not large and not args.no_multilevel:
        # the delayed field with multilevel time blocks against the k-space
        # temporal sum, on the same sphere with a history of 95 steps
        torch.cuda.empty_cache()
        r0, r1 = delay_point(torch, W, FP32, 95)
        out["multilevel"] = {"ng": r1["ng"], "window": r1["window"],
                             "delayed_ms_per_step": {"direct_sum": r0["delayed_kernels_ms_per_step"],
                                                     "multilevel": r1["delayed_kernels_ms_per_step"]},
                             "delayed_GB_per_step": {"direct_sum": r0["delayed_GB_per_step"],
                                                     "multilevel": r1["delayed_GB_per_step"]},
                             "time_steps_per_s": {"direct_sum": r0["time_steps_per_s"],
                                                  "multilevel": r1["time_steps_per_s"]},
                             "delayed_speedup": round(r0["delayed_kernels_ms_per_step"] /
                                                      r1["delayed_kernels_ms_per_step"], 3)}
        log(f"[bench] multilevel time blocks at N_g = 95: delayed field {r0['delayed_kernels_ms_per_step']:.2f} -> "
            f"{r1['delayed_kernels_ms_per_step']:.2f} ms per step")
    if large:
        out["cpu_baseline"] = None
        out["cpu_baseline_note"] = ("not run at this size: the oracle's set-up alone (13.7 M exact near-zone "
                                    "entries in numpy) takes far longer than the bench")
    elif alpha != 1.0:
        out["cpu_baseline"] = None
        out["cpu_baseline_note"] = "the CPU baseline is the EFIE run's (the workload's stated formulation)"
    elif not args.no_cpu:
        log("[bench] cpu baseline (oracle march on the host cores, child process) ...")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
