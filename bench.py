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
+ forward FFT into the history ring).  --warmup W marches W untimed steps
first; the timed region is one march of --steps K steps from a zero history,
bracketed by torch.cuda.synchronize().  Inputs (excitation) are resident in
HBM before timing.

Printed: one JSON line with the metric, the roofline record of the dominant
kernel class (algorithmic bytes / device time, HIP events on the library's
stream over the timed region), the plain FP64 GPU path on the first
direction for comparison, the FP32-vs-FP64 error on that direction, and the
CPU oracle baseline on a bounded sample.  Inside the timed region only the
roofline kernel and the delayed-field kernels are traced (their events ride
on the dispatch); the per-class table ("kernels") comes from a second,
untimed march of K steps with every class traced.
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
# FP32 vector FMA issue rate without packed FP32 instructions (the build
# disables them): 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
CSRC = os.path.join(ROOT, "paper_1408_7060_amd", "csrc")
FFT_CLASSES = ("anterp_x", "yz_green", "fft_x_inv", "interp_near", "yz_delayed", "yz_commit", "ring_far")
# traced inside the timed region: the roofline kernel and the delayed-field
# stream (single-kernel classes, whose HIP events ride on the dispatch itself)
TIMED_CLASSES = ("yz_green", "yz_delayed", "ring_far")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problem(wl, precision, batch, nt, tol, flags=1, sync_every=1):
    import workloads as W  # noqa: F401
    from paper_1408_7060_amd import Problem
    xyz, tri, rwg = wl.mesh()
    d_near = wl.near_lambda * 299_792_458.0 / wl.f0
    kw = dict(fc=wl.f0, nt=nt, grid=wl.grid, d_near=d_near, precision=precision, batch=batch, tol=tol,
              restart=50, maxit=2000, flags=flags, sync_every=sync_every)
    if wl.ng:
        kw["ng"] = wl.ng
    else:
        kw.update(beta=wl.beta, f_bw=wl.f_bw)
    return Problem(xyz, tri, rwg, **kw)


def cpu_baseline(wl, iters_per_step, budget_s=20.0):
    """Oracle (numpy FP64, as it stands) on a bounded sample: time the
    oracle's AIM operator application (FFT convolution + near SpMV) at the
    workload's size for one direction, then price one oracle time step as
    (N_g delayed-field applications + average GMRES iterations + 1)."""
    from oracle import aim, geometry, physics as ph
    xyz, tri, rwg = wl.mesh()
    s = geometry.Surface(xyz, tri, rwg)
    rmax = ph.rmax_of(xyz)
    dt = ph.dt_from_ng(rmax, wl.ng) if wl.ng else ph.dt_from_beta(wl.beta, wl.f_bw)
    ng = wl.ng or ph.ng_from(rmax, dt)
    A = aim.AIM(s, wl.grid, wl.near_lambda * ph.C0 / wl.f0, dt, wl.f0, ng)
    vals = np.zeros(len(A.rows), dtype=np.complex128)    # timing only: cost is value-independent
    import workloads as W
    x = W.complex_normal(3, s.ns)
    n, t0 = 0, time.perf_counter()
    while True:
        A.far_matvec(n % (ng + 1), x)
        A.near_matvec(vals, x)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 50:
            break
    t_mv = (time.perf_counter() - t0) / n
    step_s = (ng + iters_per_step + 1) * t_mv * wl.batch
    return {"value": 1.0 / step_s, "unit": "time-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} oracle AIM operator applications (numpy FP64, {s.ns} RWG, {2 * wl.grid}^3 FFT) "
                      f"at {t_mv:.3f} s each; one step of the {wl.batch}-direction job priced as "
                      f"{wl.batch} x ({ng} delayed + {iters_per_step:.1f} GMRES + 1) applications; "
                      f"near-zone values zero (cost is value-independent)"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="timed steps (default: the workload's N_t)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--workload", default="batch", choices=["batch", "single"])
    ap.add_argument("--sync-every", type=int, default=4,
                    help="Arnoldi steps enqueued per host convergence check")
    ap.add_argument("--graph", action="store_true",
                    help="also time the march with Arnoldi steps replayed from HIP graphs (profiling off)")
    ap.add_argument("--tune-ms", type=int, default=4000,
                    help="autotuner budget before timing (0: keep the library's default shapes)")
    ap.add_argument("--true-residual", action="store_true",
                    help="confirm each step's convergence with a recomputed true residual (one operator "
                         "application more per step) instead of stopping on the GMRES residual estimate")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="first copy this many MiB device-to-device (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is design-only"}))
        sys.exit(2)
    import torch
    import workloads as W
    from paper_1408_7060_amd import FP32, FP64
    from paper_1408_7060_amd._lib import F_CONTINUE_ON_NOCONV, F_GRAPH, F_IMPLICIT_STOP
    fl = F_CONTINUE_ON_NOCONV | (0 if args.true_residual else F_IMPLICIT_STOP)

    wl = W.SPHERE_L4_BATCH if args.workload == "batch" else W.SPHERE_L4
    K = args.steps or wl.nt
    nt = max(K, args.warmup, 1)
    torch.cuda.set_device(0)
    if args.calib_copy:
        n = args.calib_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy} MiB done")
        del src, dst
    log(f"[bench] set-up {wl.name}: B={wl.batch} nt={nt}")
    t = time.perf_counter()
    P = make_problem(wl, FP32, wl.batch, nt, 1e-5, flags=fl, sync_every=args.sync_every)
    log(f"[bench] set-up {time.perf_counter() - t:.1f} s, info {P.info}")
    tuning = None
    if args.tune_ms:
        t = time.perf_counter()
        tuning = P.autotune(budget_ms=args.tune_ms)
        log(f"[bench] autotune {time.perf_counter() - t:.1f} s: {tuning}")
    kh, pp = wl.incidence()
    V = P.excitation(kh, pp, wl.sigma, wl.td)
    if args.warmup:
        P.march(V, nsteps=args.warmup)
        log(f"[bench] warm-up {args.warmup} steps done")
    # inside the timed region only the roofline kernel and the delayed-field
    # stream are traced (single-kernel classes: their events ride on the dispatch);
    # the per-class table comes from a second, untimed pass that traces every
    # class (event markers between launches cost stream time)
    P.set_profiling(classes=TIMED_CLASSES)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    I32, st = P.march(V, nsteps=K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = P.kernel_stats()
    P.set_profiling(True)
    P.march(V, nsteps=K)
    ks = P.kernel_stats()
    P.set_profiling(False)
    wall = t1 - t0
    steps_s = K / wall
    iters = st["total_iters"] / max(K, 1)
    log(f"[bench] timed {K} steps in {wall:.2f} s: {steps_s:.2f} steps/s, {iters:.1f} GMRES it/step, "
        f"phase ms rhs {st['ms_rhs']:.0f} solve {st['ms_solve']:.0f} commit {st['ms_commit']:.0f}")
    for name, v in ks.items():
        if v["launches"]:
            log(f"[bench]   {name:12s} {v['ms']:9.1f} ms {v['launches']:7d} launches "
                f"{v['bytes'] / max(v['ms'], 1e-9) / 1e6:8.1f} GB/s")
    dom = max(FFT_CLASSES, key=lambda n: ks[n]["ms"])
    d = kt[dom] if dom in TIMED_CLASSES else ks[dom]
    avg_ms = d["ms"] / d["launches"]
    bytes_launch = d["bytes"] / d["launches"]
    hbm_gbs = bytes_launch / (avg_ms / 1e3) / 1e9
    traffic = hbm_traffic(wl.name, dom)
    flops = class_flops(dom, P.info, wl.batch)
    if flops is not None and flops / (avg_ms / 1e3) / 1e12 / ALU_PEAK_TFLOPS > hbm_gbs / HBM_PEAK_GBS:
        # the FFT work, not the bytes, bounds this kernel: roofline against the FP32 vector issue rate
        achieved = flops / (avg_ms / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 2), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / ALU_PEAK_TFLOPS, 4), "traffic": traffic, "kernel": dom,
                "flops_per_launch": flops, "bytes_per_launch": bytes_launch, "avg_launch_ms": avg_ms,
                "hbm_GBps": round(hbm_gbs, 1), "hbm_frac": round(hbm_gbs / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "bytes_per_launch": bytes_launch, "avg_launch_ms": avg_ms}
    # one AIM matvec = the four matvec classes once each (launch averages)
    per_matvec_ms = sum(ks[n]["ms"] / ks[n]["launches"] for n in ("anterp_x", "yz_green", "fft_x_inv", "interp_near"))
    copy_gbps = stream_copy_gbps(torch)
    roof["frac_of_stream_copy"] = round((hbm_gbs if roof["bound"] == "hbm" else roof["hbm_GBps"]) / copy_gbps, 4)
    # the HBM-bound stage: the delayed field streams the history (the time-block
    # pass over the ring plus the per-step sum of the block's own steps)
    dl_b = kt["yz_delayed"]["bytes"] + kt["ring_far"]["bytes"]
    dl_ms = kt["yz_delayed"]["ms"] + kt["ring_far"]["ms"]
    dl_gbs = dl_b / max(dl_ms, 1e-9) / 1e6
    hbm_stream = {"kernels": ["ring_far", "yz_delayed"], "GBps": round(dl_gbs, 1),
                  "frac": round(dl_gbs / HBM_PEAK_GBS, 4), "frac_of_stream_copy": round(dl_gbs / copy_gbps, 4),
                  "ms_per_step": round(dl_ms / max(K, 1), 3),
                  "traffic": {n: hbm_traffic(wl.name, n) for n in ("ring_far", "yz_delayed")}}
    out = {"metric": "ET-AIM time-steps/s & FFT-matvec HBM GB/s, FP32 batched vs FP64, 1 MI355X",
           "value": round(steps_s, 4), "unit": "time-steps/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
           "ms_per_step": round(1e3 * wall / K, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32 (grid/FFT/near) + fp64 (GMRES)", "data": "synthetic",
           "config": {"workload": wl.name, "ns": P.ns, "batch": wl.batch, "grid": wl.grid,
                      "sync_every": args.sync_every,
                      "gmres_stop": "true_residual" if args.true_residual else "residual_estimate",
                      "padded": 2 * wl.grid, "ng": P.info["ng"], "mn": P.info["mn"], "nt": K, "tol": 1e-5,
                      "parallelism": "1 GPU"},
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
                       if v["launches"]}}
    I32_0 = I32[:, 0].cpu().numpy()
    P.close()
    if args.graph or (tuning and tuning["graph"]):
        Pg = make_problem(wl, FP32, wl.batch, nt, 1e-5, flags=fl | F_GRAPH, sync_every=args.sync_every)
        if tuning:
            Pg.set_tuning(dict(tuning, graph=1))
        if args.warmup:
            Pg.march(V, nsteps=args.warmup)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        Ig, stg = Pg.march(V, nsteps=K)
        torch.cuda.synchronize()
        wg = time.perf_counter() - g0
        out["graph"] = {"time_steps_per_s": round(K / wg, 4), "gmres_iters_per_step": round(stg["total_iters"] / K, 2),
                        "max_abs_diff_vs_eager": float((Ig[:, 0].cpu().numpy() - I32_0).__abs__().max())}
        log(f"[bench] graph replay: {K / wg:.2f} steps/s")
        Pg.close()
        del Ig
    del V, I32
    torch.cuda.empty_cache()
    if not args.no_fp64:
        P64 = make_problem(wl, FP64, 1, nt, 1e-5, flags=fl)
        V64 = P64.excitation(kh[:1], pp[:1], wl.sigma, wl.td)
        if args.warmup:
            P64.march(V64, nsteps=args.warmup)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        I64, st64 = P64.march(V64, nsteps=K)
        torch.cuda.synchronize()
        w64 = time.perf_counter() - s0
        I64_0 = I64[:, 0].cpu().numpy()
        err = float(np.linalg.norm(I32_0[:K] - I64_0[:K]) / np.linalg.norm(I64_0[:K]))
        out["fp64_plain"] = {"direction_steps_per_s": round(K / w64, 3), "time_steps_per_s": round(K / w64, 3),
                             "gmres_iters_per_step": round(st64["total_iters"] / K, 2)}
        out["fp32_batched_over_fp64_plain"] = round(steps_s * wl.batch / (K / w64), 2)
        out["fp32_rel_l2_vs_fp64_dir0"] = err
        out["fp32_max_step_err_vs_fp64_dir0"] = step_err(I32_0[:K], I64_0[:K])
        log(f"[bench] fp64 plain: {K / w64:.2f} steps/s; fp32 batch vs fp64 rel L2 {err:.2e}")
        P64.close()
        del I64
        # precision error apart from the GMRES tolerance: FP32 at tol 1e-7
        # against FP64 at tol 1e-12, direction 0, the first Kp steps
        Kp = min(K, 100)
        Pt = make_problem(wl, FP64, 1, nt, 1e-12, flags=fl)
        It64, _ = Pt.march(V64, nsteps=Kp)
        It64 = It64[:Kp, 0].cpu().numpy()
        Pt.close()
        Pt = make_problem(wl, FP32, 1, nt, 1e-7, flags=fl)
        It32, _ = Pt.march(V64, nsteps=Kp)
        It32 = It32[:Kp, 0].cpu().numpy()
        Pt.close()
        out["fp32_precision_error_dir0"] = {
            "steps": Kp, "tol_fp32": 1e-7, "tol_fp64": 1e-12,
            "rel_l2": float(np.linalg.norm(It32 - It64) / np.linalg.norm(It64)),
            "max_step_err": step_err(It32, It64)}
        log(f"[bench] precision error (tol 1e-7 vs 1e-12, {Kp} steps): "
            f"{out['fp32_precision_error_dir0']['rel_l2']:.2e}")
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl, iters / 1.0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
