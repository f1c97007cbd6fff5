"""Oracle references and library problems for the GPU parity tests."""
import functools
import math

import numpy as np

import workloads as W
from oracle import aim, geometry, kernels, physics as ph, zfill


def params_of(wl):
    xyz, tri, rwg = wl.mesh()
    rmax = ph.rmax_of(xyz)
    if wl.ng:
        dt, ng = ph.dt_from_ng(rmax, wl.ng), wl.ng
    else:
        dt = ph.dt_from_beta(wl.beta, wl.f_bw)
        ng = ph.ng_from(rmax, dt)
    return dict(xyz=xyz, tri=tri, rwg=rwg, dt=dt, ng=ng, d_near=wl.near_lambda * ph.C0 / wl.f0)


def blif_of(wl, dt):
    """The BLIF (M = 3, beta = f_bw dt) and its extrapolation (3 samples, 6
    frequencies) for a workload."""
    from oracle import blif
    b = blif.Blif(3, wl.f_bw * dt)
    return b, blif.extrapolation(b.beta, 3, 3, 6)


@functools.lru_cache(maxsize=None)
def oracle_aim(name, alpha=1.0, basis=0):
    """(surface, AIM object, pre-corrected near values [mn+1, nnz], params);
    alpha < 1: the CFIE; basis 1: the BLIF."""
    wl = W.WORKLOADS[name]
    p = params_of(wl)
    s = geometry.Surface(p["xyz"], p["tri"], p["rwg"])
    b, a = blif_of(wl, p["dt"]) if basis else (None, None)
    A = aim.AIM(s, wl.grid, p["d_near"], p["dt"], wl.f0, p["ng"], alpha=alpha, basis=b, fold_a=a)

    def exact(rows, cols, ms):
        if alpha != 1.0:
            from oracle import mfie
            return mfie.cfie_pairs(s, rows, cols, ms, p["dt"], wl.f0, alpha, b)
        return zfill.assemble_pairs(s, rows, cols, [kernels.EnvelopeKernel(m, p["dt"], wl.f0, b) for m in ms])

    vals = A.near_values(exact)
    return s, A, vals, p


def oracle_matvec(name, m, x, direct=True, alpha=1.0, basis=0):
    """(Z^near_m + Z^FFT_m) x for x [B, ns] by the literal sums."""
    s, A, vals, p = oracle_aim(name, alpha, basis)
    out = []
    for xb in np.atleast_2d(x):
        y = A.far_matvec(m, xb, direct=direct)
        if m <= A.mn:
            y = y + A.near_matvec(vals[m], xb)
        out.append(y)
    return np.array(out)


@functools.lru_cache(maxsize=None)
def oracle_dense_aim(name, alpha=1.0, basis=0):
    """Assembled Z^AIM_m = Z^near_m + Z^FFT_m, [ng+1, ns, ns] (tiny problems)."""
    s, A, vals, p = oracle_aim(name, alpha, basis)
    Z = np.stack([A.far_dense(m) for m in range(p["ng"] + 1)])
    for m in range(A.mn + 1):
        np.add.at(Z[m], (A.rows, A.cols), vals[m])
    return Z


def gpu_problem(name, precision=0, tol=1e-13, batch=None, nt=None, restart=60, maxit=2000, flags=0, sync_every=1,
                grid=None, alpha=1.0, basis=0):
    from paper_1408_7060_amd import Problem
    wl = W.WORKLOADS[name]
    p = params_of(wl)
    kw = dict(fc=wl.f0, nt=nt or wl.nt, grid=grid or wl.grid, d_near=p["d_near"], precision=precision,
              batch=batch or wl.batch, tol=tol, restart=restart, maxit=maxit, flags=flags,
              sync_every=sync_every, alpha=alpha, basis=basis)
    if wl.ng:
        kw["ng"] = wl.ng
        if basis:
            kw["f_bw"] = wl.f_bw
    else:
        kw.update(beta=wl.beta, f_bw=wl.f_bw)
    return Problem(p["xyz"], p["tri"], p["rwg"], **kw)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
