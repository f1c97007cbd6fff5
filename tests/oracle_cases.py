"""Cached small oracle problems shared by the CPU pin tests."""
import functools
import math

import numpy as np

import workloads as W
from oracle import geometry, kernels, physics as ph, zfill


@functools.lru_cache(maxsize=None)
def sphere(level=2, radius=0.5):
    xyz, tri = W.icosphere(level, radius)
    return geometry.Surface(xyz, tri, W.rwg_table(tri))


@functools.lru_cache(maxsize=None)
def dense_z(dt, fc, ng, fd_freqs=()):
    """Dense Z_0..Z_ng (envelope) followed by FD matrices at fd_freqs."""
    s = sphere()
    ks = [kernels.EnvelopeKernel(m, dt, fc) for m in range(ng + 1)]
    ks += [kernels.FDKernel(f) for f in fd_freqs]
    return zfill.assemble_dense(s, ks)


def l2_band_params(frac=0.2, beta=0.2, fc=300e6):
    s = sphere()
    fbw = frac * fc
    dt = beta / fbw
    ng = ph.ng_from(ph.rmax_of(s.xyz), dt)
    return dt, ng


@functools.lru_cache(maxsize=None)
def dense_h(dt, fc, ng, fd_freqs=()):
    """Dense envelope MFIE Z^H_0..Z^H_ng followed by FD MFIE matrices at fd_freqs."""
    from oracle import mfie
    s = sphere()
    ks = [mfie.MFIEKernel(m, dt, fc) for m in range(ng + 1)]
    ks += [mfie.FDMFIEKernel(f) for f in fd_freqs]
    return mfie.assemble_dense(s, ks)
