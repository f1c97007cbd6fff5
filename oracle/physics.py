"""Constants and parameter rules (oracle; test infrastructure only).

* Free space (Sec. 2.1: homogeneous medium eps, mu).
* Pulse of eq. (1): band f_c +- 3/(2 pi sigma), delay t_d = 8 sigma (Sec. 2.2,
  Table I).
* Band measures (Sec. 2.3): f_bw = (f_max - f_min)/2, chi = f_max / f_bw.
* Time step dt = beta / f_bw, N_t = floor(T_s / dt) (Sec. 3, after eq. (3)).
* History depth N_g = floor(R_max / (c dt) + l_max) (Sec. 3, after eq. (4)),
  with l_max = Q for the order-Q CPPIF.
"""
from __future__ import annotations

import math

import numpy as np

C0 = 299_792_458.0
MU0 = 4.0e-7 * math.pi
EPS0 = 1.0 / (MU0 * C0 * C0)
ETA0 = math.sqrt(MU0 / EPS0)
Q_CPPIF = 3


def sigma_from_band(f_bw: float) -> float:
    """sigma such that the pulse band f_c +- 3/(2 pi sigma) has half-width f_bw."""
    return 3.0 / (2.0 * math.pi * f_bw)


def band_from_sigma(sigma: float) -> float:
    """Half-width 3/(2 pi sigma) of the pulse band (Sec. 2.2)."""
    return 3.0 / (2.0 * math.pi * sigma)


def chi(f_min: float, f_max: float) -> float:
    """chi = f_max / f_bw with f_bw = (f_max - f_min)/2 (Sec. 2.3)."""
    return f_max / ((f_max - f_min) / 2.0)


def dt_from_beta(beta: float, f_bw: float) -> float:
    return beta / f_bw


def nt_from(ts: float, dt: float) -> int:
    """N_t = floor(T_s/dt); a relative 1e-9 guard absorbs decimal rounding of
    printed values such as 0.24 us / 2 ns."""
    return int(math.floor(ts / dt * (1.0 + 1e-9)))


def ng_from(rmax: float, dt: float, lmax: int = Q_CPPIF) -> int:
    """N_g = floor(R_max/(c dt) + l_max)."""
    return int(math.floor(rmax / (C0 * dt) + lmax))


def dt_from_ng(rmax: float, ng: int, lmax: int = Q_CPPIF) -> float:
    """Time step that makes floor(R_max/(c dt) + l_max) land mid-interval on ng:
    R_max/(c dt) = ng - l_max + 1/2."""
    return rmax / (C0 * (ng - lmax + 0.5))


def rmax_of(xyz: np.ndarray) -> float:
    """Largest vertex-to-vertex distance of the mesh: brute force over the
    vertices of the point set's convex hull (a farthest pair of points is a
    pair of hull vertices); over all vertices where the hull is degenerate
    or the set is small."""
    xyz = np.asarray(xyz, dtype=np.float64)
    if len(xyz) > 2048:
        try:
            from scipy.spatial import ConvexHull
            xyz = xyz[ConvexHull(xyz).vertices]
        except Exception:       # flat or degenerate point sets: all vertices
            pass
    best = 0.0
    for s in range(0, len(xyz), 512):
        d = xyz[s:s + 512, None, :] - xyz[None, :, :]
        best = max(best, float(np.sqrt((d * d).sum(-1)).max()))
    return best
