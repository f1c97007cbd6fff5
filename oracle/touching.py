"""Touching triangle pairs: span against c dt, and a refined reference rule
(oracle; test infrastructure only).

The impedance entries of touching pairs (triangles that share a vertex, a
triangle with itself included) are integrated by singularity extraction:
f(R)/R = f(0)/R + [f(R) - f(0)]/R, the first part in closed form over the
source triangle at the 7 outer points, the bounded remainder by the 7 x 7
product of the degree-5 rule (``zfill``).  f(0) is taken from the CPPIF
piece that holds tau = m - R/(c dt) as R -> 0+.

That split assumes f is smooth over the pair.  When the pair spans more than
c dt, tau crosses an integer inside it: T' and T'' jump there (T is only
continuous at its breakpoints), so f_A = exp(-j k_c R) (T''/dt^2 +
2 j w_c T'/dt - w_c^2 T) jumps on the sphere |r - r'| = (m - n) c dt, and the
7 x 7 rule integrates a discontinuous remainder.  This module measures that:

* ``touching_spans``: the largest vertex-vertex distance of every touching
  triangle pair that the near-zone entries use, against c dt;
* ``refined_pair_entries``: Z_m[k, k'] with both triangles of every half
  pair split into n^2 congruent sub-triangles, the extraction applied per
  sub-triangle pair (closed-form 1/R and (r' - rho)/R potentials over each
  source sub-triangle, Wilton et al. 1984 / Graglia 1993), the remainder by
  the 7 x 7 rule per sub-pair.  At n = 1 it is the ``zfill`` rule itself.
  Where the remainder jumps, the error falls as 1/n (the cells the
  discontinuity cuts have measure O(h) of the 4-D domain), so
  ``extrapolated_entries`` combines n and 2n as 2 Z(2n) - Z(n).

Nothing here feeds the parity tests: both sides of the parity contract
use the 7 x 7 rule (the quadrature specification is part of it).  The
numbers this module gives are a statement about the formulation's accuracy
on meshes whose elements are not small against c dt.
"""
from __future__ import annotations

import numpy as np

from .geometry import Surface
from .physics import C0
from .potentials import triangle_potentials
from .quadrature import points, radon7


def touching_spans(surf: Surface, rows, cols):
    """For the basis pairs (rows[p], cols[p]): the largest vertex-vertex
    distance over the triangle pairs of their supports that share a vertex
    (0 where none does).  Returns spans [P]."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    out = np.zeros(len(rows))
    for h in range(2):
        for g in range(2):
            ta, tb = surf.t[rows, h], surf.t[cols, g]
            A, B = surf.tri[ta], surf.tri[tb]
            share = (A[:, :, None] == B[:, None, :]).any(axis=(1, 2))
            va, vb = surf.xyz[A], surf.xyz[B]
            d = np.linalg.norm(va[:, :, None, :] - vb[:, None, :, :], axis=-1).max(axis=(1, 2))
            out = np.where(share, np.maximum(out, d), out)
    return out


def subdivide(verts: np.ndarray, n: int) -> np.ndarray:
    """The n^2 congruent sub-triangles of a triangle verts [3,3] -> [n^2,3,3],
    each with the parent's orientation."""
    a, b, c = verts
    def node(i, j):
        return a + (b - a) * (i / n) + (c - a) * (j / n)
    subs = []
    for i in range(n):
        for j in range(n - i):
            subs.append([node(i, j), node(i + 1, j), node(i, j + 1)])
            if i + j < n - 1:
                subs.append([node(i + 1, j), node(i + 1, j + 1), node(i, j + 1)])
    return np.array(subs)


def _half_pair(surf: Surface, ta: int, va_free, tb: int, vb_free, kernels, n: int):
    """int_Ta int_Tb (r - va_free).(r' - vb_free) f_A/R and int int f_phi/R
    for each kernel, with both triangles split into n^2 sub-triangles.
    Returns (A [K], Phi [K]) without the kernels' scale factors."""
    bary, w = radon7()
    sa = subdivide(surf.tv[ta], n)
    sb = subdivide(surf.tv[tb], n)
    area_a = surf.area[ta] / n ** 2
    area_b = surf.area[tb] / n ** 2
    ra = points(sa, bary).reshape(-1, 3)              # [Pa,3]
    rb = points(sb, bary).reshape(-1, 3)              # [Pb,3]
    wa = np.tile(w, len(sa)) * area_a
    wb = np.tile(w, len(sb)) * area_b
    da = ra - va_free                                   # (r - v)
    db = rb - vb_free                                   # (r' - v')
    # closed-form potentials of each source sub-triangle at each outer point
    I0, I1 = triangle_potentials(ra[:, None, :], sb[None, :, :, :])      # [Pa,Sb], [Pa,Sb,3]
    nb = surf.normal[tb]
    d = np.einsum("px,x->p", ra - surf.tv[tb][0], nb)
    rho = ra - d[:, None] * nb                          # projection on the source plane
    # int_sb (r' - v')/R = I1 + (rho - v') I0, summed over the source sub-triangles
    Vs = I1.sum(axis=1) + (rho - vb_free) * I0.sum(axis=1)[:, None]
    singA = np.einsum("p,px,px->", wa, da, Vs)
    singF = np.einsum("p,p->", wa, I0.sum(axis=1))
    diff = ra[:, None, :] - rb[None, :, :]
    R = np.sqrt(np.einsum("pqx,pqx->pq", diff, diff))
    zero = R == 0.0
    Rs = np.where(zero, 1.0, R)
    W = wa[:, None] * wb[None, :]
    G = np.einsum("px,qx->pq", da, db)
    A, F = [], []
    for kn in kernels:
        fa, fp = kn.f(R)
        (f0a, f0p), (d0a, d0p) = kn.f0(), kn.df0()
        ka = np.where(zero, d0a, (fa - f0a) / Rs)
        kp = np.where(zero, d0p, (fp - f0p) / Rs)
        A.append(np.sum(W * G * ka) + f0a * singA)
        F.append(np.sum(W * kp) + f0p * singF)
    return np.array(A), np.array(F)


def refined_pair_entries(surf: Surface, k: int, k2: int, kernels, n: int) -> np.ndarray:
    """Z[kernel] for the basis pair (k, k2) with every half pair's triangles
    split into n^2 sub-triangles (n = 1: the 7 x 7 rule with extraction)."""
    out = np.zeros(len(kernels), dtype=np.complex128)
    sa = np.array([kn.scale_a for kn in kernels])
    sp = np.array([kn.scale_phi for kn in kernels])
    for h in range(2):
        ta = surf.t[k, h]
        ca = surf.s[k, h] * surf.length[k] / (2.0 * surf.area[ta])
        cp = surf.s[k, h] * surf.length[k] / surf.area[ta]
        for g in range(2):
            tb = surf.t[k2, g]
            cb = surf.s[k2, g] * surf.length[k2] / (2.0 * surf.area[tb])
            cq = surf.s[k2, g] * surf.length[k2] / surf.area[tb]
            A, F = _half_pair(surf, ta, surf.xyz[surf.free[k, h]], tb, surf.xyz[surf.free[k2, g]], kernels, n)
            out += sa * ca * cb * A + sp * cp * cq * F
    return out


def extrapolated_entries(surf: Surface, k: int, k2: int, kernels, n: int) -> np.ndarray:
    """2 Z(2n) - Z(n): the first-order extrapolation of the refined rule."""
    return 2.0 * refined_pair_entries(surf, k, k2, kernels, 2 * n) - refined_pair_entries(surf, k, k2, kernels, n)


def cdt(dt: float) -> float:
    return C0 * dt
