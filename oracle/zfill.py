"""Impedance matrices (oracle; test infrastructure only).

Envelope matrices of eq. (4) (Sec. 3), entries written out from the reading
in ``kernels`` (entries are deferred by the paper to refs. [5], [7]):

    Z_m[k,k'] = int int  S_k . S_k' K_A(m,R) + (div S_k)(div' S_k') K_phi(m,R)

Quadrature reading (Sec. 5.1 names cubature and singularity extraction but no
rule):
* every triangle pair: 7 x 7 product of the degree-5 rule;
* triangle pairs that share at least one vertex (touching, including a
  triangle with itself): f(R)/R = f(0)/R + [f(R) - f(0)]/R; the f(0)/R part
  integrated in closed form over the source triangle at the 7 outer points
  (``potentials``), the bounded remainder by the 7 x 7 rule, its value at
  R = 0 being f'(0).

The frequency-domain EFIE matrix at f uses the same rules (FDKernel).
Pins: Radon rule exactness, closed-form potentials vs brute force, the sum
over m of Z_m equals j w_c Z_FD(f_c) (partition of unity), symmetry, and
the FD solution against the Mie series.
"""
from __future__ import annotations

import numpy as np

from .geometry import Surface
from .potentials import triangle_potentials
from .quadrature import points, radon7

_R0_TOL = 1e-12


def touching(surf: Surface, ta: np.ndarray, tb: np.ndarray) -> np.ndarray:
    A = surf.tri[ta]
    B = surf.tri[tb]
    return (A[:, :, None] == B[:, None, :]).any(axis=(1, 2))


def tri_pair_integrals(surf: Surface, ta, tb, kernels, chunk: int = 8192):
    """Local integrals for triangle pairs (ta[p], tb[p]) and a list of kernels.

    Returns A [P, K, 3, 3] = int_Ta int_Tb (r - v_i).(r' - v'_j) f(R)/R and
    Phi [P, K] = int int f_phi(R)/R, where v_i / v'_j are the local vertices
    of Ta / Tb.  Kernel scale factors are not applied.
    """
    ta = np.asarray(ta, dtype=np.int64)
    tb = np.asarray(tb, dtype=np.int64)
    P, K = len(ta), len(kernels)
    A_out = np.zeros((P, K, 3, 3), dtype=np.complex128)
    F_out = np.zeros((P, K), dtype=np.complex128)
    bary, w = radon7()
    f0 = [kn.f0() for kn in kernels]
    df0 = [kn.df0() for kn in kernels]
    for s in range(0, P, chunk):
        a = ta[s:s + chunk]
        b = tb[s:s + chunk]
        va, vb = surf.tv[a], surf.tv[b]                     # [p,3,3]
        ra, rb = points(va, bary), points(vb, bary)         # [p,7,3]
        diff = ra[:, :, None, :] - rb[:, None, :, :]
        R = np.sqrt(np.einsum("pqrx,pqrx->pqr", diff, diff))
        W = (w[:, None] * w[None, :])[None] * (surf.area[a] * surf.area[b])[:, None, None]
        Da = ra[:, :, None, :] - va[:, None, :, :]          # [p,7,i,x]
        Db = rb[:, :, None, :] - vb[:, None, :, :]
        tch = touching(surf, a, b)
        zero = R == 0.0
        Rs = np.where(zero, 1.0, R)
        if np.any(tch):
            # closed-form inner potentials over Tb at the outer points of Ta
            I0, I1 = triangle_potentials(ra[tch], vb[tch][:, None, :, :])
            nb = np.cross(vb[tch][:, 1] - vb[tch][:, 0], vb[tch][:, 2] - vb[tch][:, 0])
            nb /= np.linalg.norm(nb, axis=-1, keepdims=True)
            d = np.einsum("pqx,px->pq", ra[tch] - vb[tch][:, None, 0, :], nb)
            rho = ra[tch] - d[..., None] * nb[:, None, :]
            # int_Tb (r' - v'_j)/R = I1 + (rho - v'_j) I0        [p,7,j,x]
            Vj = I1[:, :, None, :] + (rho[:, :, None, :] - vb[tch][:, None, :, :]) * I0[:, :, None, None]
            wa = w[None, :] * surf.area[a[tch]][:, None]
            singA = np.einsum("pq,pqix,pqjx->pij", wa, Da[tch], Vj)
            singF = np.einsum("pq,pq->p", wa, I0)
        for ki, kn in enumerate(kernels):
            fa, fp = kn.f(R)
            ka = fa / Rs
            kp = fp / Rs
            if np.any(tch):
                t3 = tch[:, None, None]
                ka = np.where(t3, (fa - f0[ki][0]) / Rs, ka)
                kp = np.where(t3, (fp - f0[ki][1]) / Rs, kp)
                ka = np.where(zero & t3, df0[ki][0], ka)
                kp = np.where(zero & t3, df0[ki][1], kp)
            WK = W * ka
            A = np.einsum("pqr,pqix,prjx->pij", WK, Da, Db, optimize=True)
            F = np.einsum("pqr,pqr->p", W, kp)
            if np.any(tch):
                A[tch] += f0[ki][0] * singA
                F[tch] += f0[ki][1] * singF
            A_out[s:s + chunk, ki] = A
            F_out[s:s + chunk, ki] = F
    return A_out, F_out


def _half_coefs(surf: Surface):
    """Per basis half h: (triangle, local free vertex, coefA, coefPhi)."""
    t = surf.t
    l = surf.length[:, None]
    ar = surf.area[t]
    ca = surf.s * l / (2.0 * ar)      # S = ca (r - v)
    cp = surf.s * l / ar              # div S = cp
    return t, surf.loc, ca, cp


def assemble_pairs(surf: Surface, rows, cols, kernels):
    """Matrix entries Z[kernel][p] for basis pairs (rows[p], cols[p])."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    t, loc, ca, cp = _half_coefs(surf)
    nt = len(surf.tri)
    keys = []
    for h in range(2):
        for g in range(2):
            keys.append(t[rows, h] * nt + t[cols, g])
    uniq, inv = np.unique(np.concatenate(keys), return_inverse=True)
    A, F = tri_pair_integrals(surf, uniq // nt, uniq % nt, kernels)
    inv = inv.reshape(4, -1)
    out = np.zeros((len(kernels), len(rows)), dtype=np.complex128)
    sa = np.array([kn.scale_a for kn in kernels])[:, None]
    sp = np.array([kn.scale_phi for kn in kernels])[:, None]
    i4 = 0
    for h in range(2):
        for g in range(2):
            u = inv[i4]
            i4 += 1
            Aij = A[u, :, loc[rows, h], loc[cols, g]].T          # [K, P]
            out += sa * (ca[rows, h] * ca[cols, g])[None] * Aij
            out += sp * (cp[rows, h] * cp[cols, g])[None] * F[u].T
    return out


def assemble_dense(surf: Surface, kernels) -> np.ndarray:
    """Dense [K, ns, ns] matrices (small meshes only)."""
    ns = surf.ns
    rr, cc = np.meshgrid(np.arange(ns), np.arange(ns), indexing="ij")
    vals = assemble_pairs(surf, rr.ravel(), cc.ravel(), kernels)
    return vals.reshape(len(kernels), ns, ns)
