"""Magnetic-field and combined-field envelope operators (oracle; test
infrastructure only).

The paper forms a CFIE from the EFIE and MFIE on the envelopes (Sec. 2.1),
with alpha = 0.5 for spheres and alpha = 1 (pure EFIE) for plates (Sec. 5.1);
the derivation is deferred to its ref. [7].  Reading, written out here:

* MFIE on the exterior side of a closed PEC surface with outward normal n,
  differentiated in time like the EFIE (so that the two combine with one
  time-stepping scheme):
      dJ/dt / 2 - n x curl(dA/dt) / mu = n x dH_inc/dt   (principal value),
  A the retarded vector potential.  On envelopes d/dt -> D = d/dt + j w_c.
* Testing with S_k (Galerkin), point testing at t = l dt and the CPPIF
  temporal basis T give, for m = l - l', tau = m - R/(c dt):
      Z^H_m[k,k'] = D_m / 2 <S_k, S_k'>
                    - int int g'_m(R) S_k . (n x (Rhat x S_k'))
  with curl(S' g) = g'(R) Rhat x S', Rhat = (r - r')/R, and
      g'_m(R) = -(exp(-j k_c R) / 4 pi) [P_A(tau) / (c R) + (DT)(tau) / R^2],
      P_A = T''/dt^2 + 2 j w_c T'/dt - w_c^2 T,  DT = T'/dt + j w_c T.
  D_m = (DT)(m) takes piece m of T (the piece that holds tau -> m from
  below, as the EFIE's R -> 0 limits do).
* Quadrature: the 7 x 7 product of the degree-5 rule on every triangle
  pair; a triangle with itself contributes nothing (on a flat triangle
  Rhat x S' is along n, so n x (Rhat x S') = 0 exactly).  The Gram term
  <S_k, S_k'> is integrated exactly by the 7-point rule (degree 2).
* CFIE: Z^C_m = alpha Z^E_m + (1 - alpha) eta Z^H_m, right-hand side
  alpha <S, D E~_inc> + (1 - alpha) <S, n x (khat x D E~_inc)> (the plane
  wave's H~ = khat x E~ / eta).
* Frequency domain at f (the pins): Z^H = 1/2 <S, S'> - int int g' S.(n x
  (Rhat x S')) with g' = -(exp(-j k R)/4 pi)(j k / R + 1 / R^2); the
  envelope matrices sum to j w_c Z^H_FD(f_c) (partition of unity of T).
* AIM form: with the tensor cubic Lagrange functions l_n of a basis's 4^3
  stencil, curl A(r) ~ sum_n grad l_n(r) x A_n, so
      <S_k, n x curl A> = sum_n sum_c H[k, c, n] A_c(node n),
      H[k, :, n] = int (S_k x n) x grad l_n dS,
  exact for potentials of degree <= 3 per axis (the matching order of the
  projection).  Far part of the MFIE: - sum_c H_c G^H_m L_c^T with
  G^H_m[d] = exp(-j k_c R) (DT)(tau) / (4 pi R), R = h |d|, G^H[0] = 0:
  the curl of the DT-weighted vector potential of the anterpolated
  currents.

Pins (tests/test_oracle_cfie.py): the FD MFIE and CFIE solutions of the
sphere against the Mie series; the EFIE's interior resonance of the
a = 0.5 m sphere (k a = 2.744) absent from the CFIE; the envelope sum rule;
H exact on polynomial potentials (their curls taken by hand); the AIM far
part against the exact entries on separated pairs.
"""
from __future__ import annotations

import math

import numpy as np

from .kernels import basis_origin, basis_T
from .geometry import Surface
from .physics import C0, ETA0
from .quadrature import collapsed_gauss, points, radon7


class MFIEKernel:
    """g'_m(R) of the envelope MFIE for one m, and its Gram factor D_m
    (basis: None for the CPPIF, or an ``oracle.blif.Blif``)."""

    def __init__(self, m: int, dt: float, fc: float, basis=None):
        self.m, self.dt, self.basis = m, dt, basis
        self.w = 2.0 * math.pi * fc
        self.k = self.w / C0

    def gp(self, R):
        tau = self.m - R / (C0 * self.dt)
        T0, T1, T2 = (basis_T(self.basis, tau, d) for d in range(3))
        pa = T2 / self.dt ** 2 + 2j * self.w * T1 / self.dt - self.w ** 2 * T0
        dt_ = T1 / self.dt + 1j * self.w * T0
        Rs = np.where(R == 0, 1.0, R)
        return -(np.exp(-1j * self.k * R) / (4.0 * math.pi)) * (pa / (C0 * Rs) + dt_ / (Rs * Rs))

    def gram(self) -> complex:
        m, b = self.m, self.basis
        return complex(basis_origin(b, m, 1) / self.dt + 1j * self.w * basis_origin(b, m, 0))

    def dt_factor(self, R):
        """(DT)(tau) exp(-j k R): the temporal factor of G^H (times 1/(4 pi R))."""
        tau = self.m - R / (C0 * self.dt)
        b = self.basis
        return np.exp(-1j * self.k * R) * (basis_T(b, tau, 1) / self.dt + 1j * self.w * basis_T(b, tau, 0))


class FDMFIEKernel:
    """g'(R) of the frequency-domain MFIE at f (Gram factor 1)."""

    def __init__(self, f: float):
        self.k = 2.0 * math.pi * f / C0

    def gp(self, R):
        Rs = np.where(R == 0, 1.0, R)
        return -(np.exp(-1j * self.k * R) / (4.0 * math.pi)) * (1j * self.k / Rs + 1.0 / (Rs * Rs))

    def gram(self) -> complex:
        return 1.0 + 0j


def tri_pair_curl(surf: Surface, ta, tb, kernels, chunk: int = 8192):
    """M [P, K, 3, 3] = int_Ta int_Tb g'(R) (r - v_i) . (n_a x (Rhat x (r' - v'_j)))
    for triangle pairs (ta[p], tb[p]); zero where ta == tb."""
    ta = np.asarray(ta, dtype=np.int64)
    tb = np.asarray(tb, dtype=np.int64)
    P, K = len(ta), len(kernels)
    out = np.zeros((P, K, 3, 3), dtype=np.complex128)
    bary, w = radon7()
    for s in range(0, P, chunk):
        a, b = ta[s:s + chunk], tb[s:s + chunk]
        va, vb = surf.tv[a], surf.tv[b]
        ra, rb = points(va, bary), points(vb, bary)           # [p,7,3]
        diff = ra[:, :, None, :] - rb[:, None, :, :]           # [p,q,r,3]
        R = np.sqrt(np.einsum("pqrx,pqrx->pqr", diff, diff))
        Rs = np.where(R == 0, 1.0, R)
        Rh = diff / Rs[..., None]
        na = surf.normal[a]                                    # [p,3]
        Da = ra[:, :, None, :] - va[:, None, :, :]             # [p,q,i,3]
        Db = rb[:, :, None, :] - vb[:, None, :, :]             # [p,r,j,3]
        nR = np.einsum("pqrx,px->pqr", Rh, na)
        DaR = np.einsum("pqix,pqrx->pqri", Da, Rh)
        nDb = np.einsum("prjx,px->prj", Db, na)
        W = (w[:, None] * w[None, :])[None] * (surf.area[a] * surf.area[b])[:, None, None]
        live = (a != b)[:, None, None] & (R > 0)
        for ki, kn in enumerate(kernels):
            Wg = np.where(live, W * kn.gp(R), 0.0)
            t1 = np.einsum("pqr,pqri,prj->pij", Wg, DaR, nDb, optimize=True)
            t2 = np.einsum("pqr,pqix,prjx->pij", Wg * nR, Da, Db, optimize=True)
            out[s:s + chunk, ki] = t1 - t2
    return out


def _halves(surf: Surface):
    ar = surf.area[surf.t]
    return surf.t, surf.loc, surf.s * surf.length[:, None] / (2.0 * ar)


def gram_pairs(surf: Surface, rows, cols) -> np.ndarray:
    """<S_k, S_k'> for basis pairs (exact: 7-point rule, integrand degree 2)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    t, loc, ca = _halves(surf)
    bary, w = radon7()
    out = np.zeros(len(rows))
    for h in range(2):
        for g in range(2):
            same = t[rows, h] == t[cols, g]
            if not np.any(same):
                continue
            r, c = rows[same], cols[same]
            tri = t[r, h]
            rp = points(surf.tv[tri], bary)                    # [p,7,3]
            va = surf.xyz[surf.free[r, h]]
            vb = surf.xyz[surf.free[c, g]]
            Sa = ca[r, h][:, None, None] * (rp - va[:, None, :])
            Sb = ca[c, g][:, None, None] * (rp - vb[:, None, :])
            out[same] += np.einsum("pqx,pqx,q->p", Sa, Sb, w) * surf.area[tri]
    return out


def assemble_pairs(surf: Surface, rows, cols, kernels) -> np.ndarray:
    """MFIE entries Z^H[kernel][p] for basis pairs (rows[p], cols[p])."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    t, loc, ca = _halves(surf)
    nt = len(surf.tri)
    keys = [t[rows, h] * nt + t[cols, g] for h in range(2) for g in range(2)]
    uniq, inv = np.unique(np.concatenate(keys), return_inverse=True)
    M = tri_pair_curl(surf, uniq // nt, uniq % nt, kernels)
    inv = inv.reshape(4, -1)
    out = np.zeros((len(kernels), len(rows)), dtype=np.complex128)
    i4 = 0
    for h in range(2):
        for g in range(2):
            Mij = M[inv[i4], :, loc[rows, h], loc[cols, g]].T  # [K, P]
            i4 += 1
            out -= (ca[rows, h] * ca[cols, g])[None] * Mij
    G = gram_pairs(surf, rows, cols)
    out += 0.5 * np.array([kn.gram() for kn in kernels])[:, None] * G[None]
    return out


def assemble_dense(surf: Surface, kernels) -> np.ndarray:
    """Dense MFIE matrices [K, ns, ns] (small meshes only)."""
    ns = surf.ns
    rr, cc = np.meshgrid(np.arange(ns), np.arange(ns), indexing="ij")
    return assemble_pairs(surf, rr.ravel(), cc.ravel(), kernels).reshape(len(kernels), ns, ns)


def combine(ZE: np.ndarray, ZH: np.ndarray, alpha: float) -> np.ndarray:
    """CFIE matrices alpha Z^E + (1 - alpha) eta Z^H."""
    return alpha * ZE + (1.0 - alpha) * ETA0 * ZH


def excitation_h(surf: Surface, nt: int, dt: float, khat, phat, sigma, td, fc) -> np.ndarray:
    """V^H [nt, B, ns]: <S_k, n x (khat x D E~_inc)> at t = l dt (eta times
    the MFIE's tested n x D H~_inc), 7-point rule on T+ and T-."""
    khat = np.atleast_2d(np.asarray(khat, dtype=np.float64))
    phat = np.atleast_2d(np.asarray(phat, dtype=np.float64))
    w = 2.0 * math.pi * fc
    bary, wq = radon7()
    V = np.zeros((nt, len(khat), surf.ns), dtype=np.complex128)
    t = np.arange(1, nt + 1) * dt
    for h in range(2):
        tri = surf.t[:, h]
        rp = points(surf.tv[tri], bary)
        vfree = surf.xyz[surf.free[:, h]]
        coef = surf.s[:, h] * surf.length / (2.0 * surf.area[tri])
        n = surf.normal[tri]                                   # [ns,3]
        for b in range(len(khat)):
            hv = np.cross(khat[b], phat[b])                    # khat x phat
            nh = np.cross(n, hv)                               # n x (khat x phat), per triangle
            rk = rp @ khat[b] / C0
            proj = np.einsum("kpx,kx->kp", rp - vfree[:, None, :], nh)
            tau = t[:, None, None] - rk[None] - td
            g = np.exp(-tau ** 2 / (2.0 * sigma ** 2))
            dg = -(tau / sigma ** 2) * g
            val = (dg + 1j * w * g) * np.exp(-1j * w * (rk + td))[None]
            V[:, b, :] += np.einsum("lkp,kp,p->lk", val, proj, wq) * (coef * surf.area[tri])[None]
    return V


# ---- AIM pieces -------------------------------------------------------------

def _lagrange4_d(u):
    """Cubic Lagrange basis on nodes 0..3 and its derivative at u: ([...,4], [...,4])."""
    val, der = [], []
    for j in range(4):
        others = [i for i in range(4) if i != j]
        den = np.prod([j - i for i in others])
        v = np.ones_like(u)
        for i in others:
            v = v * (u - i)
        d = np.zeros_like(u)
        for skip in others:
            p = np.ones_like(u)
            for i in others:
                if i != skip:
                    p = p * (u - i)
            d = d + p
        val.append(v / den)
        der.append(d / den)
    return np.stack(val, -1), np.stack(der, -1)


def projection_curl(surf: Surface, grid, i0) -> np.ndarray:
    """H [ns, 3, 64]: H[k, :, n] = int (S_k x n) x grad l_n dS (local node
    n = jx + 4 (jy + 4 jz)), 6 x 6 collapsed Gauss rule (exact, degree 9)."""
    bary, w = collapsed_gauss(6)
    H = np.zeros((surf.ns, 3, 64))
    for h in range(2):
        tri = surf.t[:, h]
        rp = points(surf.tv[tri], bary)                        # [ns,P,3]
        u = (rp - grid.x0) / grid.h - i0[:, None, :]
        (lx, dx), (ly, dy), (lz, dz) = (_lagrange4_d(u[..., a]) for a in range(3))
        # grad l_n, n = jx + 4 (jy + 4 jz): [ns,P,64,3]
        gx = np.einsum("kpa,kpb,kpc->kpcba", dx, ly, lz).reshape(surf.ns, -1, 64)
        gy = np.einsum("kpa,kpb,kpc->kpcba", lx, dy, lz).reshape(surf.ns, -1, 64)
        gz = np.einsum("kpa,kpb,kpc->kpcba", lx, ly, dz).reshape(surf.ns, -1, 64)
        grad = np.stack([gx, gy, gz], -1) / grid.h
        ca = surf.s[:, h] * surf.length / (2.0 * surf.area[tri])
        S = ca[:, None, None] * (rp - surf.xyz[surf.free[:, h]][:, None, :])
        Sn = np.cross(S, surf.normal[tri][:, None, :])          # [ns,P,3]
        v = np.cross(Sn[:, :, None, :], grad)                  # [ns,P,64,3]
        H += np.einsum("kp,kpnc->kcn", w[None, :] * surf.area[tri][:, None], v)
    return H


def green_table_h(grid, ms, dt: float, fc: float, basis=None) -> np.ndarray:
    """G^H_m on the |offset| table [len(ms), Nz, Ny, Nx] (G^H[0] = 0)."""
    nx, ny, nz = grid.n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    R = grid.h * np.sqrt((i * i + j * j + k * k).astype(np.float64))
    Rs = np.where(R == 0, 1.0, R)
    out = np.zeros((len(ms),) + R.shape, dtype=np.complex128)
    for a, m in enumerate(ms):
        out[a] = np.where(R == 0, 0.0, MFIEKernel(m, dt, fc, basis).dt_factor(R) / (4.0 * math.pi * Rs))
    return out


def cfie_pairs(surf: Surface, rows, cols, ms, dt: float, fc: float, alpha: float, basis=None) -> np.ndarray:
    """Exact CFIE entries [len(ms), P] of basis pairs for envelope steps ms."""
    from . import kernels, zfill
    ZE = zfill.assemble_pairs(surf, rows, cols, [kernels.EnvelopeKernel(m, dt, fc, basis) for m in ms])
    if alpha == 1.0:
        return ZE
    ZH = assemble_pairs(surf, rows, cols, [MFIEKernel(m, dt, fc, basis) for m in ms])
    return combine(ZE, ZH, alpha)
