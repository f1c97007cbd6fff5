"""Scattered far-field envelopes and the energy objective (oracle; test
infrastructure only).

The paper post-processes the solution into scattered fields and radar cross
sections (Sec. 2.4).  Reading (normalisation not printed): the far field of
J = Re{J~ exp(j w_c t)} is E = -dA_perp/dt with
A(r,t) ~ mu/(4 pi r) int J(r', t - r/c + r_hat.r'/c) dS'.  Dropping 1/r,
exp(-j k_c r) and the delay r/c, the envelope at t = l dt in direction d is

    u_d(l dt) = -(mu/4 pi) [I - d d^T] sum_{k', l'} I_l'[k'] int S_k'(r')
                  [T'(tau')/dt + j w_c T(tau')] exp(j k_c d.r') dS',
    tau' = l - l' + d.r'/(c dt)

(7-point rule on each triangle).  Objective J = sum_l sum_d |u_d(l dt)|^2.
Written as u = F I with F a block-Toeplitz operator in time; F^H is its
adjoint.  Parity unpinned beyond the dot-product identity <F a, b> =
<a, F^H b> and the narrow-band limit against the frequency-domain far field.
"""
from __future__ import annotations

import math

import numpy as np

from . import cppif
from .kernels import basis_T
from .geometry import Surface
from .physics import C0, MU0
from .quadrature import points, radon7


class FarField:
    def __init__(self, surf: Surface, dirs: np.ndarray, dt: float, fc: float, basis=None):
        dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
        self.dirs, self.dt, self.ns = dirs, dt, surf.ns
        w = 2.0 * math.pi * fc
        k = w / C0
        bary, wq = radon7()
        # tap range: tau' = m + d.r'/(c dt) must lie in (-1, Q]
        rad = np.abs(surf.xyz).max() * math.sqrt(3.0)
        s_max = rad / (C0 * dt)
        lo, hi = (-1.0, cppif.Q) if basis is None else (-basis.M, basis.M)
        self.m_lo = int(math.floor(lo - s_max))
        self.m_hi = int(math.ceil(hi + s_max))
        taps = np.arange(self.m_lo, self.m_hi + 1)
        self.taps = taps
        F = np.zeros((len(taps), len(dirs), 3, surf.ns), dtype=np.complex128)
        proj = np.eye(3)[None] - dirs[:, :, None] * dirs[:, None, :]     # [D,3,3]
        for h in range(2):
            tri = surf.t[:, h]
            rp = points(surf.tv[tri], bary)                               # [ns,7,3]
            coef = surf.s[:, h] * surf.length / (2.0 * surf.area[tri]) * surf.area[tri]
            S = coef[:, None, None] * (rp - surf.xyz[surf.free[:, h]][:, None, :])   # [ns,7,3]
            for d in range(len(dirs)):
                dr = rp @ dirs[d]                                         # [ns,7]
                ph = np.exp(1j * k * dr)
                for ti, m in enumerate(taps):
                    tau = m + dr / (C0 * dt)
                    f = basis_T(basis, tau, 1) / dt + 1j * w * basis_T(basis, tau, 0)
                    vec = np.einsum("kp,kp,p,kpx->kx", f, ph, wq, S)      # [ns,3]
                    F[ti, d] += -(MU0 / (4.0 * math.pi)) * (proj[d] @ vec.T)
        self.F = F                                     # [taps, D, 3, ns]

    def apply(self, I: np.ndarray) -> np.ndarray:
        """u [nt, B, D, 3] from I [nt, B, ns]: u_l = sum_m F_m I_{l-m}."""
        nt = I.shape[0]
        u = np.zeros((nt, I.shape[1], len(self.dirs), 3), dtype=np.complex128)
        for ti, m in enumerate(self.taps):
            for l in range(nt):
                j = l - m
                if 0 <= j < nt:
                    u[l] += np.einsum("dxk,bk->bdx", self.F[ti], I[j])
        return u

    def adjoint(self, U: np.ndarray) -> np.ndarray:
        """F^H applied to U [nt, B, D, 3] -> [nt, B, ns]."""
        nt = U.shape[0]
        out = np.zeros((nt, U.shape[1], self.ns), dtype=np.complex128)
        for ti, m in enumerate(self.taps):
            for l in range(nt):
                j = l - m
                if 0 <= j < nt:
                    out[j] += np.einsum("dxk,bdx->bk", self.F[ti].conj(), U[l])
        return out


def energy(u: np.ndarray) -> float:
    return float(np.sum(np.abs(u) ** 2))
