"""Incident envelope and excitation vectors (oracle; test infrastructure only).

The incident field of eq. (1) (Sec. 2.2) is E = p g(tau) cos(w_c tau) with
g = exp(-tau^2 / 2 sigma^2), tau = t - r.k/c - t_d.  Its complex envelope
(reading: x(t) = Re{x~(t) exp(j w_c t)}, no extra factor) is

    E~(r,t) = p g(tau) exp(-j w_c (r.k/c + t_d))

and the differentiated EFIE is driven by (d/dt + j w_c) E~ =
p [g'(tau) + j w_c g(tau)] exp(-j w_c (r.k/c + t_d)), g' = -(tau/sigma^2) g.
The excitation vector at step l (testing at t = l dt, eq. (4)):

    V_l[k] = int S_k(r) . (d/dt + j w_c) E~(r, l dt) dS

integrated with the 7-point rule on T+ and T-.  The closed form of the
envelope is pinned against the analytic signal of eq. (1) computed by FFT
(tests/test_oracle_excitation.py).
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Surface
from .physics import C0
from .quadrature import points, radon7


def envelope_field(r, t, khat, phat, sigma, td, fc):
    """E~(r,t) [...,3] for points r [...,3] and times t (broadcast)."""
    w = 2.0 * math.pi * fc
    rk = np.einsum("...x,x->...", r, khat) / C0
    tau = t - rk - td
    g = np.exp(-tau ** 2 / (2.0 * sigma ** 2))
    return (g * np.exp(-1j * w * (rk + td)))[..., None] * phat


def excitation(surf: Surface, nt: int, dt: float, khat, phat, sigma, td, fc) -> np.ndarray:
    """V [nt, B, ns] for B incidences (khat, phat [B,3]); V[l-1] tests at l dt."""
    khat = np.atleast_2d(np.asarray(khat, dtype=np.float64))
    phat = np.atleast_2d(np.asarray(phat, dtype=np.float64))
    w = 2.0 * math.pi * fc
    bary, wq = radon7()
    V = np.zeros((nt, len(khat), surf.ns), dtype=np.complex128)
    t = np.arange(1, nt + 1) * dt
    for h in range(2):
        tri = surf.t[:, h]
        vt = surf.tv[tri]                                    # [ns,3,3]
        rp = points(vt, bary)                                # [ns,7,3]
        vfree = surf.xyz[surf.free[:, h]]
        coef = surf.s[:, h] * surf.length / (2.0 * surf.area[tri])
        for b in range(len(khat)):
            rk = rp @ khat[b] / C0                           # [ns,7]
            proj = np.einsum("kpx,x->kp", rp - vfree[:, None, :], phat[b])
            tau = t[:, None, None] - rk[None] - td           # [nt,ns,7]
            g = np.exp(-tau ** 2 / (2.0 * sigma ** 2))
            dg = -(tau / sigma ** 2) * g
            val = (dg + 1j * w * g) * np.exp(-1j * w * (rk + td))[None]
            V[:, b, :] += np.einsum("lkp,kp,p->lk", val, proj, wq) * (coef * surf.area[tri])[None]
    return V
