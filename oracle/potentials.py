"""Closed-form static potentials of a flat triangle (oracle; test
infrastructure only).

For an observation point r and a flat triangle T' (the singular part of the
impedance integrals, Sec. 5.1 "order of singularity extraction"; reading:
closed forms of Wilton et al. 1984 / Graglia 1993):

    I0(r) = int_T' 1/|r - r'| dS'
    I1(r) = int_T' (r' - rho)/|r - r'| dS'

where rho is the projection of r on the plane of T'.  With d the signed
height of r over the plane and, for each edge i (endpoints a -> b in
counter-clockwise order about the normal n): unit edge direction l_i, in-plane
outward edge normal u_i = l_i x n, l+ = (b - rho).l_i, l- = (a - rho).l_i,
P0 = (a - rho).u_i, R0^2 = P0^2 + d^2, R+- = |r - b|, |r - a|:

    I0 = sum_i [ P0 ln((R+ + l+)/(R- + l-))
                 - |d| (atan(P0 l+/(R0^2 + |d| R+)) - atan(P0 l-/(R0^2 + |d| R-))) ]
    I1 = 1/2 sum_i u_i [ R0^2 ln((R+ + l+)/(R- + l-)) + l+ R+ - l- R- ]

Pinned against brute-force Duffy-transformed Gauss quadrature
(tests/test_oracle_quadrature.py).
"""
from __future__ import annotations

import numpy as np


def _log_ratio(rp, lp, rm, lm):
    """ln((R+ + l+)/(R- + l-)) evaluated without cancellation: when both l are
    negative use the equal ratio (R- - l-)/(R+ - l+)."""
    neg = (lp < 0) & (lm < 0)
    num = np.where(neg, rm - lm, rp + lp)
    den = np.where(neg, rp - lp, rm + lm)
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.log(num / den)
    return np.where((num > 0) & (den > 0), out, 0.0)


def triangle_potentials(r: np.ndarray, verts: np.ndarray):
    """r [...,3], verts [...,3,3] (broadcastable).  Returns (I0 [...], I1 [...,3])."""
    r = np.asarray(r, dtype=np.float64)
    v = np.asarray(verts, dtype=np.float64)
    n = np.cross(v[..., 1, :] - v[..., 0, :], v[..., 2, :] - v[..., 0, :])
    n = n / np.linalg.norm(n, axis=-1, keepdims=True)
    d = np.einsum("...x,...x->...", r - v[..., 0, :], n)
    rho = r - d[..., None] * n
    ad = np.abs(d)
    I0 = np.zeros(np.broadcast_shapes(r.shape[:-1], v.shape[:-2]))
    I1 = np.zeros(I0.shape + (3,))
    for i in range(3):
        a = v[..., i, :]
        b = v[..., (i + 1) % 3, :]
        e = b - a
        le = e / np.linalg.norm(e, axis=-1, keepdims=True)
        u = np.cross(le, n)
        lp = np.einsum("...x,...x->...", b - rho, le)
        lm = np.einsum("...x,...x->...", a - rho, le)
        p0 = np.einsum("...x,...x->...", a - rho, u)
        r02 = p0 * p0 + d * d
        rp = np.sqrt(r02 + lp * lp)
        rm = np.sqrt(r02 + lm * lm)
        lr = _log_ratio(rp, lp, rm, lm)
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = np.where(r02 > 0, np.arctan2(p0 * lp, r02 + ad * rp), 0.0)
            t2 = np.where(r02 > 0, np.arctan2(p0 * lm, r02 + ad * rm), 0.0)
        I0 = I0 + p0 * lr - ad * (t1 - t2)
        I1 = I1 + 0.5 * u * (r02 * lr + lp * rp - lm * rm)[..., None]
    return I0, I1
