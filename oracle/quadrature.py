"""Triangle quadrature (oracle; test infrastructure only).

Sec. 5.1 only says the cubature rules are identical across the methods; the
reading fixed here:

* ``radon7``: the 7-point degree-5 rule (Radon 1948) for the excitation, the
  regular impedance integrals and the far field.
* ``collapsed_gauss``: Gauss-Legendre product rule on the collapsed square
  (lambda1 = u, lambda2 = (1-u) v, Jacobian 2A(1-u)); with n points per
  direction it integrates polynomials of total degree <= 2n-2 exactly.  Used
  with n = 6 (exact to degree 10) for the moment-matching projection.
* ``simplex_monomial``: closed form of the integral of
  l1^a l2^b l3^c over a triangle, 2A a! b! c! / (a+b+c+2)!  (pins only).

Points are barycentric (l1, l2, l3); weights are normalised to sum to 1, so
an integral is area * sum(w f).
"""
from __future__ import annotations

import math

import numpy as np


def radon7():
    s15 = math.sqrt(15.0)
    a1 = (6.0 - s15) / 21.0
    a2 = (6.0 + s15) / 21.0
    w0 = 9.0 / 40.0
    w1 = (155.0 - s15) / 1200.0
    w2 = (155.0 + s15) / 1200.0
    bary = [(1 / 3, 1 / 3, 1 / 3),
            (a1, a1, 1 - 2 * a1), (a1, 1 - 2 * a1, a1), (1 - 2 * a1, a1, a1),
            (a2, a2, 1 - 2 * a2), (a2, 1 - 2 * a2, a2), (1 - 2 * a2, a2, a2)]
    w = [w0, w1, w1, w1, w2, w2, w2]
    return np.array(bary), np.array(w)


def collapsed_gauss(n: int):
    x, wx = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (x + 1.0)
    wu = 0.5 * wx
    U, V = np.meshgrid(u, u, indexing="ij")
    WU, WV = np.meshgrid(wu, wu, indexing="ij")
    l1 = U
    l2 = (1.0 - U) * V
    l3 = 1.0 - l1 - l2
    w = 2.0 * (1.0 - U) * WU * WV
    return np.stack([l1.ravel(), l2.ravel(), l3.ravel()], axis=1), w.ravel()


def simplex_monomial(a: int, b: int, c: int, area: float = 1.0) -> float:
    return 2.0 * area * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 2)


def points(verts: np.ndarray, bary: np.ndarray) -> np.ndarray:
    """Physical points: verts [...,3(vertex),3(xyz)], bary [P,3] -> [...,P,3]."""
    return np.einsum("pv,...vx->...px", bary, verts)
