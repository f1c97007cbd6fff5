"""Causal piecewise-polynomial interpolatory function (CPPIF) of order Q
(oracle; test infrastructure only).

The temporal basis T of eq. (3) (Sec. 3; CPPIF of order Q = 3 for the
envelope-tracking runs, Sec. 3.1 and Table III).  With samples at integer
times, the interpolant on (n-1, n] is the degree-Q Lagrange polynomial
through samples n, n-1, ..., n-Q.  Written as a basis function of the
normalised time tau = t/dt - l', on the piece tau in (i-1, i], i = 0..Q:

    T(tau) = prod_{k=0, k != i}^{Q} (tau - i + k) / (k - i)

and T = 0 outside (-1, Q].  A breakpoint tau = i belongs to the left piece
(index ceil(tau)).  Derivatives are the derivatives of the piece polynomial.

Pins: partition of unity, reproduction of polynomials of degree <= Q,
interpolation T(n) = delta_n0, continuity at the breakpoints, derivatives
against finite differences (tests/test_oracle_basis.py).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import Polynomial

Q = 3


def piece_poly(i: int, q: int = Q) -> Polynomial:
    """Polynomial of piece i (tau in (i-1, i]) in the variable tau."""
    p = Polynomial([1.0])
    for k in range(q + 1):
        if k != i:
            p = p * Polynomial([float(k - i), 1.0]) / float(k - i)
    return p


def _pieces(q: int = Q):
    return [piece_poly(i, q) for i in range(q + 1)]


_CACHE: dict[int, list[list[Polynomial]]] = {}


def _table(q: int):
    if q not in _CACHE:
        base = _pieces(q)
        tab = [base]
        for _ in range(4):
            tab.append([p.deriv() for p in tab[-1]])
        _CACHE[q] = tab
    return _CACHE[q]


def T(tau, deriv: int = 0, q: int = Q):
    """T^(deriv)(tau), elementwise, left-piece convention at breakpoints."""
    tau = np.asarray(tau, dtype=np.float64)
    out = np.zeros_like(tau)
    idx = np.ceil(tau)
    tab = _table(q)[deriv]
    for i in range(q + 1):
        sel = (idx == i) & (tau > -1.0) & (tau <= q)
        if np.any(sel):
            out[sel] = tab[i](tau[sel])
    return out


def T_piece(i: int, tau, deriv: int = 0, q: int = Q):
    """Piece i's polynomial (or derivative) evaluated at tau, no support test.
    Zero for i outside 0..Q."""
    tau = np.asarray(tau, dtype=np.float64)
    if i < 0 or i > q:
        return np.zeros_like(tau)
    return _table(q)[deriv][i](tau)
