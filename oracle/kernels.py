"""Envelope Green-function kernels of the differentiated EFIE (oracle; test
infrastructure only).

Reading (the entries themselves are deferred by the paper to its refs. [5],
[7]; Sec. 3 eq. (3)-(4)): with J(r,t) = Re{J~(r,t) exp(j w_c t)}, the
retarded potentials of J give the envelope kernel delta(t - R/c) exp(-j k_c R)
/ (4 pi R) and d/dt -> d/dt + j w_c.  Differentiating the EFIE in time, using
the Lorenz gauge, Galerkin testing in space with the RWG functions and point
testing at t = l dt, the interaction of a basis sample l' with a test at l
depends on m = l - l' through tau = m - R/(c dt):

    K_A(m, R)   = (mu / 4 pi R)  exp(-j k_c R) P_A(tau),
                  P_A = T''/dt^2 + 2 j w_c T'/dt - w_c^2 T
    K_phi(m, R) = (1 / 4 pi eps R) exp(-j k_c R) T(tau)

Both are written f(R)/R.  For singularity extraction on touching triangle
pairs, f(0) and f'(0) come from the CPPIF piece that holds tau for R -> 0+
(piece m).  The frequency-domain EFIE kernel at f uses f(R) = exp(-j k R)
for both parts.
"""
from __future__ import annotations

import math

import numpy as np

from . import cppif
from .physics import C0, EPS0, MU0


def basis_T(basis, tau, d):
    """T^(d)(tau) of the temporal basis: the CPPIF (basis None) or a BLIF."""
    return cppif.T(tau, d) if basis is None else basis.T(tau, d)


def basis_origin(basis, m, d):
    """T^(d) at tau = m approached from below (R -> 0+): the CPPIF's piece m,
    or the BLIF's smooth value (its support's right end included)."""
    if basis is None:
        return float(cppif.T_piece(m, m, d))
    return float(basis.T(np.array([float(m)]), d)[0])


class EnvelopeKernel:
    """Kernel of Z_m for one m; A-part scale mu/(4 pi), phi-part 1/(4 pi eps).
    basis: None for the CPPIF, or an ``oracle.blif.Blif``."""

    def __init__(self, m: int, dt: float, fc: float, basis=None):
        self.m, self.dt, self.basis = m, dt, basis
        self.w = 2.0 * math.pi * fc
        self.k = self.w / C0
        self.scale_a = MU0 / (4.0 * math.pi)
        self.scale_phi = 1.0 / (4.0 * math.pi * EPS0)

    def _pa(self, T0, T1, T2):
        return T2 / self.dt ** 2 + 2j * self.w * T1 / self.dt - self.w ** 2 * T0

    def f(self, R):
        tau = self.m - R / (C0 * self.dt)
        ph = np.exp(-1j * self.k * R)
        T0, T1, T2 = (basis_T(self.basis, tau, d) for d in range(3))
        return ph * self._pa(T0, T1, T2), ph * T0

    def f0(self):
        T0, T1, T2 = (basis_origin(self.basis, self.m, d) for d in range(3))
        return self._pa(T0, T1, T2), complex(T0)

    def df0(self):
        """d f / dR at R = 0+ (piece m)."""
        cdt = C0 * self.dt
        T = [basis_origin(self.basis, self.m, d) for d in range(4)]
        pa = self._pa(T[0], T[1], T[2])
        dpa = self._pa(T[1], T[2], T[3])          # d/dtau of P_A
        return (-1j * self.k * pa - dpa / cdt,
                -1j * self.k * T[0] - T[1] / cdt)


class FDKernel:
    """Frequency-domain EFIE kernel exp(-jkR)/(4 pi R) at frequency f:
    Z = j w mu <S, g S'> - j/(w eps) <div S, g div' S'>."""

    def __init__(self, f: float):
        self.w = 2.0 * math.pi * f
        self.k = self.w / C0
        self.scale_a = 1j * self.w * MU0 / (4.0 * math.pi)
        self.scale_phi = -1j / (self.w * EPS0) / (4.0 * math.pi)

    def f(self, R):
        e = np.exp(-1j * self.k * R)
        return e, e

    def f0(self):
        return 1.0 + 0j, 1.0 + 0j

    def df0(self):
        return -1j * self.k, -1j * self.k
