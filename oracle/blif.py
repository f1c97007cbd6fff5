"""Band-limited interpolatory temporal basis (BLIF) with causal
extrapolation (oracle; test infrastructure only).

The paper's broad-band ET runs use a BLIF of half-width M = 3 (Sec. 3,
Sec. 3.1.2, Table III) instead of the CPPIF; its non-causal part is removed
by extrapolating the M - 1 future samples from N_samp past ones, with
N_omega = 2 N_samp, by the scheme of its ref. [15] (not available).
Reading, written out here:

* T(tau) = sinc(tau) W(tau) on -M < tau <= M (zero outside; the right end
  belongs to the support, as the CPPIF's breakpoints belong to their left
  piece), with W the approximate prolate window of Knab,
      W = sinh(a sqrt(u)) / (sqrt(u) sinh a),  u = 1 - (tau / M)^2,
      a = pi M (1 - 2 beta),  beta = f_bw dt
  (the envelope's half band over the sampling rate).  T is interpolatory:
  T(n) = delta_n0.  W is evaluated as its power series in u,
  sum_k a^(2k+1) u^k / ((2k+1)! sinh a), entire in tau, so T, T', T'', T'''
  follow from the product rule with closed-form sinc derivatives.
* Extrapolation: I_{l+k} ~ sum_{p < N_samp} a_{kp} I_{l-p}, k = 1..M-1,
  with a_k the least-squares fit of exp(j w k dt) by exp(-j w p dt) at
  N_omega frequencies w spread evenly over [-2 pi f_bw, 2 pi f_bw]
  (the set is symmetric, so the fit is taken over real a).
* The march keeps eq. (4)'s form with the folded matrices
  Z~_p = Z_p + sum_k a_{kp} Z_{-k} (p < N_samp) and Z~_m = Z_m (m >= N_samp),
  m = 0..N_g, N_g = floor(R_max / (c dt) + M); Z_{-k} are the envelope
  kernels at negative m (tau = -k - R / (c dt) > -M).  Folding is linear,
  so the Green tables and the exact near-zone entries fold the same way.

Pins (tests/test_oracle_blif.py): T(n) = delta_n0; the derivatives against
finite differences; the window series against the sinh formula; shifted
BLIFs reproduce exp(j Omega tau) for |Omega| <= 2 pi beta to the window's
bound; the extrapolation exact on the fit frequencies when N_omega =
N_samp; the folded matrices of a band-limited current reproduce the
unfolded sum.
"""
from __future__ import annotations

import math

import numpy as np

_NSER = 24   # a^(2k+1)/(2k+1)! < 1e-17 of the sum beyond this for a <= 3 pi


class Blif:
    """The BLIF of half-width M for oversampling beta = f_bw dt."""

    def __init__(self, M: int = 3, beta: float = 0.2):
        if not 0.0 < beta < 0.5:
            raise ValueError("beta must lie in (0, 1/2)")
        self.M = int(M)
        self.beta = float(beta)
        self.a = math.pi * self.M * (1.0 - 2.0 * self.beta)
        sha = math.sinh(self.a)
        self._c = [self.a ** (2 * k + 1) / math.factorial(2 * k + 1) / sha for k in range(_NSER)]

    def _w(self, u, d):
        """d-th derivative of the window series in u (Horner)."""
        out = np.zeros_like(u)
        for k in range(_NSER - 1, d - 1, -1):
            out = out * u + self._c[k] * math.perm(k, d)
        return out

    @staticmethod
    def _sinc(t, d):
        """d-th derivative (in t) of sin(pi t) / (pi t), d <= 3."""
        t = np.asarray(t, dtype=np.float64)
        out = np.empty_like(t)
        small = np.abs(t) < 0.25
        ts = t[small]
        acc = np.zeros_like(ts)
        for k in range(16):
            e = 2 * k
            if e >= d:
                acc = acc + (-1) ** k * math.pi ** e / math.factorial(e + 1) * math.perm(e, d) * ts ** (e - d)
        out[small] = acc
        x = math.pi * t[~small]
        s, c = np.sin(x), np.cos(x)
        if d == 0:
            v = s / x
        elif d == 1:
            v = (x * c - s) / x ** 2
        elif d == 2:
            v = (-x * x * s - 2 * x * c + 2 * s) / x ** 3
        else:
            v = (-x ** 3 * c + 3 * x * x * s + 6 * x * c - 6 * s) / x ** 4
        out[~small] = v * math.pi ** d
        return out

    def T(self, tau, deriv: int = 0):
        """T^(deriv)(tau), elementwise; zero outside -M < tau <= M."""
        tau = np.asarray(tau, dtype=np.float64)
        M = self.M
        inside = (tau > -M) & (tau <= M)
        t = np.where(inside, tau, 0.0)
        u = 1.0 - t * t / (M * M)
        u1, u2 = -2.0 * t / (M * M), -2.0 / (M * M)
        w = [self._w(u, k) for k in range(deriv + 1)] + [None] * (3 - deriv)
        W = [w[0]]
        if deriv >= 1:
            W.append(w[1] * u1)
        if deriv >= 2:
            W.append(w[2] * u1 ** 2 + w[1] * u2)
        if deriv >= 3:
            W.append(w[3] * u1 ** 3 + 3.0 * w[2] * u1 * u2)
        S = [self._sinc(t, k) for k in range(deriv + 1)]
        out = sum(math.comb(deriv, k) * S[k] * W[deriv - k] for k in range(deriv + 1))
        return np.where(inside, out, 0.0)

    def window_closed_form(self, tau):
        """W by its sinh formula (pins only; |tau| < M)."""
        u = 1.0 - np.asarray(tau, dtype=np.float64) ** 2 / self.M ** 2
        r = np.sqrt(u)
        return np.sinh(self.a * r) / (r * math.sinh(self.a))


def extrapolation(beta: float, M: int, nsamp: int, nomega: int) -> np.ndarray:
    """a [M-1, nsamp]: I_{l+k} ~ sum_p a[k-1, p] I_{l-p}, fitted at nomega
    frequencies w dt = 2 pi beta x, x evenly spaced on [-1, 1]."""
    wdt = 2.0 * math.pi * beta * np.linspace(-1.0, 1.0, nomega)
    A = np.exp(-1j * np.outer(wdt, np.arange(nsamp)))
    Ar = np.concatenate([A.real, A.imag])
    out = np.zeros((M - 1, nsamp))
    for k in range(1, M):
        b = np.exp(1j * wdt * k)
        out[k - 1] = np.linalg.lstsq(Ar, np.concatenate([b.real, b.imag]), rcond=None)[0]
    return out


def fold(Z: dict, a: np.ndarray, ng: int) -> np.ndarray:
    """Folded matrices [ng+1, ...] from Z[m] for m = -(M-1)..ng (a dict)."""
    out = np.stack([np.array(Z[m], copy=True) for m in range(ng + 1)])
    for k in range(1, a.shape[0] + 1):
        for p in range(a.shape[1]):
            out[p] = out[p] + a[k - 1, p] * Z[-k]
    return out
