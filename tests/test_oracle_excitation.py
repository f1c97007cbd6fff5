"""Excitation pins: the closed-form envelope equals the analytic-signal
envelope of eq. (1); V_l applies d/dt + j w_c (checked by differences)."""
import math

import numpy as np
import pytest

from oracle import excitation, physics as ph
from oracle.quadrature import points, radon7
from oracle_cases import sphere


def test_envelope_equals_analytic_signal_of_eq1():
    fc, sigma = 300e6, 8e-9
    td = 8 * sigma
    khat, phat = np.array([0, 0, -1.0]), np.array([1.0, 0, 0])
    r = np.array([0.1, -0.2, 0.3])
    n, T = 1 << 16, 400e-9
    t = np.arange(n) * (T / n)
    tau = t - r @ khat / ph.C0 - td
    real = np.exp(-tau ** 2 / (2 * sigma ** 2)) * np.cos(2 * math.pi * fc * tau)   # eq. (1)
    spec = np.fft.fft(real)
    h = np.zeros(n)
    h[0] = 1
    h[1:n // 2] = 2
    h[n // 2] = 1
    analytic = np.fft.ifft(spec * h)
    env = analytic * np.exp(-1j * 2 * math.pi * fc * t)
    ref = excitation.envelope_field(r[None, :], t[:, None], khat, phat, sigma, td, fc)[:, 0, 0]
    assert np.max(np.abs(env - ref)) < 1e-9
    # and x(t) = Re{x~ exp(j w_c t)} reproduces the real pulse
    assert np.max(np.abs(np.real(ref * np.exp(1j * 2 * math.pi * fc * t)) - real)) < 1e-12


def test_excitation_is_time_derivative_plus_jw_of_envelope():
    s = sphere()
    fc, sigma = 300e6, 8e-9
    td, dt, nt = 8 * sigma, 3e-9, 40
    khat, phat = np.array([0.3, -0.4, -0.866]), np.array([1.0, 0.0, 0.0])
    phat = phat - (phat @ khat) * khat / (khat @ khat)
    khat = khat / np.linalg.norm(khat)
    phat = phat / np.linalg.norm(phat)
    V = excitation.excitation(s, nt, dt, khat, phat, sigma, td, fc)[:, 0, :]
    bary, w = radon7()
    h = 1e-13
    ref = np.zeros_like(V)
    for half in range(2):
        tri = s.t[:, half]
        rp = points(s.tv[tri], bary)
        S = (s.s[:, half] * s.length / 2.0)[:, None, None] * (rp - s.xyz[s.free[:, half]][:, None, :])
        for l in range(nt):
            t = (l + 1) * dt
            e0 = excitation.envelope_field(rp, t, khat, phat, sigma, td, fc)
            ep = excitation.envelope_field(rp, t + h, khat, phat, sigma, td, fc)
            em = excitation.envelope_field(rp, t - h, khat, phat, sigma, td, fc)
            de = (ep - em) / (2 * h) + 1j * 2 * math.pi * fc * e0
            ref[l] += np.einsum("kpx,kpx,p->k", S, de, w)
    assert np.linalg.norm(V - ref) / np.linalg.norm(ref) < 1e-5
