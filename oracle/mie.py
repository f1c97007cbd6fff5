"""Mie series of a PEC sphere, frequency-domain RCS and the dB-error norm
(oracle; test infrastructure only).

The paper measures accuracy against the Mie series (Sec. 5, ref. [18]) with
the thresholded dB-error norm of eq. (2) (Sec. 2.4): sigma^TH =
max(10 log10 sigma, TH) - TH, TH = peak - 80 dB, and the error is the
sin(theta)-weighted L2 ratio over the sphere of directions.

Mie series (textbook form, Bohren & Huffman 1983 with a perfectly
conducting sphere): a_n = psi_n'(x)/xi_n'(x), b_n = psi_n(x)/xi_n(x),
S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n),
S2 = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n),
with the incident wave along z' = k_hat, polarised along x' = p_hat; the
scattered far field is proportional to cos(phi') S2 theta' - sin(phi') S1
phi', and sigma = (4 pi / k^2) |.|^2.  Pins: Rayleigh backscatter 9 (ka)^4
pi a^2, optical backscatter pi a^2, optical theorem.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import spherical_jn, spherical_yn

from .physics import C0, MU0


def coefficients(x: float):
    nmax = int(x + 4.0 * x ** (1.0 / 3.0) + 2.0)
    n = np.arange(1, nmax + 1)
    jn, jnp = spherical_jn(n, x), spherical_jn(n, x, derivative=True)
    yn, ynp = spherical_yn(n, x), spherical_yn(n, x, derivative=True)
    psi, dpsi = x * jn, jn + x * jnp
    hn, hnp = jn + 1j * yn, jnp + 1j * ynp
    xi, dxi = x * hn, hn + x * hnp
    return n, dpsi / dxi, psi / xi


def amplitudes(x: float, theta: np.ndarray):
    n, a, b = coefficients(x)
    mu = np.cos(theta)
    pi_prev = np.zeros_like(mu)
    pi_cur = np.ones_like(mu)
    S1 = np.zeros(mu.shape, dtype=np.complex128)
    S2 = np.zeros_like(S1)
    for i, nn in enumerate(n):
        if nn > 1:
            pi_new = ((2 * nn - 1) / (nn - 1)) * mu * pi_cur - (nn / (nn - 1)) * pi_prev
            pi_prev, pi_cur = pi_cur, pi_new
        tau = nn * mu * pi_cur - (nn + 1) * pi_prev
        c = (2 * nn + 1) / (nn * (nn + 1))
        S1 += c * (a[i] * pi_cur + b[i] * tau)
        S2 += c * (a[i] * tau + b[i] * pi_cur)
    return S1, S2


def backscatter(ka: float, radius: float) -> float:
    """Monostatic RCS [m^2]."""
    n, a, b = coefficients(ka)
    k = ka / radius
    s = np.sum((-1.0) ** n * (2 * n + 1) * (a - b))
    return float(abs(s) ** 2 * math.pi / k ** 2)


def cross_sections(ka: float, radius: float):
    """(extinction, scattering) cross sections [m^2]; equal for a PEC sphere."""
    n, a, b = coefficients(ka)
    k = ka / radius
    ext = 2 * math.pi / k ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    sca = 2 * math.pi / k ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return float(ext), float(sca)


def far_field_vector(ka: float, radius: float, khat, phat, dirs: np.ndarray) -> np.ndarray:
    """Scattered far-field vectors (arbitrary common phase) with
    |E|^2 * 4 pi = sigma, directions dirs [P,3]."""
    khat, phat = np.asarray(khat, float), np.asarray(phat, float)
    yhat = np.cross(khat, phat)
    cz, cx, cy = dirs @ khat, dirs @ phat, dirs @ yhat
    theta = np.arccos(np.clip(cz, -1, 1))
    phi = np.arctan2(cy, cx)
    S1, S2 = amplitudes(ka, theta)
    k = ka / radius
    th_hat = (np.cos(theta) * np.cos(phi))[:, None] * phat + (np.cos(theta) * np.sin(phi))[:, None] * yhat \
        - np.sin(theta)[:, None] * khat
    ph_hat = -np.sin(phi)[:, None] * phat + np.cos(phi)[:, None] * yhat
    E = (np.cos(phi) * S2)[:, None] * th_hat - (np.sin(phi) * S1)[:, None] * ph_hat
    return E / k


def sphere_grid(nth: int = 91, nph: int = 180):
    th = np.linspace(0.0, math.pi, nth)
    ph = np.linspace(0.0, 2 * math.pi, nph, endpoint=False)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    th_hat = np.stack([np.cos(TH) * np.cos(PH), np.cos(TH) * np.sin(PH), -np.sin(TH)], -1)
    return TH, PH, d, th_hat


def rcs_theta_mie(ka, radius, khat, phat, d, th_hat):
    E = far_field_vector(ka, radius, khat, phat, d.reshape(-1, 3)).reshape(d.shape)
    return 4.0 * math.pi * np.abs(np.einsum("...x,...x->...", E, th_hat)) ** 2


def rcs_theta_current(surf, I: np.ndarray, f: float, d, th_hat):
    """sigma_theta-theta from a frequency-domain RWG current (unit incident E),
    E_far = -j w mu/(4 pi) [I - dd] int J exp(j k d.r') dS' (7-point rule)."""
    from .quadrature import points, radon7
    w = 2 * math.pi * f
    k = w / C0
    bary, wq = radon7()
    dirs = d.reshape(-1, 3)
    acc = np.zeros((len(dirs), 3), dtype=np.complex128)
    for h in range(2):
        tri = surf.t[:, h]
        rp = points(surf.tv[tri], bary)
        coef = surf.s[:, h] * surf.length / 2.0
        S = coef[:, None, None] * (rp - surf.xyz[surf.free[:, h]][:, None, :])
        ph = np.exp(1j * k * np.einsum("kpx,dx->dkp", rp, dirs))
        acc += np.einsum("dkp,p,kpx,k->dx", ph, wq, S, I)
    E = -1j * w * MU0 / (4 * math.pi) * acc
    Eth = np.einsum("dx,dx->d", E, th_hat.reshape(-1, 3))
    return (4 * math.pi * np.abs(Eth) ** 2).reshape(d.shape[:-1])


def rcs_envelope(u: np.ndarray, dt: float, df: float, sigma: float, pol: np.ndarray) -> np.ndarray:
    """sigma_pol(f_c + df) [D] from the far-field envelope samples u [nt, D, 3]
    of one incidence (u[l] at t = (l+1) dt, the march's sample times) driven
    by the Gaussian pulse of eq. (1) with width sigma.  The time-harmonic
    far field at f = f_c + df is the envelope's Fourier transform at df
    divided by the incident envelope's at the origin,
        U(df) = dt sum_l u_l exp(-j 2 pi df (l+1) dt),
        G(df) = sigma sqrt(2 pi) exp(-2 pi^2 sigma^2 df^2)
    (the transform of g = exp(-t^2/2 sigma^2); its delay and carrier phase
    drop out of |.|), so sigma_pol = 4 pi |pol . U(df)|^2 / G(df)^2 as for a
    unit incident field (Sec. 2.4)."""
    nt = u.shape[0]
    ph = np.exp(-2j * math.pi * df * (np.arange(nt) + 1.0) * dt)
    U = dt * np.einsum("l,ldx->dx", ph, u)
    G = sigma * math.sqrt(2.0 * math.pi) * math.exp(-2.0 * math.pi ** 2 * sigma ** 2 * df ** 2)
    return 4.0 * math.pi * np.abs(np.einsum("dx,dx->d", U, pol)) ** 2 / G ** 2


def db_error(sig: np.ndarray, sig_ref: np.ndarray, theta: np.ndarray, floor_db: float = 80.0) -> float:
    """Eq. (2): thresholded dB-error norm over the (theta, phi) grid."""
    TH = 10 * np.log10(np.max(sig_ref)) - floor_db
    a = np.maximum(10 * np.log10(np.maximum(sig, 1e-300)), TH) - TH
    b = np.maximum(10 * np.log10(np.maximum(sig_ref, 1e-300)), TH) - TH
    w = np.sin(theta)
    return float(np.sum((a - b) ** 2 * w) / np.sum(b ** 2 * w))
