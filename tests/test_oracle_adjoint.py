"""Adjoint pins: far-field dot-product identity and central finite
differences of the energy objective."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, farfield, march
from oracle_cases import dense_z, l2_band_params, sphere

FC = 300e6


def _setup(nt=10):
    s = sphere()
    dt, ng = l2_band_params(frac=0.01)
    Z = dense_z(dt, FC, ng)
    dirs = W.unit_vectors(0, 4, 3)
    F = farfield.FarField(s, dirs, dt, FC)
    V = W.complex_normal(2, (nt, 1, s.ns))
    return s, Z, F, V


def test_farfield_dot_product():
    s, Z, F, V = _setup()
    a = W.complex_normal(3, V.shape)
    b = W.complex_normal(4, (V.shape[0], 1, 3, 3))
    lhs = np.vdot(b, F.apply(a))
    rhs = np.vdot(F.adjoint(b), a)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gradient_matches_finite_differences():
    s, Z, F, V = _setup()

    def J(v):
        return farfield.energy(F.apply(march.march_dense(Z, v)))

    I = march.march_dense(Z, V)
    lam = adjoint.adjoint_march(Z, F.adjoint(F.apply(I)))
    grad = 2 * lam
    eps = 1e-4 * np.abs(V).max()
    for (l, k) in [(0, 5), (3, 100), (7, 311), (9, 479)]:
        e = np.zeros_like(V)
        e[l, 0, k] = eps
        d_re = (J(V + e) - J(V - e)) / (2 * eps)
        d_im = (J(V + 1j * e) - J(V - 1j * e)) / (2 * eps)
        g = grad[l, 0, k]
        scale = np.abs(grad).max()
        assert abs(d_re - g.real) < 1e-6 * scale
        assert abs(d_im - g.imag) < 1e-6 * scale
