"""CPPIF temporal basis pins (closed forms)."""
import numpy as np
import pytest

from oracle import cppif


def _taus():
    return np.linspace(-3.0, 3.0, 601) + 0.0037


def test_partition_of_unity_and_reproduction():
    tau = _taus()
    ls = np.arange(-8, 9)
    for p in range(4):
        s = sum((l ** p) * cppif.T(tau - l) for l in ls)
        assert np.allclose(s, tau ** p, atol=1e-11 * (1 + np.abs(tau) ** p))


def test_derivative_sums_vanish():
    tau = _taus()
    ls = np.arange(-8, 9)
    for d in (1, 2, 3):
        s = sum(cppif.T(tau - l, d) for l in ls)
        assert np.allclose(s, 0.0, atol=1e-10)


def test_interpolatory_and_support():
    n = np.arange(-3, 6).astype(float)
    assert np.allclose(cppif.T(n), (n == 0).astype(float))
    assert np.all(cppif.T(np.array([-1.0, -1.5, 3.01, 4.0])) == 0)
    assert abs(cppif.T(np.array([3.0]))[0]) < 1e-14     # left piece at tau = Q


def test_continuity_at_breakpoints():
    for i in range(-1, 4):
        a = cppif.T(np.array([i - 1e-9]))[0]
        b = cppif.T(np.array([i + 1e-9]))[0]
        assert abs(a - b) < 1e-7


def test_derivatives_match_finite_differences():
    tau = np.array([-0.7, -0.2, 0.3, 0.9, 1.4, 1.8, 2.2, 2.7])
    h = 1e-5
    for d in range(3):
        fd = (cppif.T(tau + h, d) - cppif.T(tau - h, d)) / (2 * h)
        assert np.allclose(fd, cppif.T(tau, d + 1), rtol=1e-6, atol=1e-6)


def test_piece_zero_closed_form():
    tau = np.array([-0.9, -0.5, -0.1, 0.0])
    assert np.allclose(cppif.T(tau), (tau + 1) * (tau + 2) * (tau + 3) / 6)
    tau = np.array([2.1, 2.5, 3.0])
    assert np.allclose(cppif.T(tau), -(tau - 3) * (tau - 2) * (tau - 1) / 6)
