"""Quadrature and closed-form potential pins."""
import numpy as np
import pytest

from oracle import potentials, quadrature


def _monomials(deg):
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                yield a, b, c


@pytest.mark.parametrize("rule,deg", [("radon7", 5), ("cg6", 10)])
def test_rules_exact_on_monomials(rule, deg):
    bary, w = quadrature.radon7() if rule == "radon7" else quadrature.collapsed_gauss(6)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    for a, b, c in _monomials(deg):
        q = np.sum(w * bary[:, 0] ** a * bary[:, 1] ** b * bary[:, 2] ** c)
        # weights are normalised to area 1 -> the formula's 2A = 2
        assert q == pytest.approx(quadrature.simplex_monomial(a, b, c), rel=1e-13, abs=1e-16)


def test_radon7_not_exact_at_degree_6():
    bary, w = quadrature.radon7()
    q = np.sum(w * bary[:, 0] ** 6)
    assert abs(q - quadrature.simplex_monomial(6, 0, 0)) > 1e-6


def _brute(r, V, n=300):
    nrm = np.cross(V[1] - V[0], V[2] - V[0])
    nrm /= np.linalg.norm(nrm)
    d = np.dot(r - V[0], nrm)
    rho = r - d * nrm
    bary, w = quadrature.collapsed_gauss(n)
    I0, I1 = 0.0, np.zeros(3)
    for i in range(3):
        sub = np.array([rho, V[i], V[(i + 1) % 3]])
        a = 0.5 * np.dot(np.cross(sub[1] - sub[0], sub[2] - sub[0]), nrm)
        P = bary @ sub
        R = np.linalg.norm(r - P, axis=1)
        I0 += a * np.sum(w / R)
        I1 += a * np.sum(w[:, None] * (P - rho) / R[:, None], axis=0)
    return I0, I1


def test_closed_form_potentials_against_duffy_quadrature():
    rng = np.random.default_rng(7)
    for trial in range(6):
        V = rng.standard_normal((3, 3))
        nrm = np.cross(V[1] - V[0], V[2] - V[0])
        nrm /= np.linalg.norm(nrm)
        pts = [(V[0] + V[1] + V[2]) / 3,                    # in-plane, inside
               0.1 * V[0] + 0.6 * V[1] + 0.3 * V[2],         # in-plane, inside
               1.4 * V[0] - 0.4 * V[1],                      # in-plane, outside
               (V[0] + V[1] + V[2]) / 3 + 0.3 * nrm,         # above
               1.3 * V[1] - 0.3 * V[2] - 0.05 * nrm]         # below, outside
        for r in pts:
            I0, I1 = potentials.triangle_potentials(r, V)
            b0, b1 = _brute(r, V)
            assert I0 == pytest.approx(b0, rel=1e-12)
            assert np.allclose(I1, b1, rtol=1e-11, atol=1e-12 * abs(b0))
