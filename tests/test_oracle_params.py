"""Parameter rules of the oracle against values the paper prints."""
import math
import os

import numpy as np
import pytest
from scipy.special import erfc

from oracle import physics as ph

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    return np.loadtxt(os.path.join(GOLD, name), comments="#")


def test_table1_band_edge_is_300mhz():
    # Table I / Sec. 5.1: f_c + 3/(2 pi sigma) = 300 MHz for every pulse
    for chi_approx, fc, num, den in _rows("table1_pulses.txt"):
        sigma = num / (den * math.pi) * 1e-6
        fbw = ph.band_from_sigma(sigma)
        assert fc * 1e6 + fbw == pytest.approx(300e6, rel=1e-12)
        chi = ph.chi(fc * 1e6 - fbw, fc * 1e6 + fbw)
        assert chi == pytest.approx(300e6 / fbw, rel=1e-12)
        assert round(chi) == chi_approx
        assert ph.sigma_from_band(fbw) == pytest.approx(sigma, rel=1e-12)


def test_chi_examples():
    for fmin, fmax, chi in _rows("chi_examples.txt"):
        assert ph.chi(fmin, fmax) == pytest.approx(chi, rel=1e-12)


def test_step_counts():
    for ts, dt, nt in _rows("timestep_counts.txt"):
        assert ph.nt_from(ts, dt) == int(nt)


def test_energy_outside_three_sigma():
    # Sec. 2.2: less than ~2.2e-3 % of the pulse energy lies outside t_d +- 3 sigma.
    # Energy of exp(-t^2/2s^2) cos(...) ~ exp(-t^2/s^2): outside fraction erfc(3).
    from scipy.integrate import quad
    sigma, fc = 1.0, 40.0          # narrow band: cos^2 averages to 1/2
    e = lambda t: (np.exp(-t ** 2 / (2 * sigma ** 2)) * np.cos(2 * np.pi * fc * t)) ** 2
    inside = quad(e, -3 * sigma, 3 * sigma, limit=2000)[0]
    total = quad(e, -12 * sigma, 12 * sigma, limit=4000)[0]
    frac_t = 1.0 - inside / total
    assert frac_t == pytest.approx(erfc(3.0), rel=1e-3)   # carrier ripple at the cut
    # frequency side: |spectrum|^2 ~ exp(-(2 pi f sigma)^2) about f_c
    s = lambda f: np.exp(-(2 * np.pi * f * sigma) ** 2)
    fb = 3.0 / (2 * np.pi * sigma)
    frac_f = 1.0 - quad(s, -fb, fb)[0] / quad(s, -10 * fb, 10 * fb)[0]
    assert frac_f == pytest.approx(erfc(3.0), rel=1e-6)
    assert max(frac_t, frac_f) < 2.2e-5 * 1.005


def test_history_depth_rule():
    # N_g = floor(R_max/(c dt) + l_max) and the mid-interval time-step rule
    for ng in (5, 9, 24, 32):
        dt = ph.dt_from_ng(2.0, ng)
        assert ph.ng_from(2.0, dt) == ng
    # the missile run of Sec. 6 prints dt = 2 ns and N_g = 21 with a 3 m class
    # object; the rule is monotone in R_max
    assert ph.ng_from(1.0, 2e-9) < ph.ng_from(5.0, 2e-9)
