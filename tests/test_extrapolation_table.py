"""The initial-guess extrapolation table of the GMRES kernels (host-side
check of the constant the kernels read): row p must give the polynomial of
degree p - 1 through the last p solutions evaluated one step ahead, i.e. be
exact on every polynomial of degree < p and equal (-1)^(i+1) C(p, i)."""
import math
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1408_7060_amd", "csrc", "krylov.inc.hip")


def _table():
    src = open(SRC).read()
    kmax = int(re.search(r"constexpr int kMaxGuess = (\d+);", src).group(1))
    body = re.search(r"kExtrap\[kMaxGuess\]\[kMaxGuess\] = \{(.*?)\};", src, re.S).group(1)
    rows = [[float(v) for v in r.split(",")] for r in re.findall(r"\{([^{}]*)\}", body)]
    return kmax, np.array(rows)


def test_rows_are_exact_on_polynomials():
    kmax, a = _table()
    assert a.shape == (kmax, kmax)
    rng = np.random.default_rng(3)
    for p in range(1, kmax + 1):
        c = a[p - 1]
        assert np.all(c[p:] == 0)
        for deg in range(p):
            q = np.polynomial.Polynomial(rng.standard_normal(deg + 1))
            pred = sum(c[i - 1] * q(10.0 - i) for i in range(1, p + 1))
            assert abs(pred - q(10.0)) <= 1e-9 * max(1.0, abs(q(10.0)))
        # and not exact one degree higher (the order is exactly p)
        q = np.polynomial.Polynomial([0] * p + [1.0])
        assert abs(sum(c[i - 1] * q(10.0 - i) for i in range(1, p + 1)) - q(10.0)) > 0.5


def test_rows_are_signed_binomials():
    kmax, a = _table()
    for p in range(1, kmax + 1):
        for i in range(1, p + 1):
            assert a[p - 1, i - 1] == (-1) ** (i + 1) * math.comb(p, i)
