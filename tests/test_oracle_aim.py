"""AIM pins: projection moments (exact polynomial integrals), FFT
convolution against the literal double sum, far-part symmetry, the
pre-correction identity and the AIM accuracy on separated pairs."""
import math
from itertools import product

import numpy as np
import pytest

import workloads as W
from oracle import aim, kernels, physics as ph, zfill
from oracle_cases import dense_z, l2_band_params, sphere

FC = 300e6


def _aim():
    s = sphere()
    dt, ng = l2_band_params()
    return aim.AIM(s, 16, 0.3 * ph.C0 / FC, dt, FC, ng), dt, ng


_CACHE = {}


def get_aim():
    if "a" not in _CACHE:
        _CACHE["a"] = _aim()
    return _CACHE["a"]


def _poly_mul(p, q):
    out = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0.0) + ca * cb
    return out


def _linear(vals):
    """Linear function with vertex values vals -> barycentric polynomial."""
    return {(1, 0, 0): vals[0], (0, 1, 0): vals[1], (0, 0, 1): vals[2]}


def _integrate(p, area):
    return sum(c * 2 * area * math.factorial(a) * math.factorial(b) * math.factorial(d)
               / math.factorial(a + b + d + 2) for (a, b, d), c in p.items())


def test_projection_matches_moments_exactly():
    A, _, _ = get_aim()
    s, g = A.surf, A.grid
    for k in (0, 17, 123, 250, 479):
        for (a, b, c) in product(range(4), repeat=3):
            for comp in range(4):
                exact = 0.0
                for half in range(2):
                    t = s.t[k, half]
                    V = s.tv[t]
                    loc = (V - g.x0) / g.h - A.i0[k]            # local stencil coords of vertices
                    p = {(0, 0, 0): 1.0}
                    for axis, power in ((0, a), (1, b), (2, c)):
                        for _ in range(power):
                            p = _poly_mul(p, _linear(loc[:, axis]))
                    if comp < 3:
                        coef = s.s[k, half] * s.length[k] / (2 * s.area[t])
                        lin = _linear((V[:, comp] - s.xyz[s.free[k, half], comp]) * coef)
                        p = _poly_mul(p, lin)
                    else:
                        p = {e: v * s.s[k, half] * s.length[k] / s.area[t] for e, v in p.items()}
                    exact += _integrate(p, s.area[t])
                j = np.arange(64)
                jx, jy, jz = j % 4, (j // 4) % 4, j // 16
                moment = np.sum(A.L[k, comp] * jx ** a * jy ** b * jz ** c)
                scale = np.abs(A.L[k, comp]).sum() * 27
                assert abs(moment - exact) <= 1e-12 * scale


def test_fft_convolution_equals_direct_sum():
    A, dt, ng = get_aim()
    x = W.complex_normal(1, A.surf.ns)
    for m in range(ng + 1):
        y1 = A.far_matvec(m, x)
        y2 = A.far_matvec(m, x, direct=True)
        assert np.linalg.norm(y1 - y2) <= 1e-13 * np.linalg.norm(y2)


def test_circulant_embedding_small_grid():
    rng = np.random.default_rng(3)
    tab = rng.standard_normal((3, 4, 5)) + 1j * rng.standard_normal((3, 4, 5))
    q = rng.standard_normal((3, 4, 5)) + 1j * rng.standard_normal((3, 4, 5))
    circ = aim.circulant(tab)
    qq = np.zeros((6, 8, 10), complex)
    qq[:3, :4, :5] = q
    p = np.fft.ifftn(np.fft.fftn(circ) * np.fft.fftn(qq))[:3, :4, :5]
    ref = np.zeros_like(q)
    for z, y, x in product(range(3), range(4), range(5)):
        for z2, y2, x2 in product(range(3), range(4), range(5)):
            ref[z, y, x] += tab[abs(z - z2), abs(y - y2), abs(x - x2)] * q[z2, y2, x2]
    assert np.max(np.abs(p - ref)) < 1e-13 * np.max(np.abs(ref))


def test_far_part_symmetric_and_pairs_match_dense():
    A, dt, ng = get_aim()
    for m in (0, 2):
        Zf = A.far_dense(m)
        assert np.linalg.norm(Zf - Zf.T) <= 1e-14 * np.linalg.norm(Zf)
        r, c = A.rows[::37], A.cols[::37]
        assert np.max(np.abs(A.far_pairs(m, r, c) - Zf[r, c])) <= 1e-13 * np.abs(Zf).max()


def test_precorrection_restores_exact_near_entries():
    A, dt, ng = get_aim()
    Z = dense_z(dt, FC, ng)
    s = A.surf

    def exact(rows, cols, ms):
        return zfill.assemble_pairs(s, rows, cols, [kernels.EnvelopeKernel(m, dt, FC) for m in ms])

    vals = A.near_values(exact)
    for m in range(A.mn + 1):
        zf = A.far_pairs(m, A.rows, A.cols)
        got = vals[m] + zf
        ref = Z[m][A.rows, A.cols]
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.abs(Z[m]).max()
    # beyond M_n both parts vanish on every near pair
    if A.mn < ng:
        assert np.abs(Z[A.mn + 1][A.rows, A.cols]).max() == 0.0
        assert np.abs(A.far_pairs(A.mn + 1, A.rows, A.cols)).max() == 0.0


def test_aim_far_accuracy_on_separated_pairs():
    A, dt, ng = get_aim()
    Z = dense_z(dt, FC, ng)
    c = A.surf.c
    sep = np.linalg.norm(c[:, None] - c[None], axis=2) > A.d_near
    Zf = A.far_dense(0)
    err = np.linalg.norm((Zf - Z[0])[sep]) / np.linalg.norm(Z[0][sep])
    assert err < 0.05


@pytest.mark.parametrize("level,radius,lam_frac,fc", [(2, 0.5, 0.3, 300e6), (3, 1.0, 0.3, 300e6)])
def test_near_pairs_equal_brute_force_distance_scan(level, radius, lam_frac, fc):
    """The near-zone pattern (stage (iv)): every ordered pair (k, k') with
    |c_k - c_k'| <= d_near, the basis itself included, by the full O(N_s^2)
    distance matrix of the basis centres (no spatial tree), row-major."""
    xyz, tri = W.icosphere(level, radius)
    s = sphere(level, radius)
    d_near = lam_frac * ph.C0 / fc
    rows, cols = aim.near_pairs(s, d_near)
    c = s.c
    D = np.sqrt(((c[:, None, :] - c[None, :, :]) ** 2).sum(axis=-1))
    br, bc = np.nonzero(D <= d_near)          # row-major order, columns ascending
    assert np.array_equal(rows, br) and np.array_equal(cols, bc)
    assert np.all(D[rows, rows] == 0) and len(rows) == int((D <= d_near).sum())
    # the test is inclusive: a radius equal to one pair's distance keeps that pair
    k, k2 = 0, int(np.argsort(D[0])[5])
    r2, c2 = aim.near_pairs(s, float(np.linalg.norm(c[k] - c[k2])))
    assert np.any((r2 == k) & (c2 == k2)) and np.any((r2 == k2) & (c2 == k))


def test_sampled_row_helpers_equal_the_full_operator():
    """The sampled-row forms used at full size (a k-space sum of several
    terms before one inverse transform, interpolated at chosen rows; the
    pre-corrected near values of the chosen rows' pairs) equal the full
    operator's rows: the sum of far_matvec over the terms, and near_values
    restricted to those rows."""
    A, dt, ng = get_aim()
    s = A.surf
    rows = np.array([0, 5, 77, 200, 479])
    xs = [W.complex_normal(60 + i, s.ns) for i in range(3)]
    ms = [0, 2, ng]
    ref = sum(A.far_matvec(m, x) for m, x in zip(ms, xs))[rows]
    got = A.far_sum_rows([(m, A.spectra(x)) for m, x in zip(ms, xs)], rows)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()

    def exact(r, c, mm):
        return zfill.assemble_pairs(s, r, c, [kernels.EnvelopeKernel(m, dt, FC) for m in mm])

    full = A.near_values(exact)
    sel, vals = A.near_values_rows(exact, rows)
    np.testing.assert_allclose(vals, full[:, sel], rtol=0, atol=1e-13 * np.abs(full).max())
    for m in range(A.mn + 1):
        y = A.near_matvec(full[m], xs[0])[rows]
        assert np.abs(A.near_rows(sel, vals[m], xs[0], rows) - y).max() <= 1e-13 * np.abs(y).max()
