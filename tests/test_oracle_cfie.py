"""Pins of the combined-field operators (the MFIE and the CFIE with alpha =
0.5 of the paper's spheres, Sec. 2.1 and Sec. 5.1):

* the frequency-domain MFIE and CFIE solutions of the level-2 sphere give
  the Mie series' RCS (a sign error in the curl term, a wrong normal or a
  dropped Gram term fails it);
* the EFIE and MFIE of the a = 0.5 m sphere are near-singular at its first
  interior resonance (k a = 2.744, 262 MHz, shifted to about 265 MHz by
  the inscribed mesh) and the CFIE is not;
* the envelope MFIE matrices sum to j w_c times the FD MFIE (partition of
  unity of the CPPIF and of its derivative);
* the curl projection H reproduces the tested n x curl A of polynomial
  potentials of degree <= 3 per axis exactly (curls taken by hand);
* the AIM's MFIE far part approximates the exact entries on separated
  pairs and converges with the grid; its seven channels agree through
  the literal double sum, the FFT convolution with the k-space history
  sum and the stencil sums of the pre-correction;
* the CPPIF march of the sphere at +-10 % is unstable with the EFIE
  (companion spectral radius > 1) and stable with the CFIE.
"""
import math

import numpy as np
import pytest

from oracle import aim, excitation, kernels, mfie, mie, physics as ph, zfill
from oracle.quadrature import collapsed_gauss, points
from oracle_cases import dense_h, dense_z, l2_band_params, sphere

FC = 300e6


def _fd(f):
    s = sphere()
    ZE = zfill.assemble_dense(s, [kernels.FDKernel(f)])[0]
    ZH = mfie.assemble_dense(s, [mfie.FDMFIEKernel(f)])[0]
    return s, ZE, ZH


@pytest.mark.parametrize("f", [200e6, 300e6])
def test_fd_mfie_and_cfie_against_mie(f):
    s, ZE, ZH = _fd(f)
    w = 2 * math.pi * f
    inc = ([[0, 0, -1.0]], [[1.0, 0, 0]], 1e30, 0.0, f)
    VE = excitation.excitation(s, 1, 1.0, *inc)[0, 0] / (1j * w)
    VH = mfie.excitation_h(s, 1, 1.0, *inc)[0, 0] / (1j * w)
    TH, PH, d, th = mie.sphere_grid(46, 90)
    sm = mie.rcs_theta_mie(w / ph.C0 * 0.5, 0.5, [0, 0, -1.0], [1.0, 0, 0], d, th)
    for Z, V in ((ph.ETA0 * ZH, VH), (mfie.combine(ZE, ZH, 0.5), 0.5 * VE + 0.5 * VH)):
        I = np.linalg.solve(Z, V)
        sc = mie.rcs_theta_current(s, I, f, d, th)
        assert mie.db_error(sc, sm, TH) < 1e-4
        assert sc[0, 0] == pytest.approx(sm[0, 0], rel=0.2)
    # the EFIE and MFIE currents of the same field agree to the discretisation
    IE = np.linalg.solve(ZE, VE)
    IH = np.linalg.solve(ph.ETA0 * ZH, VH)
    assert np.linalg.norm(IE - IH) < 0.1 * np.linalg.norm(IE)


def test_cfie_removes_the_interior_resonance():
    ratio = {}
    for f in (255e6, 265e6, 275e6):
        s, ZE, ZH = _fd(f)
        for name, Z in (("E", ZE), ("H", ZH), ("C", mfie.combine(ZE, ZH, 0.5))):
            sv = np.linalg.svd(Z, compute_uv=False)
            ratio[name, f] = sv[-1] / sv[0]
    for name in ("E", "H"):
        assert ratio[name, 265e6] < 0.1 * min(ratio[name, 255e6], ratio[name, 275e6])
    c = [ratio["C", f] for f in (255e6, 265e6, 275e6)]
    assert min(c) > 0.25 and max(c) < 1.1 * min(c)


def test_envelope_mfie_sums_to_the_frequency_domain_mfie():
    dt, ng = l2_band_params()
    Z = dense_h(dt, FC, ng)
    w = 2 * math.pi * FC
    ref = 1j * w * mfie.assemble_dense(sphere(), [mfie.FDMFIEKernel(FC)])[0]
    assert np.abs(Z.sum(0) - ref).max() <= 1e-13 * np.abs(ref).max()
    g = sum(mfie.MFIEKernel(m, dt, FC).gram() for m in range(ng + 1))
    assert abs(g - 1j * w) <= 1e-12 * w


def test_curl_projection_exact_on_polynomials():
    s = sphere()
    grid = aim.Grid(s.xyz, 16)
    i0 = aim.stencil_corner(grid, s.c)
    nodes = aim.stencil_nodes(grid, i0)
    H = mfie.projection_curl(s, grid, i0)
    n = np.arange(grid.nnodes)
    nx, ny = grid.n[0], grid.n[1]
    r = grid.node_xyz(np.stack([n % nx, (n // nx) % ny, n // (nx * ny)], 1))

    def A(p):
        x, y, z = p[..., 0], p[..., 1], p[..., 2]
        return np.stack([y * y * z, x ** 3 + z, x * y * z * z], -1)

    def curlA(p):
        x, y, z = p[..., 0], p[..., 1], p[..., 2]
        return np.stack([x * z * z - 1.0, y * y - y * z * z, 3 * x * x - 2 * y * z], -1)

    An = A(r)                                                   # [N,3]
    got = np.einsum("kcn,knc->k", H, An[nodes])
    bary, w = collapsed_gauss(8)
    ref = np.zeros(s.ns)
    for h in range(2):
        tri = s.t[:, h]
        rp = points(s.tv[tri], bary)
        S = (s.s[:, h] * s.length / (2 * s.area[tri]))[:, None, None] * (rp - s.xyz[s.free[:, h]][:, None, :])
        ncurl = np.cross(s.normal[tri][:, None, :], curlA(rp))
        ref += np.einsum("kpx,kpx,p->k", S, ncurl, w) * s.area[tri]
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


_CACHE = {}


def _cfie_aim():
    if "a" not in _CACHE:
        s = sphere()
        dt, ng = l2_band_params()
        A = aim.AIM(s, 16, 0.3 * ph.C0 / FC, dt, FC, ng, alpha=0.5)
        _CACHE["a"] = A, dt, ng
    return _CACHE["a"]


def test_mfie_far_part_converges_with_the_grid():
    """The AIM's MFIE far part (alpha = 0) against the exact entries on pairs
    0.3-0.6 m apart: a few per cent on the 16^3 grid, and the error falls
    with the grid spacing (h^3 or faster for the curl of a cubic
    interpolant) on the 24^3 grid."""
    s = sphere()
    dt, ng = l2_band_params()
    ZH = ph.ETA0 * dense_h(dt, FC, ng)
    c = s.c
    D = np.linalg.norm(c[:, None] - c[None], axis=2)
    r, cc = np.nonzero((D > 0.3) & (D < 0.6))
    sel = np.random.default_rng(0).choice(len(r), 3000, replace=False)
    r, cc = r[sel], cc[sel]
    err = {}
    for n in (16, 24):
        A = aim.AIM(s, n, 0.3 * ph.C0 / FC, dt, FC, ng, alpha=0.0)
        err[n] = max(np.linalg.norm(A.far_pairs(m, r, cc) - ZH[m][r, cc]) / np.linalg.norm(ZH[m][r, cc])
                     for m in (0, 1))
    assert err[16] < 0.03
    assert err[24] < err[16] / 3


def test_cfie_far_part_paths_agree_and_vanish_beyond_the_near_depth():
    """The CFIE's seven channels through the three far-part paths: the
    literal node double sum, the circulant FFT convolution (one inverse
    transform per channel after the k-space sum over m, as the march's
    history sum) and the stencil double sum of the pre-correction.  Beyond
    M_n the exact entries and the far part both vanish on every near pair
    (the MFIE's temporal support equals the EFIE's)."""
    A, dt, ng = _cfie_aim()
    rng = np.random.default_rng(3)
    xs = [rng.standard_normal(A.surf.ns) + 1j * rng.standard_normal(A.surf.ns) for _ in range(2)]
    for m in (0, 2):
        d = A.far_matvec(m, xs[0], direct=True)
        assert np.abs(A.far_matvec(m, xs[0]) - d).max() <= 1e-12 * np.abs(d).max()
    rows = np.arange(0, A.surf.ns, 7)
    ref = A.far_matvec(1, xs[0]) + A.far_matvec(2, xs[1])
    got = A.far_sum_rows([(1, A.spectra(xs[0])), (2, A.spectra(xs[1]))], rows)
    assert np.abs(got - ref[rows]).max() <= 1e-12 * np.abs(ref).max()
    Zf = A.far_dense(0)
    r, cc = A.rows[::29], A.cols[::29]
    assert np.abs(A.far_pairs(0, r, cc) - Zf[r, cc]).max() <= 1e-13 * np.abs(Zf).max()
    assert np.abs(Zf @ xs[0] - A.far_matvec(0, xs[0])).max() <= 1e-12 * np.abs(Zf @ xs[0]).max()
    if A.mn < ng:
        m = A.mn + 1
        assert np.abs(mfie.cfie_pairs(A.surf, A.rows, A.cols, [m], dt, FC, 0.5)).max() == 0.0
        assert np.abs(A.far_pairs(m, A.rows, A.cols)).max() == 0.0


def _spectral_radius(Z):
    ng, ns = len(Z) - 1, Z.shape[1]
    Z0i = np.linalg.inv(Z[0])
    C = np.zeros((ns * ng, ns * ng), dtype=np.complex128)
    for m in range(1, ng + 1):
        C[:ns, (m - 1) * ns:m * ns] = -Z0i @ Z[m]
    C[ns:, :-ns] = np.eye(ns * (ng - 1))
    return float(np.abs(np.linalg.eigvals(C)).max())


def test_cfie_cppif_march_is_stable_where_the_efie_is_not():
    dt, ng = l2_band_params(frac=0.1)
    ZE = dense_z(dt, FC, ng)
    ZH = dense_h(dt, FC, ng)
    assert _spectral_radius(ZE) > 1.1
    assert _spectral_radius(mfie.combine(ZE, ZH, 0.5)) < 0.8
