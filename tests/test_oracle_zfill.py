"""Impedance-matrix pins: partition-of-unity sum rule, nonzero-frequency
sum rule (pins the time-derivative terms), CW march limit, symmetry."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import excitation, geometry, kernels, march, physics as ph, zfill
from oracle_cases import dense_z, l2_band_params, sphere

FC = 300e6


def test_sum_over_m_equals_frequency_domain_matrix():
    # sum_m T(m - rho) = 1 and sum_m T'(.) = sum_m T''(.) = 0, so
    # sum_m Z_m = j w_c Z_FD(f_c) with the same quadrature.
    dt, ng = l2_band_params()
    Z = dense_z(dt, FC, ng, (FC,))
    zs = Z[:ng + 1].sum(0)
    zfd = 1j * 2 * math.pi * FC * Z[-1]
    assert np.linalg.norm(zs - zfd) / np.linalg.norm(zfd) < 1e-13


def test_temporal_spectrum_matches_fd_matrix_off_centre():
    # sum_m Z_m exp(-j dw m dt) -> j (w_c + dw) Z_FD(f_c + df) as dt -> 0;
    # the T' and T'' terms carry the dw dependence.  Second order or better.
    dfs = (+0.1 * FC, -0.1 * FC)
    errs = {df: [] for df in dfs}
    for dt in (1.0e-9, 0.5e-9):
        ng = ph.ng_from(1.0, dt)
        Z = dense_z(dt, FC, ng, tuple(FC + df for df in dfs))
        for i, df in enumerate(dfs):
            dw = 2 * math.pi * df
            zt = sum(Z[m] * np.exp(-1j * dw * m * dt) for m in range(ng + 1))
            ref = 1j * 2 * math.pi * (FC + df) * Z[ng + 1 + i]
            errs[df].append(np.linalg.norm(zt - ref) / np.linalg.norm(ref))
    for df in dfs:
        assert errs[df][1] < 5e-5
        assert errs[df][0] / errs[df][1] > 3.5


def test_cw_march_converges_to_fd_solution():
    # Constant drive V_l = j w_c V_FD: a stable (narrow-band) march settles on
    # Z_FD(f_c)^-1 V_FD, i.e. the frequency-domain MoM solution.
    s = sphere()
    dt, ng = l2_band_params(frac=0.01)
    Z = dense_z(dt, FC, ng, (FC,))
    V1 = excitation.excitation(s, 1, 1.0, [[0, 0, -1.0]], [[1.0, 0, 0]], 1e30, 0.0, FC)
    V = np.repeat(V1, 120, axis=0)
    I = march.march_dense(Z[:ng + 1], V)
    ifd = np.linalg.solve(Z[-1], V1[0, 0] / (1j * 2 * math.pi * FC))
    assert np.linalg.norm(I[-1, 0] - ifd) / np.linalg.norm(ifd) < 1e-11


def test_matrices_nearly_symmetric_and_decay():
    dt, ng = l2_band_params()
    Z = dense_z(dt, FC, ng, (FC,))
    for m in range(ng + 1):
        n = np.linalg.norm(Z[m])
        if n > 0:
            # Galerkin symmetry up to the one-sided singular quadrature
            assert np.linalg.norm(Z[m] - Z[m].T) / n < 2e-3
    # the object (1 m) is crossed within one step: Z_4 vanishes for C1
    assert np.linalg.norm(Z[4]) == 0.0
    assert np.linalg.norm(Z[0]) > np.linalg.norm(Z[1]) > np.linalg.norm(Z[2])


def test_broadband_cppif_march_is_unstable_narrowband_stable():
    # Sec. 3.1.1: CPPIF envelope marching loses stability as the band widens.
    s = sphere()
    out = {}
    for frac in (0.01, 0.2):
        dt, ng = l2_band_params(frac=frac)
        Z = dense_z(dt, FC, ng)
        sigma = ph.sigma_from_band(frac * FC)
        V = excitation.excitation(s, 160, dt, [[0, 0, -1.0]], [[1.0, 0, 0]], sigma, 8 * sigma, FC)
        I = march.march_dense(Z, V)
        nrm = np.linalg.norm(I[:, 0], axis=1)
        out[frac] = nrm[-1] / nrm.max()
    assert out[0.01] < 1e-6
    assert out[0.2] > 0.5


def test_refined_touching_rule_is_the_7x7_rule_at_n1():
    """The refined reference rule for touching pairs (both triangles split
    into n^2 sub-triangles, extraction per sub-pair) is the 7 x 7 rule with
    extraction itself at n = 1: on a self pair, where all four half pairs
    touch, it reproduces the impedance entries to rounding."""
    from oracle import touching
    s = sphere()
    dt, ng = l2_band_params()
    ks = [kernels.EnvelopeKernel(m, dt, 300e6) for m in range(ng + 1)]
    for k in (0, 211):
        z = zfill.assemble_pairs(s, [k], [k], ks)[:, 0]
        assert np.abs(touching.refined_pair_entries(s, k, k, ks, 1) - z).max() <= 1e-13 * np.abs(z).max()


def test_touching_pair_spans_against_c_dt():
    """Reading of the touching-pair quadrature: the extraction assumes f(R)
    smooth over the pair, i.e. tau = m - R/(c dt) on one CPPIF piece, which
    holds when the pair spans less than c dt.  On the level-2 sphere (dt from
    beta = 1/5, c dt = 1 m) every touching pair does; on the level-4 sphere
    with N_g = 24 (c dt = 9.3 cm) every touching pair spans more, so the
    library and the oracle apply the same 7 x 7 remainder rule across a
    CPPIF breakpoint there rather than reject the configuration."""
    from oracle import aim, touching
    from gpu_cases import params_of
    for wl, inside in ((W.SPHERE_L2, True), (W.SPHERE_L4, False)):
        p = params_of(wl)
        s = geometry.Surface(p["xyz"], p["tri"], p["rwg"])
        rows, cols = aim.near_pairs(s, p["d_near"])
        span = touching.touching_spans(s, rows, cols)
        t = span > 0
        assert t.sum() > len(rows) // 2
        if inside:
            assert span[t].max() < touching.cdt(p["dt"])
        else:
            assert span[t].min() > touching.cdt(p["dt"])
