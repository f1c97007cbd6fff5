"""Pins of the plate (Sec. 5.1: the paper's plates use the EFIE, alpha = 1)
through the same oracle operators as the spheres:

* the frequency-domain MoM broadside backscatter of 1 m and 2 m plates at
  300 MHz approaches physical optics, 4 pi A^2 / lambda^2, from below as
  the plate grows (0.85 and 0.93 of it; a wrong normalisation of the
  excitation or the current fails it);
* the envelope matrices of the plate workload sum to j w_c Z_FD(f_c);
* the CPPIF march of the plate workload (+-5 %, c dt = 4 m) is stable: its
  companion matrix's spectral radius is below one.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import excitation, geometry, kernels, mie, physics as ph, zfill


def _plate(size, edge=0.1):
    xyz, tri = W.plate_mesh(size, edge)
    return geometry.Surface(xyz, tri, W.rwg_table(tri, open_ok=True))


def test_plate_broadside_rcs_approaches_physical_optics():
    f = 300e6
    lam = ph.C0 / f
    ratio = {}
    for size in (1.0, 2.0):
        s = _plate(size)
        Z = zfill.assemble_dense(s, [kernels.FDKernel(f)])[0]
        w = 2 * math.pi * f
        V = excitation.excitation(s, 1, 1.0, [[0, 0, -1.0]], [[1.0, 0, 0]], 1e30, 0.0, f)[0, 0] / (1j * w)
        I = np.linalg.solve(Z, V)
        sig = mie.rcs_theta_current(s, I, f, np.array([[[0, 0, 1.0]]]), np.array([[[1.0, 0, 0]]]))[0, 0]
        ratio[size] = sig / (4 * math.pi * size ** 4 / lam ** 2)
    assert 0.75 < ratio[1.0] < ratio[2.0] < 1.0


def _plate_workload_matrices():
    wl = W.PLATE_1M
    xyz, tri, rwg = wl.mesh()
    s = geometry.Surface(xyz, tri, rwg)
    dt = ph.dt_from_beta(wl.beta, wl.f_bw)
    ng = ph.ng_from(ph.rmax_of(xyz), dt)
    Z = zfill.assemble_dense(s, [kernels.EnvelopeKernel(m, dt, wl.f0) for m in range(ng + 1)]
                             + [kernels.FDKernel(wl.f0)])
    return wl, Z, ng


def test_plate_envelope_sum_rule_and_stability():
    wl, Z, ng = _plate_workload_matrices()
    ref = 1j * 2 * math.pi * wl.f0 * Z[ng + 1]
    assert np.abs(Z[:ng + 1].sum(0) - ref).max() <= 1e-13 * np.abs(ref).max()
    ns = Z.shape[1]
    Z0i = np.linalg.inv(Z[0])
    C = np.zeros((ns * ng, ns * ng), dtype=np.complex128)
    for m in range(1, ng + 1):
        C[:ns, (m - 1) * ns:m * ns] = -Z0i @ Z[m]
    C[ns:, :-ns] = np.eye(ns * (ng - 1))
    assert np.abs(np.linalg.eigvals(C)).max() < 0.9
