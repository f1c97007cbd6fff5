"""Marching-on-in-time (oracle; test infrastructure only).

* ``gmres``: restarted GMRES (Saad & Schultz 1986) with a right diagonal
  (Jacobi) preconditioner, the solver of Sec. 5.1 ("diagonally
  preconditioned", ref. [20]).  Each Arnoldi step orthogonalises twice
  against the basis (classical Gram-Schmidt, repeated) and solves the small
  least-squares problem of the Hessenberg matrix directly; a cycle ends when
  that problem's residual meets the tolerance, and the solve ends when the
  true residual ||b - A x|| / ||b|| does.
* ``march_fft``: eq. (5) of Sec. 4 with the AIM operator applied by FFT
  convolution (stage (ii)); the right-hand side's history sum over
  m = 1..N_g multiplies the stored spectra of the past currents by the Green
  spectra and adds them before one inverse transform (the transform is
  linear), as the k-space temporal sum of the library does.

* ``march_dense``: eq. (4) of Sec. 3 with dense matrices,
      Z_0 I_l = V_l - sum_{m=1}^{min(N_g, l-1)} Z_m I_{l-m},  l = 1..N_t,
  solved with one LU factorisation of Z_0 (used both for the direct ET-MOT
  matrices and for the assembled ET-AIM matrices Z^near_m + Z^FFT_m of
  eq. (5)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def march_dense(Z: np.ndarray, V: np.ndarray) -> np.ndarray:
    """I [nt, B, ns] from matrices Z [N_g+1, ns, ns] and V [nt, B, ns]."""
    nt = V.shape[0]
    ng = len(Z) - 1
    lu = sla.lu_factor(Z[0])
    I = np.zeros_like(V)
    for l in range(nt):
        rhs = V[l].copy()
        for m in range(1, min(ng, l) + 1):
            rhs -= I[l - m] @ Z[m].T
        I[l] = sla.lu_solve(lu, rhs.T).T
    return I


def gmres(apply, b: np.ndarray, dinv: np.ndarray, x0: np.ndarray, tol: float, restart: int = 50,
          maxit: int = 1000):
    """x with ||b - apply(x)|| <= tol ||b|| (or maxit Arnoldi steps); the
    Krylov space is built on apply(dinv * v).  Returns (x, iterations)."""
    x = x0.astype(np.complex128, copy=True)
    bn = np.linalg.norm(b)
    its = 0
    if bn == 0:
        return np.zeros_like(x), 0
    while True:
        r = b - apply(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bn or its >= maxit:
            return x, its
        V = [r / beta]
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        y = np.zeros(0, dtype=np.complex128)
        for j in range(restart):
            w = apply(dinv * V[j])
            its += 1
            for _ in range(2):
                for i in range(j + 1):
                    h = np.vdot(V[i], w)
                    H[i, j] += h
                    w = w - h * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            y = np.linalg.lstsq(H[:j + 2, :j + 1], g[:j + 2], rcond=None)[0]
            res = np.linalg.norm(g[:j + 2] - H[:j + 2, :j + 1] @ y)
            if H[j + 1, j] == 0 or res <= tol * bn or its >= maxit:
                break
            V.append(w / H[j + 1, j])
        x = x + dinv * (np.array(V[:len(y)]).T @ y)


def march_fft(A, near_vals: np.ndarray, V: np.ndarray, tol: float, restart: int = 50, maxit: int = 1000,
              nsteps: int | None = None, on_step=None):
    """I [nsteps, ns] of eq. (5) for one excitation V [nt, ns] with the AIM
    operator of ``A`` (oracle.aim.AIM) and its pre-corrected near values
    [M_n+1, nnz]; right-Jacobi GMRES with diag(Z^AIM_0) from the zero initial
    guess's predecessor (x0 = I_{l-1}).  on_step(l, iterations) is called
    after each step."""
    nt = V.shape[0] if nsteps is None else nsteps
    ns, ng = V.shape[1], A.ng
    allr = np.arange(ns)
    diag = A.far_pairs(0, allr, allr) + near_vals[0][A.rows == A.cols]   # one self pair per row, in row order
    dinv = 1.0 / diag

    def z0(x):
        return A.far_matvec(0, x) + A.near_matvec(near_vals[0], x)

    I = np.zeros((nt, ns), dtype=np.complex128)
    spec = {}
    for l in range(nt):
        hist = [m for m in range(1, min(ng, l) + 1)]
        rhs = V[l].copy()
        if hist:
            rhs -= A.far_sum_rows([(m, spec[l - m]) for m in hist], allr)
            for m in hist:
                if m <= A.mn:
                    rhs -= A.near_matvec(near_vals[m], I[l - m])
        I[l], its = gmres(z0, rhs, dinv, I[l - 1] if l > 0 else np.zeros(ns, dtype=np.complex128), tol,
                          restart, maxit)
        spec[l] = A.spectra(I[l])
        spec.pop(l - ng, None)
        if on_step is not None:
            on_step(l, its)
    return I
