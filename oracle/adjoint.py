"""Adjoint (backward) march and gradient (oracle; test infrastructure only).

The forward march of eq. (4)/(5) is the block lower-triangular Toeplitz
system  sum_{m=0}^{N_g} Z_m I_{l-m} = V_l, l = 1..N_t.  For the objective
J = |F I|^2 (``farfield``), dJ/d conj(V) = lambda with

    Z_0^H lambda_l = s_l - sum_{m=1}^{N_g} Z_m^H lambda_{l+m},  l = N_t..1,
    s = F^H F I,

solved backward in time by LU.  With torch's complex-gradient convention
the gradient of the real J with respect to V is 2 lambda.  Pinned by central
finite differences on the real and imaginary parts of V entries.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def adjoint_march(Z: np.ndarray, S: np.ndarray) -> np.ndarray:
    """lambda [nt, B, ns] for the source S [nt, B, ns]."""
    nt = S.shape[0]
    ng = len(Z) - 1
    ZH = np.conj(np.transpose(Z, (0, 2, 1)))
    lu = sla.lu_factor(ZH[0])
    lam = np.zeros_like(S)
    for l in range(nt - 1, -1, -1):
        rhs = S[l].copy()
        for m in range(1, ng + 1):
            if l + m < nt:
                rhs -= lam[l + m] @ ZH[m].T
        lam[l] = sla.lu_solve(lu, rhs.T).T
    return lam
