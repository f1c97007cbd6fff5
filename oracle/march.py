"""Marching-on-in-time (oracle; test infrastructure only).

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
