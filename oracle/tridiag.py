"""The small exponential of the Krylov method: y = exp(T - theta* I) e1 for the Lanczos tridiagonal T.

With the m-step Lanczos relation A V_m ~ V_m T_m, exp(A) v1 ~ V_m exp(T_m) e1 (the Krylov
approximation of exp(A) 1 used after eq. (4)). T_m is symmetric tridiagonal (diagonal alpha,
off-diagonal beta). theta* = max eigenvalue of T_m is factored out so that exp never overflows:
exp(T) e1 = e^{theta*} exp(T - theta* I) e1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def tridiag_dense(alpha, beta) -> np.ndarray:
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    return np.diag(a) + np.diag(b, 1) + np.diag(b, -1)


def expv_e1(alpha, beta, shift: bool = True):
    """(y, theta*) with y = exp(T - theta* I) e1; theta* = lambda_max(T), or 0 when shift is False."""
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)[: max(a.size - 1, 0)]
    if a.size == 1:
        theta = float(a[0]) if shift else 0.0
        return np.array([np.exp(a[0] - theta)]), theta
    lam, Q = sla.eigh_tridiagonal(a, b)
    theta = float(lam[-1]) if shift else 0.0
    return Q @ (np.exp(lam - theta) * Q[0, :]), theta


def saad_estimate(y: np.ndarray, beta_last: float) -> float:
    """Relative a-posteriori error estimate beta_m |e_m^T y| / ||y|| (Saad 1992, first term)."""
    ny = float(np.linalg.norm(y))
    return float(beta_last * abs(y[-1]) / ny) if ny > 0 else 0.0
