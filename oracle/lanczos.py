"""Reference FP64 Lanczos approximation of exp(A) v (v = 1 for the total communicability, eq. 4).

The paper computes exp(A) 1 "directly" with a Krylov method of linear cost (the text after eq. (4),
citing Afanasjew, Eiermann, Ernst and Guettel 2008) and accepts the approximation error in exchange
for speed. A is symmetric, so the Krylov method is the symmetric Lanczos process. Steps, for one
realization (0-based indices):

  1. beta0 = ||v||, v_0 = v / beta0                       (v = 1: beta0 = sqrt(n), v_0 = 1/sqrt(n))
  2. for j = 0, 1, ...:
       w = A v_j
       h = V_j^T w,  w = w - V_j h                          classical Gram-Schmidt against v_0..v_j,
       h' = V_j^T w, w = w - V_j h'                         applied twice (full reorthogonalisation)
       alpha_j = h_j + h'_j,  beta_j = ||w||
       stop  -- breakdown: beta_j == 0 or beta_j <= 64 eps max(|alpha_0..j|, beta_0..j-1)
             -- fixed m: j + 1 == m
             -- adaptive: Saad's estimate beta_j |y_j| / ||y|| < tol, or j + 1 == m_max (capped)
       v_{j+1} = w / beta_j
  3. T = tridiag(beta_0..k-2; alpha_0..k-1; beta_0..k-2), k = number of steps taken

  window = 2 (the memory-bounded variant): step 2 orthogonalises against v_{j-1} and v_j only, with
  the coefficients computed as dot products (in exact arithmetic V_j^T w has no other nonzero entry,
  since A is symmetric: this is the three-term recurrence of Lanczos' method), so only the last two
  basis vectors are needed to continue; the basis is still kept here to form u.
  4. theta* = lambda_max(T); y = exp(T - theta* I) e1                (tridiag.expv_e1)
  5. u = beta0 V_k y, so exp(A) v ~ e^{theta*} u.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import tridiag

FLAG_BREAKDOWN = 1
FLAG_CAPPED = 2


@dataclass
class LanczosResult:
    u: np.ndarray        # beta0 V y; exp(A) v ~ e^theta u
    theta: float         # shift theta* (log-scale of this realization)
    m_used: int
    flags: int
    est: float           # Saad's relative estimate at the last step (0 after a breakdown)
    alpha: np.ndarray    # [m_used]
    beta: np.ndarray     # [m_used]; beta[m_used - 1] is the residual norm of the last step
    beta0: float
    V: np.ndarray | None = None  # n x m_used basis when requested


def lanczos_expv(A, m: int = 0, tol: float = 0.0, m_max: int = 60, shift: bool = True, reorth: int = 2,
                 eps: float = 2.0 ** -53, v: np.ndarray | None = None, keep_basis: bool = False,
                 window: int = 0) -> LanczosResult:
    """m > 0: fixed dimension m; m == 0: adaptive with tolerance tol and cap m_max. window > 0:
    orthogonalise against the last `window` basis vectors only (2 = the three-term recurrence)."""
    n = A.shape[0]
    start = np.ones(n) if v is None else np.asarray(v, dtype=np.float64)
    beta0 = float(np.linalg.norm(start))
    limit = m if m > 0 else m_max
    V = np.zeros((n, limit + 1))
    V[:, 0] = start / beta0
    alpha: list[float] = []
    beta: list[float] = []
    scale = 0.0
    flags = 0
    k = 0
    for j in range(limit):
        w = A @ V[:, j]
        Vj = V[:, (max(0, j - window + 1) if window > 0 else 0): j + 1]
        h = Vj.T @ w
        w = w - Vj @ h
        for _ in range(reorth - 1):
            h2 = Vj.T @ w
            w = w - Vj @ h2
            h = h + h2
        a = float(h[-1])  # the coefficient of v_j
        b = float(np.linalg.norm(w))
        scale = max(scale, abs(a))
        alpha.append(a)
        beta.append(b)
        k = j + 1
        if b == 0.0 or b <= 64.0 * eps * scale:
            flags |= FLAG_BREAKDOWN
            break
        scale = max(scale, b)
        if m > 0:
            if k == m:
                break
        else:
            y, _ = tridiag.expv_e1(alpha, beta[:-1], shift)
            if tridiag.saad_estimate(y, b) < tol:
                break
            if k == m_max:
                flags |= FLAG_CAPPED
                break
        V[:, k] = w / b
    y, theta = tridiag.expv_e1(alpha, beta[: k - 1], shift)
    est = 0.0 if flags & FLAG_BREAKDOWN else tridiag.saad_estimate(y, beta[k - 1])
    u = beta0 * (V[:, :k] @ y)
    return LanczosResult(u, theta, k, flags, est, np.array(alpha), np.array(beta), beta0,
                         V[:, :k].copy() if keep_basis else None)
