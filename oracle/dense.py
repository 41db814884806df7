"""Dense FP64 routes to exp(A) 1 and diag(exp(A)) -- the plain definitions (small n only).

eq. (4): EBTC_i = sum_j [exp(A)]_ij, i.e. exp(A) applied to the all-ones vector.
eq. (3): SC_i = [exp(A)]_ii.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def to_dense(A) -> np.ndarray:
    if sp.issparse(A):
        return np.asarray(A.toarray(), dtype=np.float64)
    return np.asarray(A, dtype=np.float64)


def ebtc_eigh(A, shift: bool = False):
    """exp(A) 1 = U exp(L) U^T 1 for symmetric A. With shift=True returns (exp(A - lmax I) 1, lmax)."""
    A = to_dense(A)
    lam, U = np.linalg.eigh(A)
    c = U.T @ np.ones(A.shape[0])
    if shift:
        lmax = float(lam[-1]) if lam.size else 0.0
        return U @ (np.exp(lam - lmax) * c), lmax
    return U @ (np.exp(lam) * c)


def ebtc_pade(A) -> np.ndarray:
    """exp(A) 1 through scipy's Pade scaling-and-squaring expm (independent of the eigen route)."""
    A = to_dense(A)
    return sla.expm(A) @ np.ones(A.shape[0])


def subgraph_centrality(A) -> np.ndarray:
    """diag(exp(A)), eq. (3)."""
    A = to_dense(A)
    lam, U = np.linalg.eigh(A)
    return (U * U) @ np.exp(lam)


def csr_to_scipy(n, row_ptr, col_idx, values=None) -> sp.csr_matrix:
    """FP64 scipy CSR matrix from one realization's arrays (values None = all ones)."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    v = np.ones(ci.size, np.float64) if values is None else np.asarray(values, dtype=np.float64)
    return sp.csr_matrix((v, ci, rp - rp[0]), shape=(n, n))
