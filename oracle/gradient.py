"""Edge-weight gradient of L = <g, exp(A) 1> (the sensitivity of the eq. (4) scores to each entry).

For a perturbation E of A the Frechet derivative of exp is L(A, E) = int_0^1 e^{(1-s)A} E e^{sA} ds,
so dL[E] = sum_ij E_ij G_ij with
    G = int_0^1 e^{sA} g 1^T e^{(1-s)A} ds          (A symmetric).
G_ij is the derivative with respect to the stored entry (i, j); an undirected edge weight that feeds
both (i, j) and (j, i) gets G_ij + G_ji.

Three independent routes:
  vanloan   -- the (1,2) block of expm([[A, g 1^T], [0, A]])        (Van Loan 1978)
  divdiff   -- U (F o (U^T g)(U^T 1)^T) U^T with divided differences F_kl of exp on the spectrum
  frechet   -- scipy.linalg.expm_frechet(A, E) contracted with g and 1, per edge
plus central finite differences of any score function, and the Euler identity
    sum_ij A_ij G_ij = g^T A exp(A) 1   (d/dt <g, e^{tA} 1> at t = 1).
Shifting A by theta I scales G by e^{-theta}; callers pass shifted matrices to avoid overflow.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .dense import to_dense


def grad_vanloan(A, g) -> np.ndarray:
    A = to_dense(A)
    n = A.shape[0]
    M = np.zeros((2 * n, 2 * n))
    M[:n, :n] = A
    M[n:, n:] = A
    M[:n, n:] = np.outer(np.asarray(g, dtype=np.float64), np.ones(n))
    return sla.expm(M)[:n, n:]


def _divided_differences(lam: np.ndarray) -> np.ndarray:
    lk = lam[:, None]
    ll = lam[None, :]
    d = lk - ll
    with np.errstate(invalid="ignore", divide="ignore"):
        ratio = np.where(np.abs(d) > 1e-8, np.expm1(d) / np.where(d == 0, 1.0, d), 1.0 + d / 2 + d * d / 6)
    return np.exp(ll) * ratio


def grad_divdiff(A, g) -> np.ndarray:
    A = to_dense(A)
    lam, U = np.linalg.eigh(A)
    F = _divided_differences(lam)
    a = U.T @ np.asarray(g, dtype=np.float64)
    b = U.T @ np.ones(A.shape[0])
    return U @ (F * np.outer(a, b)) @ U.T


def frechet_edge(A, g, i: int, j: int, symmetric: bool = True) -> float:
    """d/dh <g, exp(A + h E) 1> at h = 0, E = e_i e_j^T (+ e_j e_i^T when symmetric)."""
    A = to_dense(A)
    n = A.shape[0]
    E = np.zeros((n, n))
    E[i, j] = 1.0
    if symmetric:
        E[j, i] += 1.0
    L = sla.expm_frechet(A, E, compute_expm=False)
    return float(np.asarray(g, dtype=np.float64) @ L @ np.ones(n))


def central_difference(f, h: float) -> float:
    """(f(+h) - f(-h)) / (2h) for a scalar function of the step."""
    return (f(h) - f(-h)) / (2.0 * h)


def euler_identity(A, g, G) -> tuple[float, float]:
    """(sum_ij A_ij G_ij, g^T A exp(A) 1)."""
    A = to_dense(A)
    lhs = float(np.sum(A * G))
    rhs = float(np.asarray(g, dtype=np.float64) @ A @ (sla.expm(A) @ np.ones(A.shape[0])))
    return lhs, rhs
