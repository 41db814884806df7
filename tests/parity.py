"""Comparison rules between the HIP path and the oracle (shared by the GPU tests and the smoke check).

Scores are compared in the oracle's log-domain: s_hat = S~_gpu * exp(Sigma_gpu - Sigma_ref) against
s = S~_ref (both FP64 on the host).
  err_norm = max_i |s_hat_i - s_i| / max_i |s_i|
  err_top  = max over the oracle's top-2K of |s_hat_i - s_i| / |s_i|
Top-K sets must be identical unless the oracle's K-th and (K+1)-th scores lie within twice the
tolerance of each other (a tie band), in which case the test reports it and accepts any set that is
consistent with the band.
"""
from __future__ import annotations

import numpy as np

TOL = {"f32": 1e-5, "f64": 1e-12}


def scaled(gpu_s: np.ndarray, gpu_sigma: float, ref_sigma: float) -> np.ndarray:
    return np.asarray(gpu_s, dtype=np.float64) * np.exp(gpu_sigma - ref_sigma)


def errors(s_hat: np.ndarray, s: np.ndarray, K: int) -> tuple[float, float]:
    err_norm = float(np.max(np.abs(s_hat - s)) / np.max(np.abs(s)))
    top = np.lexsort((np.arange(s.size), -s))[: min(2 * K, s.size)]
    err_top = float(np.max(np.abs(s_hat[top] - s[top]) / np.abs(s[top])))
    return err_norm, err_top


def topk_consistent(gpu_idx: np.ndarray, s: np.ndarray, K: int, tol: float) -> tuple[bool, bool]:
    """(ok, tie_band): the GPU's top-K set agrees with the oracle's, exactly or within the tie band."""
    order = np.lexsort((np.arange(s.size), -s))
    ref = set(order[:K].tolist())
    got = set(np.asarray(gpu_idx).tolist())
    if got == ref:
        return True, False
    if K >= s.size:
        return False, False
    kth, nxt = s[order[K - 1]], s[order[K]]
    band = abs(kth - nxt) <= 2 * tol * abs(kth)
    if not band:
        return False, False
    lo = kth * (1 - 2 * tol)
    sure = set(order[: K][s[order[:K]] > kth * (1 + 2 * tol)].tolist())
    allowed = set(np.flatnonzero(s >= lo).tolist())
    return sure <= got and got <= allowed, True
