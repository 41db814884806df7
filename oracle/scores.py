"""Summed communicability over background realizations (eq. 5) and the top-K selection rule.

eq. (5): EBTC(i) = EBTC_1^i + ... + EBTC_N^i -- a plain sum, no averaging ("Multiple backgrounds
scenario"). Each term is exp(A_k) 1 ~ e^{theta_k} u_k (lanczos.lanczos_expv). To stay finite the sum
is carried with one log-scale per graph: Sigma = max_k theta_k and
    S~ = sum_k e^{theta_k - Sigma} u_k         (k ascending, FP64),
so the true summed score is e^{Sigma} S~. Scaling by a positive constant leaves the ranking intact.

Selection: the K largest summed scores are the candidate target nodes ("The total communicability":
largest 20 values; K = target size). Ties go to the lower node id; output sorted by descending score.

`batch` is any object with: R, graph_of [R], n [G], nreal [G], and csr(r) -> (n, row_ptr, col_idx,
values-or-None). Realizations of a graph are consecutive and in k order.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

from . import dense, lanczos


@dataclass
class GraphScores:
    s: np.ndarray          # S~_g [n_g], FP64
    log_scale: float       # Sigma_g
    thetas: np.ndarray     # theta_k per realization
    m_used: np.ndarray
    flags: np.ndarray
    est: np.ndarray
    alpha: list
    beta: list


def realization_result(batch, r: int, m: int, tol: float, m_max: int, shift: bool = True, reorth: int = 2):
    n, rp, ci, v = batch.csr(r)
    A = dense.csr_to_scipy(n, rp, ci, v)
    return lanczos.lanczos_expv(A, m=m, tol=tol, m_max=m_max, shift=shift, reorth=reorth)


_SHARED = {}  # the batch, inherited by forked worker processes instead of being pickled per job


def _one(args):
    r, m, tol, m_max, shift, reorth = args
    batch = _SHARED["batch"]
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            return realization_result(batch, r, m, tol, m_max, shift, reorth)
    except ImportError:  # pragma: no cover
        return realization_result(batch, r, m, tol, m_max, shift, reorth)


def realization_sum(results: list) -> tuple[np.ndarray, float]:
    """S~ and Sigma from the per-realization results of one graph (k ascending)."""
    thetas = np.array([x.theta for x in results])
    sigma = float(thetas.max())
    s = np.zeros_like(results[0].u)
    for x in results:
        s += np.exp(x.theta - sigma) * x.u
    return s, sigma


def batch_scores(batch, m: int = 0, tol: float = 0.0, m_max: int = 60, shift: bool = True, reorth: int = 2,
                 workers: int = 1, realizations: list | None = None) -> list[GraphScores]:
    rs = list(range(batch.R)) if realizations is None else list(realizations)
    jobs = [(r, m, tol, m_max, shift, reorth) for r in rs]
    _SHARED["batch"] = batch
    try:
        if workers > 1 and len(jobs) > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
                res = pool.map(_one, jobs, chunksize=1)
        else:
            res = [_one(j) for j in jobs]
    finally:
        _SHARED.pop("batch", None)
    by_graph: dict[int, list] = {}
    for r, x in zip(rs, res):
        by_graph.setdefault(int(batch.graph_of[r]), []).append(x)
    out = []
    for g in sorted(by_graph):
        xs = by_graph[g]
        s, sigma = realization_sum(xs)
        out.append(GraphScores(s, sigma, np.array([x.theta for x in xs]), np.array([x.m_used for x in xs]),
                               np.array([x.flags for x in xs]), np.array([x.est for x in xs]),
                               [x.alpha for x in xs], [x.beta for x in xs]))
    return out


def topk(s: np.ndarray, K: int) -> np.ndarray:
    """Indices of the K largest entries, descending; ties to the lower index."""
    ids = np.arange(s.size)
    return np.lexsort((ids, -np.asarray(s, dtype=np.float64)))[:K]


def default_workers() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1
