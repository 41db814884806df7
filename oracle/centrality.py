"""Subgraph centrality SC(i) = [exp(A)]_ii (eq. 3) by Gauss quadrature: the m-step Lanczos process
started at e_i gives e_i^T f(A) e_i ~ e1^T f(T_m) e1 (Golub-Meurant); for the start e_i, ||e_i|| = 1
and every later basis vector is orthogonal to e_i, so the approximation of [exp(A)]_ii is the first
entry of exp(T_m) e1. With the shift of the main path it is e^{theta*} y_0, y = exp(T_m - theta* I) e1.

Test infrastructure: the HIP path never imports this module.
"""
from __future__ import annotations

import numpy as np

from . import lanczos


def gauss_subgraph_centrality(A, nodes, m: int, reorth: int = 2, eps: float = 2.0 ** -53) -> np.ndarray:
    """FP64 m-point Gauss rule for [exp(A)]_ii of each node i in `nodes` (one Lanczos run each)."""
    n = A.shape[0]
    out = np.empty(len(nodes))
    for q, i in enumerate(nodes):
        e = np.zeros(n)
        e[int(i)] = 1.0
        r = lanczos.lanczos_expv(A, m=m, reorth=reorth, eps=eps, v=e)
        out[q] = np.exp(r.theta) * r.u[int(i)]
    return out
