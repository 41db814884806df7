"""Small deterministic test graphs with known closed forms (dense FP64 adjacency matrices)."""
import numpy as np


def complete(n):
    return np.ones((n, n)) - np.eye(n)


def cycle(n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, (i + 1) % n] = A[(i + 1) % n, i] = 1.0
    return A


def path(n):
    A = np.zeros((n, n))
    for i in range(n - 1):
        A[i, i + 1] = A[i + 1, i] = 1.0
    return A


def bipartite(p, q):
    A = np.zeros((p + q, p + q))
    A[:p, p:] = 1.0
    A[p:, :p] = 1.0
    return A


def random_graph(n, p, seed, weighted=False):
    rng = np.random.default_rng(seed)
    U = np.triu((rng.random((n, n)) < p).astype(float), 1)
    if weighted:
        U *= rng.uniform(0.5, 1.5, size=(n, n))
    return U + U.T


def lollipop(k, tail):
    """K_k with a path of `tail` further nodes hanging off its last node: the leading eigenvector sits
    on the clique, far from the uniform start vector of eq. (4)."""
    n = k + tail
    A = np.zeros((n, n))
    A[:k, :k] = 1.0 - np.eye(k)
    for i in range(k - 1, n - 1):
        A[i, i + 1] = A[i + 1, i] = 1.0
    return A
