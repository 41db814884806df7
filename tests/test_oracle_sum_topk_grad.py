"""Pins for the realization sum (eq. 5), the top-K rule and the gradient oracle.

Realization sum: e^{Sigma} S~ must equal the plain sum of exp(A_k) 1 computed densely; the ranking is
invariant under the common scale; a batch of graphs equals the graphs run alone.
Top-K: brute force over (score, id) pairs with planted ties.
Gradient: Van Loan block exponential, divided differences, scipy's Frechet derivative and central
finite differences agree; the Euler identity sum A_ij G_ij = g^T A exp(A) 1 holds.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dense, gradient, scores
from tests import graphs_small as gs


class _Batch:
    """Minimal batch view over dense matrices (one entry of `graphs` per graph, a list of realizations)."""

    def __init__(self, graphs):
        self.mats = []
        gof = []
        for g, reals in enumerate(graphs):
            for A in reals:
                self.mats.append(sp.csr_matrix(A))
                gof.append(g)
        self.graph_of = np.array(gof)
        self.R = len(self.mats)

    def csr(self, r):
        A = self.mats[r]
        return A.shape[0], A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def test_realization_sum_equals_plain_sum():
    reals = [gs.random_graph(60, 0.15 + 0.05 * k, 30 + k) for k in range(5)]
    out = scores.batch_scores(_Batch([reals]), m=40)[0]
    plain = sum(dense.ebtc_pade(A) for A in reals)
    assert rel(np.exp(out.log_scale) * out.s, plain) < 1e-12
    assert out.log_scale == pytest.approx(max(np.linalg.eigvalsh(A)[-1] for A in reals), abs=1e-10)


def test_sum_is_not_an_average_and_k_order_irrelevant_to_value():
    reals = [gs.random_graph(40, 0.2, 40 + k) for k in range(3)]
    a = scores.batch_scores(_Batch([reals]), m=30)[0]
    b = scores.batch_scores(_Batch([reals[::-1]]), m=30)[0]
    assert rel(np.exp(a.log_scale) * a.s, np.exp(b.log_scale) * b.s) < 1e-13
    one = scores.batch_scores(_Batch([reals[:1]]), m=30)[0]
    # three realizations of similar graphs: the sum is about 3x one term, not 1x
    ratio = np.exp(a.log_scale) * a.s.sum() / (np.exp(one.log_scale) * one.s.sum())
    assert 1.5 < ratio < 6.0


def test_batch_of_graphs_equals_singles():
    g1 = [gs.random_graph(50, 0.1, 1), gs.random_graph(50, 0.1, 2)]
    g2 = [gs.random_graph(30, 0.3, 3)]
    both = scores.batch_scores(_Batch([g1, g2]), m=30)
    s1 = scores.batch_scores(_Batch([g1]), m=30)[0]
    s2 = scores.batch_scores(_Batch([g2]), m=30)[0]
    assert rel(both[0].s, s1.s) == 0.0 and rel(both[1].s, s2.s) == 0.0


def test_topk_invariant_under_common_scale():
    reals = [gs.random_graph(80, 0.1, 50 + k) for k in range(4)]
    out = scores.batch_scores(_Batch([reals]), m=40)[0]
    plain = sum(dense.ebtc_pade(A) for A in reals)
    assert scores.topk(out.s, 10).tolist() == scores.topk(plain, 10).tolist()


def test_topk_brute_force_with_ties():
    rng = np.random.default_rng(3)
    s = rng.integers(0, 20, size=300).astype(np.float64)  # many exact ties
    for K in (1, 7, 50, 300):
        brute = [i for _, i in sorted(((-v, i) for i, v in enumerate(s)))][:K]
        assert scores.topk(s, K).tolist() == brute


def test_topk_all_equal_takes_lowest_ids():
    assert scores.topk(np.full(10, 2.5), 4).tolist() == [0, 1, 2, 3]


# ---------------------------------------------------------------- gradient routes

@pytest.fixture(scope="module")
def small_weighted():
    A = gs.random_graph(36, 0.15, 77, weighted=True)
    g = np.random.default_rng(1).normal(size=36)
    return A, g


def test_vanloan_vs_divdiff(small_weighted):
    A, g = small_weighted
    assert rel(gradient.grad_vanloan(A, g), gradient.grad_divdiff(A, g)) < 1e-11


def test_frechet_per_edge(small_weighted):
    A, g = small_weighted
    G = gradient.grad_divdiff(A, g)
    ii, jj = np.nonzero(np.triu(A, 1))
    for i, j in list(zip(ii, jj))[:12]:
        ref = gradient.frechet_edge(A, g, i, j)
        assert abs((G[i, j] + G[j, i]) - ref) < 1e-10 * max(1.0, abs(ref))


def test_central_difference(small_weighted):
    A, g = small_weighted
    G = gradient.grad_vanloan(A, g)
    ii, jj = np.nonzero(np.triu(A, 1))
    for i, j in list(zip(ii, jj))[:8]:
        E = np.zeros_like(A)
        E[i, j] = E[j, i] = 1.0
        fd = gradient.central_difference(lambda h: g @ dense.ebtc_pade(A + h * E), 1e-4)
        assert abs(fd - (G[i, j] + G[j, i])) < 1e-6 * max(1.0, abs(fd))


def test_non_symmetric_entry_derivative(small_weighted):
    # one stored entry alone: derivative is G_ij (not symmetrised); checked against Frechet with E = e_i e_j^T
    A, g = small_weighted
    G = gradient.grad_vanloan(A, g)
    assert abs(G[2, 5] - gradient.frechet_edge(A, g, 2, 5, symmetric=False)) < 1e-10 * max(1.0, abs(G[2, 5]))


def test_euler_identity(small_weighted):
    A, g = small_weighted
    G = gradient.grad_divdiff(A, g)
    lhs, rhs = gradient.euler_identity(A, g, G)
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)


def test_shift_scales_gradient(small_weighted):
    A, g = small_weighted
    th = 3.7
    G = gradient.grad_divdiff(A, g)
    Gs = gradient.grad_divdiff(A - th * np.eye(A.shape[0]), g)
    assert rel(Gs * np.exp(th), G) < 1e-12
