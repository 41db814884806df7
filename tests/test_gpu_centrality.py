"""GPU subgraph centrality (eq. 3 by the Gauss rule of the Lanczos process started at e_i) against
the FP64 oracle of the same rule, the dense diagonal of exp(A) where the Krylov space closes, and
closed forms."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from fixtures import configs as C, graphs as G
from oracle import centrality, dense as odense
from tests.test_gpu_parity import api, torch_mod

pytestmark = pytest.mark.gpu


def device_csr(S, dtype="f64", weighted=False):
    torch = torch_mod()
    S = sp.csr_matrix(S)
    S.sort_indices()
    dev = torch.device("cuda")
    rp = torch.as_tensor(S.indptr.astype(np.int32)).to(dev)
    ci = torch.as_tensor(S.indices.astype(np.int32)).to(dev)
    vals = None
    if weighted:
        vals = torch.as_tensor(S.data.astype(np.float64 if dtype == "f64" else np.float32)).to(dev)
    return rp, ci, vals


def gpu_sc(S, nodes, m, dtype="f64", weighted=False):
    torch = torch_mod()
    rp, ci, vals = device_csr(S, dtype, weighted)
    out = api().subgraph_centrality(rp, ci, vals, nodes, m=m, dtype=dtype)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def er(n, p, seed):
    keys = G.er_keys(n, p, G.rng_for(77, seed, 1))
    rp, ci = G.csr_from_keys(keys, n)
    return odense.csr_to_scipy(n, rp, ci)


@pytest.mark.parametrize("m", [1, 5, 20])
def test_fp64_matches_oracle_gauss_rule(gpu_lib, m):
    A = er(3000, 0.004, 1)  # 2 row blocks, ragged
    nodes = [0, 5, 2047, 2048, 2999, 5, 1234]
    want = centrality.gauss_subgraph_centrality(A, nodes, m)
    got = gpu_sc(A, nodes, m)
    assert np.max(np.abs(got - want) / want) < 1e-12


def test_fp64_weighted_matches_oracle(gpu_lib):
    A = er(800, 0.02, 2).tocoo()
    w = 0.5 + ((np.minimum(A.row, A.col) * 31 + np.maximum(A.row, A.col) * 7) % 17) / 17.0
    W = sp.csr_matrix((w, (A.row, A.col)), shape=A.shape)
    nodes = list(range(0, 800, 97))
    want = centrality.gauss_subgraph_centrality(W, nodes, 15)
    got = gpu_sc(W, nodes, 15, weighted=True)
    assert np.max(np.abs(got - want) / want) < 1e-12


def test_exact_when_the_krylov_space_closes(gpu_lib):
    A = er(40, 0.2, 3)
    nodes = list(range(40))
    exact = np.diag(sla.expm(A.toarray()))
    got = gpu_sc(A, nodes, 40)
    assert np.max(np.abs(got - exact) / exact) < 1e-11


def test_closed_forms_isolated_and_invalid(gpu_lib):
    n = 9
    K = sp.csr_matrix(np.ones((n, n)) - np.eye(n))
    got = gpu_sc(K, [0, 3, 8], 4)
    assert np.allclose(got, (np.exp(n - 1) + (n - 1) * np.exp(-1.0)) / n, rtol=1e-13)
    S = np.zeros((n, n))
    S[0, 1:] = S[1:, 0] = 1.0
    c = np.cosh(np.sqrt(n - 1))
    assert np.allclose(gpu_sc(sp.csr_matrix(S), [0, 2], 4), [c, (n - 2 + c) / (n - 1)], rtol=1e-13)
    Z = np.zeros((6, 6))
    Z[0, 1] = Z[1, 0] = 1.0
    got = gpu_sc(sp.csr_matrix(Z), [3, 0, 6, -1], 3)  # isolated node, an edge's end, two invalid ids
    assert got[0] == 1.0 and abs(got[1] - np.cosh(1.0)) < 1e-14 and np.isnan(got[2]) and np.isnan(got[3])


def test_gauss_rule_lower_bound_monotone(gpu_lib):
    A = er(500, 0.03, 4)
    exact = odense.subgraph_centrality(A)
    nodes = [0, 100, 499]
    prev = np.zeros(3)
    for m in (1, 2, 4, 8, 16):
        got = gpu_sc(A, nodes, m)
        assert np.all(got <= exact[nodes] * (1 + 1e-12)) and np.all(got >= prev * (1 - 1e-12))
        prev = got
    assert np.allclose(prev, exact[nodes], rtol=1e-8)


def test_fp32_on_a_benchmark_realization(gpu_lib):
    # realization 0 of the n=1e5 degree-20 workload; ten planted target nodes and ten others
    w = C.scaled(C.workload(1), N=1)
    hb = C.build(w, with_values=False)
    n, rp, ci, _ = hb.csr(0)
    A = odense.csr_to_scipy(n, rp, ci)
    nodes = np.concatenate([hb.targets[0][:10], np.arange(0, n, n // 10)[:10]]).astype(np.int64)
    want = centrality.gauss_subgraph_centrality(A, nodes, 20)
    got = gpu_sc(A, nodes, 20, dtype="f32")
    assert np.max(np.abs(got - want) / want) < 1e-5
