"""Synthetic input generators: graph laws, embedding invariants, determinism (no method arithmetic)."""
import numpy as np
import pytest

from fixtures import configs as C, graphs as G


def check_simple_symmetric(n, rp, ci):
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert ci.min() >= 0 and ci.max() < n
    assert not np.any(rows == ci), "self-loop"
    key = rows.astype(np.int64) * n + ci
    assert np.all(np.diff(key) > 0), "columns not strictly increasing (duplicate or unsorted)"
    tkey = ci.astype(np.int64) * n + rows
    assert np.array_equal(np.sort(tkey), key), "pattern not symmetric"


@pytest.mark.parametrize("fam,param,deg", [("er", 12.0, 12.0), ("ws", 10, 10.0), ("ba", 4, 8.0)])
def test_family_mean_degree_and_simplicity(fam, param, deg):
    n = 20000
    rng = G.rng_for(7, 0, 1)
    if fam == "er":
        keys = G.er_keys(n, param / (n - 1), rng)
    elif fam == "ws":
        keys = G.ws_keys(n, param, 0.1, rng)
    else:
        keys = G.ba_keys(n, param, rng)
    rp, ci = G.csr_from_keys(keys, n)
    check_simple_symmetric(n, rp, ci)
    d = np.diff(rp)
    assert abs(d.mean() - deg) < 0.03 * deg + 0.1
    if fam == "ba":
        assert d.max() > 20 * deg  # heavy tail (hubs)
    if fam == "ws":
        assert d.min() >= 1 and d.max() < 3 * deg


def test_er_degree_variance_is_binomial():
    n, p = 30000, 10.0 / 29999
    rp, _ = G.csr_from_keys(G.er_keys(n, p, G.rng_for(7, 1, 1)), n)
    d = np.diff(rp)
    assert abs(d.var() - (n - 1) * p * (1 - p)) < 0.05 * (n - 1) * p


def test_embedding_fixes_pattern_in_every_realization():
    w = C.scaled(C.workload(1), n=3000, N=4)
    spec = w.graphs[0]
    d = C.draw_graph(w.ci, 0, spec)
    t = d.targets
    pa, pb = d.pattern // spec.t, d.pattern % spec.t
    want = np.zeros((spec.t, spec.t), bool)
    want[pa, pb] = want[pb, pa] = True
    outside = 0
    for k in range(spec.N):
        rp, ci = C.realization(w.ci, 0, k, d)
        check_simple_symmetric(spec.n, rp, ci)
        got = np.zeros((spec.t, spec.t), bool)
        pos = {int(v): i for i, v in enumerate(t)}
        for i, v in enumerate(t):
            for c in ci[rp[v]:rp[v + 1]]:
                if int(c) in pos:
                    got[i, pos[int(c)]] = True
                else:
                    outside += 1
        assert np.array_equal(got, want)
    assert outside > 0  # target-to-background links come from the background draw


def test_clique_target():
    w = C.scaled(C.workload(2), n=5000, graphs=slice(2, 3))
    d = C.draw_graph(2, 0, w.graphs[0])
    rp, ci = C.realization(2, 0, 0, d)
    for v in d.targets:
        nb = set(ci[rp[v]:rp[v + 1]].tolist())
        assert set(int(x) for x in d.targets if x != v) <= nb


def test_seed_determinism_and_independence():
    w = C.scaled(C.workload(1), n=2000, N=2)
    d1 = C.draw_graph(1, 0, w.graphs[0])
    d2 = C.draw_graph(1, 0, w.graphs[0])
    assert np.array_equal(d1.targets, d2.targets) and np.array_equal(d1.pattern, d2.pattern)
    a = C.realization(1, 0, 0, d1)
    b = C.realization(1, 0, 0, d2)
    c = C.realization(1, 0, 1, d1)
    assert np.array_equal(a[1], b[1]) and not np.array_equal(a[1], c[1][: a[1].size])


def test_workload_shapes():
    w0 = C.workload(0)
    assert w0.dtype == "f64" and w0.m == 20 and w0.graphs[0].N == 20 and w0.graphs[0].n == 200
    w4 = C.workload(4)
    assert len(w4.graphs) == 256 and w4.m == 0 and w4.m_max == 60
    ns = np.array([s.n for s in w4.graphs])
    assert ns.min() >= 10_000 and ns.max() <= 500_000
    assert {s.family for s in w4.graphs} == {"er", "ba", "ws"}
    assert all(20 <= s.t <= 100 and s.K == s.t for s in w4.graphs)


def test_host_batch_offsets():
    b = C.build(C.scaled(C.workload(0), N=3))
    assert b.R == 3 and b.nnz_off[0] == 0 and b.nnz_off[-1] == b.col_idx.size
    for r in range(b.R):
        n, rp, ci, v = b.csr(r)
        assert rp[0] == 0 and rp[-1] == ci.size and v.dtype == np.float64


def test_sparse_target_pattern_statistics():
    # connected, exactly 21 edges on 20 nodes (average degree 2.1), degrees <= 4 with a hub of 4
    for s in range(20):
        keys = G.sparse_target_keys(20, 21, 4, G.rng_for(300, s, 0))
        a, b = keys // 20, keys % 20
        assert keys.size == 21 and np.all(a < b)
        deg = np.bincount(np.concatenate([a, b]), minlength=20)
        assert deg.max() == 4 and deg.min() >= 1
        seen, stack = {0}, [0]
        adj = {i: set() for i in range(20)}
        for i, j in zip(a.tolist(), b.tolist()):
            adj[i].add(j)
            adj[j].add(i)
        while stack:
            for v in adj[stack.pop()]:
                if v not in seen:
                    seen.add(v)
                    stack.append(v)
        assert len(seen) == 20


def test_identification_rate_bookkeeping():
    from paper_1409_5000_amd import idrate
    idx = np.array([3, 1, 2, 9, 8, 7])  # K = 3 per run
    rates = idrate.run_rates(idx, [np.array([1, 2, 3]), np.array([7, 10, 11])], 3)
    assert np.allclose(rates, [1.0, 1 / 3])
    w = idrate.column_workload(idrate.COLUMNS[0], 5, 11)
    assert len(w.graphs) == 5 and w.graphs[0].N == 40 and w.graphs[0].target == "sparse"
    assert abs(w.graphs[0].bg * 1023 - 2.0) < 1e-12
    hb = C.build(idrate.column_workload(idrate.COLUMNS[10], 2, 12), with_values=False)
    assert [t.size for t in hb.targets] == [20, 20] and not np.array_equal(hb.targets[0], hb.targets[1])
