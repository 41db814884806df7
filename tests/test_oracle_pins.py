"""Pins of the FP64 oracle against what mathematics fixes independently of the oracle's own code.

Closed forms of exp(A) 1 (eq. 4) for complete, regular, complete-bipartite, star, path and empty
graphs; exact rational Taylor sums on tiny graphs; two independent library routes (eigendecomposition
vs Pade expm, scipy's expm_multiply); invariants (symmetry, permutation equivariance, disjoint
union, shift invariance); Lanczos special cases (exactness when the Krylov space closes, breakdown).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import dense, taylor, tridiag, lanczos
from tests import graphs_small as gs


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# ---------------------------------------------------------------- closed forms (eq. 4)

def closed_complete(n):
    return np.full(n, math.exp(n - 1))


def closed_regular(n, r):
    return np.full(n, math.exp(r))


def closed_bipartite(p, q):
    a = math.sqrt(p * q)
    side_p = math.cosh(a) + q * math.sinh(a) / a
    side_q = math.cosh(a) + p * math.sinh(a) / a
    return np.concatenate([np.full(p, side_p), np.full(q, side_q)])


def closed_path(n):
    k = np.arange(1, n + 1)
    i = np.arange(1, n + 1)
    U = np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(i, k) / (n + 1))  # columns = eigenvectors
    lam = 2.0 * np.cos(np.pi * k / (n + 1))
    return U @ (np.exp(lam) * (U.T @ np.ones(n)))


CLOSED = [
    ("K5", lambda: gs.complete(5), lambda: closed_complete(5)),
    ("K37", lambda: gs.complete(37), lambda: closed_complete(37)),
    ("C9", lambda: gs.cycle(9), lambda: closed_regular(9, 2)),
    ("C40", lambda: gs.cycle(40), lambda: closed_regular(40, 2)),
    ("K3_7", lambda: gs.bipartite(3, 7), lambda: closed_bipartite(3, 7)),
    ("star12", lambda: gs.bipartite(1, 11), lambda: closed_bipartite(1, 11)),
    ("P17", lambda: gs.path(17), lambda: closed_path(17)),
    ("empty6", lambda: np.zeros((6, 6)), lambda: np.ones(6)),
]


def test_star_closed_form_matches_its_two_line_statement():
    # hub: cosh a + a sinh a, leaves: cosh a + sinh(a)/a with a = sqrt(n - 1)
    n = 12
    a = math.sqrt(n - 1)
    v = closed_bipartite(1, n - 1)
    assert abs(v[0] - (math.cosh(a) + a * math.sinh(a))) < 1e-12 * v[0]
    assert abs(v[1] - (math.cosh(a) + math.sinh(a) / a)) < 1e-12 * v[1]


@pytest.mark.parametrize("name,mk,closed", CLOSED, ids=[c[0] for c in CLOSED])
def test_dense_routes_closed_forms(name, mk, closed):
    A = mk()
    assert rel(dense.ebtc_eigh(A), closed()) < 1e-13
    # scaling-and-squaring carries about u * ||A|| * (number of squarings) of rounding
    assert rel(dense.ebtc_pade(A), closed()) < 1e-14 * max(10.0, np.abs(A).sum(axis=1).max()) * 10
    s, lmax = dense.ebtc_eigh(A, shift=True)
    assert rel(np.exp(lmax) * s, closed()) < 1e-13


@pytest.mark.parametrize("name,mk,closed", CLOSED, ids=[c[0] for c in CLOSED])
def test_lanczos_closed_forms(name, mk, closed):
    A = sp.csr_matrix(mk())
    res = lanczos.lanczos_expv(A, m=20)
    assert rel(np.exp(res.theta) * res.u, closed()) < 1e-13


@pytest.mark.parametrize("A,steps", [
    (gs.complete(9), 1), (gs.cycle(11), 1), (np.zeros((5, 5)), 1), (gs.bipartite(3, 7), 2), (gs.bipartite(1, 9), 2),
], ids=["K9", "C11", "empty", "K3_7", "star10"])
def test_lanczos_breakdown_steps(A, steps):
    res = lanczos.lanczos_expv(sp.csr_matrix(A), m=20)
    assert res.m_used == steps
    assert res.flags & lanczos.FLAG_BREAKDOWN


def test_empty_graph_alpha_beta_zero():
    res = lanczos.lanczos_expv(sp.csr_matrix(np.zeros((4, 4))), m=5)
    assert res.alpha.tolist() == [0.0] and res.beta.tolist() == [0.0] and res.theta == 0.0
    assert np.allclose(res.u, 1.0, rtol=0, atol=1e-15)


def test_path_symmetric_krylov_space_closes():
    # 1 lies in the reflection-symmetric subspace (dimension ceil(n/2)), so Lanczos ends there, exact.
    n = 15
    res = lanczos.lanczos_expv(sp.csr_matrix(gs.path(n)), m=40)
    assert res.m_used == (n + 1) // 2
    assert rel(np.exp(res.theta) * res.u, closed_path(n)) < 1e-13


# ---------------------------------------------------------------- brute force: exact Taylor series

@pytest.mark.parametrize("seed", range(6))
def test_taylor_exact_vs_eigh(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 11))
    A = gs.random_graph(n, 0.45, seed)
    exact = np.array([float(x) for x in taylor.ebtc_taylor_exact(A)])
    assert rel(dense.ebtc_eigh(A), exact) < 1e-14
    assert rel(dense.ebtc_pade(A), exact) < 1e-12


def test_taylor_exact_closed_form_K4():
    exact = taylor.ebtc_taylor_exact(gs.complete(4))
    assert abs(float(exact[0]) - math.exp(3)) < 1e-14 * math.exp(3)


# ---------------------------------------------------------------- two library routes, invariants

@pytest.mark.parametrize("seed", range(4))
def test_eigh_vs_pade_random(seed):
    A = gs.random_graph(120, 0.08, seed, weighted=bool(seed % 2))
    assert rel(dense.ebtc_eigh(A), dense.ebtc_pade(A)) < 1e-12


def test_symmetry_rows_equal_columns():
    A = gs.random_graph(60, 0.1, 7, weighted=True)
    E = sla.expm(A)
    assert np.max(np.abs(E - E.T)) < 1e-12 * np.max(np.abs(E))
    assert rel(np.ones(60) @ E, dense.ebtc_eigh(A)) < 1e-12


def test_subgraph_centrality_is_diagonal():
    A = gs.random_graph(50, 0.15, 3)
    assert rel(dense.subgraph_centrality(A), np.diag(sla.expm(A))) < 1e-12


def test_permutation_equivariance():
    A = gs.random_graph(80, 0.1, 11)
    perm = np.random.default_rng(5).permutation(80)
    P = np.eye(80)[perm]
    s = dense.ebtc_eigh(A)
    sp_ = dense.ebtc_eigh(P @ A @ P.T)
    assert rel(sp_, P @ s) < 1e-12
    r1 = lanczos.lanczos_expv(sp.csr_matrix(A), m=30)
    r2 = lanczos.lanczos_expv(sp.csr_matrix(P @ A @ P.T), m=30)
    assert rel(np.exp(r2.theta) * r2.u, P @ (np.exp(r1.theta) * r1.u)) < 1e-12


def test_disjoint_union_is_concatenation():
    A = gs.random_graph(30, 0.2, 1)
    B = gs.random_graph(20, 0.3, 2)
    U = sla.block_diag(A, B)
    assert rel(dense.ebtc_eigh(U), np.concatenate([dense.ebtc_eigh(A), dense.ebtc_eigh(B)])) < 1e-12
    res = lanczos.lanczos_expv(sp.csr_matrix(U), m=50)
    assert rel(np.exp(res.theta) * res.u, dense.ebtc_eigh(U)) < 1e-12


# ---------------------------------------------------------------- the small exponential

def test_tridiag_two_by_two_closed_form():
    a, c, b = 1.3, -0.4, 0.7
    mean, half = (a + c) / 2, math.sqrt(((a - c) / 2) ** 2 + b * b)
    # exp([[a,b],[b,c]]) e1 = e^mean [cosh h + (a-c)/(2h) sinh h, b/h sinh h]
    ref = math.exp(mean) * np.array([math.cosh(half) + (a - c) / (2 * half) * math.sinh(half),
                                     b / half * math.sinh(half)])
    y, theta = tridiag.expv_e1([a, c], [b])
    assert abs(theta - (mean + half)) < 1e-15
    assert rel(np.exp(theta) * y, ref) < 1e-14


@pytest.mark.parametrize("kind", ["random", "clustered", "split", "one"])
def test_tridiag_vs_pade(kind):
    rng = np.random.default_rng(42)
    k = 1 if kind == "one" else 30
    a = rng.normal(0, 4, k)
    b = np.abs(rng.normal(0, 2, max(k - 1, 0)))
    if kind == "clustered":
        a = np.full(k, 3.0) + 1e-9 * rng.normal(size=k)
        b = np.full(k - 1, 1e-7)
    if kind == "split":
        b[10] = 0.0
    y, theta = tridiag.expv_e1(a, b)
    T = tridiag.tridiag_dense(a, b)
    ref = sla.expm(T - theta * np.eye(k))[:, 0]
    assert rel(y, ref) < 1e-13
    assert abs(theta - np.linalg.eigvalsh(T)[-1]) < 1e-12 * max(1.0, abs(theta))


# ---------------------------------------------------------------- Lanczos vs the plain definition

@pytest.mark.parametrize("seed", range(3))
def test_lanczos_vs_dense_c0_shape(seed):
    A = gs.random_graph(200, 0.1, 20 + seed)
    res = lanczos.lanczos_expv(sp.csr_matrix(A), m=20)
    s, lmax = dense.ebtc_eigh(A, shift=True)
    assert abs(res.theta - lmax) < 1e-10
    assert rel(res.u * np.exp(res.theta - lmax), s) < 1e-12


def test_lanczos_vs_expm_multiply_large():
    from fixtures import graphs as G
    n = 20000
    keys = G.er_keys(n, 20.0 / (n - 1), G.rng_for(99, 0, 1))
    rp, ci = G.csr_from_keys(keys, n)
    A = dense.csr_to_scipy(n, rp, ci)
    res = lanczos.lanczos_expv(A, m=30)
    ref = spla.expm_multiply(A - res.theta * sp.identity(n, format="csr"), np.ones(n))
    assert rel(res.u, ref) < 1e-11


def test_lanczos_basis_orthonormal_and_relation():
    A = sp.csr_matrix(gs.random_graph(300, 0.05, 8))
    res = lanczos.lanczos_expv(A, m=25, keep_basis=True)
    V = res.V
    assert np.max(np.abs(V.T @ V - np.eye(V.shape[1]))) < 1e-13
    T = tridiag.tridiag_dense(res.alpha, res.beta[:-1])
    R = A @ V - V @ T
    # residual lives only in the last column, with norm beta_{m-1}
    assert np.max(np.abs(R[:, :-1])) < 1e-12
    assert abs(np.linalg.norm(R[:, -1]) - res.beta[-1]) < 1e-12


def test_reorth_once_vs_twice_fp64():
    A = sp.csr_matrix(gs.random_graph(400, 0.04, 9))
    r1 = lanczos.lanczos_expv(A, m=30, reorth=1)
    r2 = lanczos.lanczos_expv(A, m=30, reorth=2)
    assert rel(r1.u, r2.u) < 1e-12 and abs(r1.theta - r2.theta) < 1e-12


def test_shift_off_gives_same_product():
    A = sp.csr_matrix(gs.random_graph(100, 0.05, 10))
    r_on = lanczos.lanczos_expv(A, m=20)
    r_off = lanczos.lanczos_expv(A, m=20, shift=False)
    assert r_off.theta == 0.0
    assert rel(r_off.u, np.exp(r_on.theta) * r_on.u) < 1e-13


def test_adaptive_stop_and_cap():
    A = sp.csr_matrix(gs.random_graph(500, 0.03, 12))
    s, lmax = dense.ebtc_eigh(A.toarray(), shift=True)
    r = lanczos.lanczos_expv(A, m=0, tol=1e-6, m_max=60)
    assert r.est < 1e-6 and not (r.flags & lanczos.FLAG_CAPPED)
    assert rel(r.u * np.exp(r.theta - lmax), s) < 1e-5
    r_cap = lanczos.lanczos_expv(A, m=0, tol=1e-14, m_max=3)
    assert r_cap.m_used == 3 and (r_cap.flags & lanczos.FLAG_CAPPED)
    # the estimate is monotone enough to stop earlier for a looser tolerance
    r_loose = lanczos.lanczos_expv(A, m=0, tol=1e-3, m_max=60)
    assert r_loose.m_used < r.m_used


# ------------------------------------------------------------------ Saad's a-posteriori estimate

def p5_lanczos_by_hand():
    """Two Lanczos steps on the path P_5 from 1/sqrt(5), worked out by hand in exact arithmetic.

    alpha_0 = 1^T A 1 / 5 = 8/5 (twice the 4 edges over 5 nodes). A v_0 - alpha_0 v_0 = (d - 8/5)/sqrt(5)
    with degrees d = (1,2,2,2,1): (-0.6, 0.4, 0.4, 0.4, -0.6)/sqrt(5), so beta_0 = sqrt(1.2/5) = sqrt(6)/5
    and v_1 = (-0.6, 0.4, 0.4, 0.4, -0.6)/sqrt(1.2). A v_1 = (0.4, -0.2, 0.8, -0.2, 0.4)/sqrt(1.2), so
    alpha_1 = -0.32/1.2 = -4/15, and w = A v_1 - alpha_1 v_1 - beta_0 v_0 = (0, -1/3, 2/3, -1/3, 0)/sqrt(1.2)
    gives beta_1 = sqrt((6/9)/1.2) = sqrt(5)/3.
    """
    return (8 / 5, -4 / 15), math.sqrt(6) / 5, math.sqrt(5) / 3


def expm2_e1(a, b, c):
    """exp([[a, b], [b, c]]) e1 in closed form: with mu = (a+c)/2, d = (a-c)/2, r = sqrt(d^2 + b^2),
    exp(T) = e^mu (cosh(r) I + sinh(r)/r (T - mu I))."""
    mu, d = (a + c) / 2, (a - c) / 2
    r = math.hypot(d, b)
    return math.exp(mu) * np.array([math.cosh(r) + d * math.sinh(r) / r, b * math.sinh(r) / r])


def test_saad_estimate_two_by_two_by_hand():
    """Saad's relative estimate beta_m |e_m^T exp(T_m) e1| / ||exp(T_m) e1||_2 (the stop rule of the
    adaptive Krylov approximation, text after eq. (4)) on 2 x 2 tridiagonals whose exponential is a
    closed form, through the oracle's whole Lanczos path (P_5, m = 2) and through the helper alone."""
    (a0, a1), b0, b1 = p5_lanczos_by_hand()
    r = lanczos.lanczos_expv(sp.csr_matrix(gs.path(5)), m=2)
    assert r.m_used == 2 and r.flags == 0
    assert abs(r.alpha[0] - a0) < 1e-15 and abs(r.alpha[1] - a1) < 1e-15
    assert abs(r.beta[0] - b0) < 1e-15 and abs(r.beta[1] - b1) < 1e-15
    y = expm2_e1(a0, b0, a1)
    est = b1 * abs(y[1]) / math.hypot(y[0], y[1])
    assert abs(r.est - est) < 1e-14 * est
    # T = [[1, 2], [2, -2]]: r = 5/2, exp(T) e1 = e^{-1/2} (cosh 2.5 + 0.6 sinh 2.5, 0.8 sinh 2.5)
    c, s = math.cosh(2.5), math.sinh(2.5)
    want = 0.5 * 0.8 * s / math.hypot(c + 0.6 * s, 0.8 * s)
    y2, _ = tridiag.expv_e1([1.0, -2.0], [2.0])
    assert abs(tridiag.saad_estimate(y2, 0.5) - want) < 1e-15
    assert abs(want - 0.22209888659244936) < 1e-15


def test_saad_estimate_is_relative():
    """The estimate is a relative error: exp(A + cI) 1 = e^c exp(A) 1 has the same relative error, the
    same Lanczos basis and T shifted by c, so without the shift (y = exp(T) e1 grows by e^c) the
    estimate must not change."""
    for A in (gs.lollipop(8, 40), gs.random_graph(200, 0.04, 21)):
        n = A.shape[0]
        e = [lanczos.lanczos_expv(sp.csr_matrix(A + c * np.eye(n)), m=8, shift=False).est for c in (0.0, 3.0)]
        assert e[0] > 1e-8 and abs(e[1] - e[0]) < 1e-9 * e[0]


@pytest.mark.parametrize("name, A", [("lollipop8_60", gs.lollipop(8, 60)), ("er300", gs.random_graph(300, 0.05, 3))])
def test_saad_estimate_tracks_the_true_error(name, A):
    """Against the true relative error ||u_m - exp(A) 1|| / ||u_m|| (dense expm): while the error is
    above rounding, the estimate stays above it and within a factor 40 (the first-term estimate uses
    exp(T) where the exact error term has (exp(T) - I) T^{-1}, so it runs high by about lambda_max)
    and falls with it."""
    n = A.shape[0]
    ex = sla.expm(A) @ np.ones(n)
    prev = None
    for m in range(4, 20, 2):
        r = lanczos.lanczos_expv(sp.csr_matrix(A), m=m)
        u = np.exp(r.theta) * r.u
        err = np.linalg.norm(u - ex) / np.linalg.norm(u)
        if err < 1e-10:
            break
        assert err <= r.est <= 40.0 * err, (name, m, err, r.est)
        if prev is not None:
            assert r.est < 0.2 * prev
        prev = r.est
    assert prev is not None


# ------------------------------------------------------------------ subgraph centrality (Gauss rule)

def test_gauss_subgraph_centrality_exact_when_the_krylov_space_closes():
    from oracle import centrality
    rng = np.random.default_rng(5)
    A = (rng.random((30, 30)) < 0.15).astype(float)
    A = np.triu(A, 1)
    A = A + A.T
    nodes = np.arange(30)
    exact = np.diag(sla.expm(A))
    got = centrality.gauss_subgraph_centrality(sp.csr_matrix(A), nodes, m=30)
    assert np.max(np.abs(got - exact) / exact) < 1e-12


def test_gauss_subgraph_centrality_closed_forms():
    from oracle import centrality
    n = 9
    K = np.ones((n, n)) - np.eye(n)
    sc = centrality.gauss_subgraph_centrality(sp.csr_matrix(K), [0, 4], m=5)
    want = (np.exp(n - 1) + (n - 1) * np.exp(-1.0)) / n   # K_n: eigenvalues n-1 and -1 (n-1 times)
    assert np.allclose(sc, want, rtol=1e-13)
    S = np.zeros((n, n))
    S[0, 1:] = S[1:, 0] = 1.0                               # star: eigenvalues +-sqrt(n-1), 0
    sc = centrality.gauss_subgraph_centrality(sp.csr_matrix(S), [0, 3], m=5)
    c = np.cosh(np.sqrt(n - 1))
    assert np.allclose(sc, [c, (n - 2 + c) / (n - 1)], rtol=1e-13)
    Z = sp.csr_matrix((5, 5))                               # isolated nodes: SC = 1
    assert np.allclose(centrality.gauss_subgraph_centrality(Z, [0, 4], m=3), 1.0)


def test_gauss_rule_is_a_monotone_lower_bound():
    # exp has positive even derivatives, so every m-point Gauss rule underestimates [exp(A)]_ii and
    # the estimates increase with m
    from oracle import centrality
    rng = np.random.default_rng(9)
    A = (rng.random((60, 60)) < 0.1).astype(float)
    A = np.triu(A, 1)
    A = sp.csr_matrix(A + A.T)
    exact = dense.subgraph_centrality(A)
    nodes = [0, 7, 33]
    prev = np.zeros(3)
    for m in (1, 2, 3, 5, 8):
        sc = centrality.gauss_subgraph_centrality(A, nodes, m=m)
        assert np.all(sc <= exact[nodes] * (1 + 1e-12)) and np.all(sc >= prev * (1 - 1e-12))
        prev = sc
    assert np.allclose(prev, exact[nodes], rtol=1e-6)


# ------------------------------------------------------------------ memory-bounded (windowed) Lanczos

@pytest.mark.parametrize("n,p,m", [(300, 0.05, 20), (1500, 0.01, 60), (500, 0.1, 40)])
def test_windowed_lanczos_matches_full_reorthogonalisation(n, p, m):
    # the three-term recurrence (Gram-Schmidt against v_{j-1}, v_j only) approximates exp(A)1 as well
    # as full reorthogonalisation does: the loss of orthogonality does not spoil f(A)v (FP64)
    from fixtures import graphs as G
    keys = G.er_keys(n, p, G.rng_for(5, n, 1))
    rp, ci = G.csr_from_keys(keys, n)
    A = dense.csr_to_scipy(n, rp, ci)
    full = lanczos.lanczos_expv(A, m=m, reorth=2)
    win = lanczos.lanczos_expv(A, m=m, reorth=1, window=2)
    assert win.m_used == full.m_used == m
    uf, uw = np.exp(full.theta) * full.u, np.exp(win.theta) * win.u
    assert np.max(np.abs(uw - uf)) / np.max(np.abs(uf)) < 1e-12
    # the first coefficients agree; later ones drift once orthogonality is lost (ghost Ritz values),
    # which the approximation of exp(A)1 does not notice
    assert np.max(np.abs(np.asarray(win.alpha[:5]) - np.asarray(full.alpha[:5]))) < 1e-12 * abs(full.alpha[0])


def test_windowed_lanczos_needs_the_previous_vector():
    # with a window of one vector (v_j only) the recurrence drops the beta_{j-1} v_{j-1} term and the
    # basis loses orthogonality at once: the approximation is visibly wrong -- the window of two is
    # what makes the three-term recurrence
    from fixtures import graphs as G
    n = 400
    keys = G.er_keys(n, 0.05, G.rng_for(6, 0, 1))
    rp, ci = G.csr_from_keys(keys, n)
    A = dense.csr_to_scipy(n, rp, ci)
    exact = sla.expm(A.toarray()) @ np.ones(n)
    full = lanczos.lanczos_expv(A, m=25, reorth=2)
    w2 = lanczos.lanczos_expv(A, m=25, reorth=1, window=2)
    w1 = lanczos.lanczos_expv(A, m=25, reorth=1, window=1)
    err = lambda r: np.max(np.abs(np.exp(r.theta) * r.u - exact)) / np.max(np.abs(exact))
    assert err(w2) < 1.01 * err(full) + 1e-14 and err(w1) > 1e-3


def test_windowed_lanczos_exact_on_a_closing_space():
    P = np.zeros((8, 8))
    for i in range(7):
        P[i, i + 1] = P[i + 1, i] = 1.0
    r = lanczos.lanczos_expv(sp.csr_matrix(P), m=8, reorth=1, window=2)
    exact = sla.expm(P) @ np.ones(8)
    assert np.max(np.abs(np.exp(r.theta) * r.u - exact)) / np.max(exact) < 1e-13
