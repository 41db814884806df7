"""Planted mistakes: a copy of the oracle with one plausible error must fail the pin battery.

Each mutation edits one line of a temporary copy of the oracle package (never the real one) -- a wrong
sign, a dropped term, a wrong index, a transposed operand -- and the battery below (closed forms,
dense/Pade/Taylor routes, the realization sum, tie-breaking, gradient routes) must reject it. The
unmodified copy must pass the same battery.
"""
import importlib.util
import math
import os
import shutil
import sys

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from tests import graphs_small as gs

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

MUTATIONS = [
    ("lanczos.py", "beta0 = float(np.linalg.norm(start))", "beta0 = float(np.sum(start))"),
    ("lanczos.py", "        w = w - Vj @ h\n", "        w = w + Vj @ h\n"),
    ("lanczos.py", "        a = float(h[-1])  # the coefficient of v_j", "        a = float(h[0])  # the coefficient of v_j"),
    ("lanczos.py", "y, theta = tridiag.expv_e1(alpha, beta[: k - 1], shift)",
     "y, theta = tridiag.expv_e1(alpha, beta[1:k], shift)"),
    ("lanczos.py", "u = beta0 * (V[:, :k] @ y)", "u = (V[:, :k] @ y)"),
    ("lanczos.py", "        w = w - Vj @ h\n        for _ in range(reorth - 1):",
     "        w = w - Vj[:, -1:] @ h[-1:]\n        for _ in range(0):"),
    ("tridiag.py", "return Q @ (np.exp(lam - theta) * Q[0, :]), theta", "return Q @ (np.exp(lam - theta) * Q[:, 0]), theta"),
    ("tridiag.py", "theta = float(lam[-1]) if shift else 0.0", "theta = float(lam[0]) if shift else 0.0"),
    ("scores.py", "s += np.exp(x.theta - sigma) * x.u", "s += np.exp(sigma - x.theta) * x.u"),
    ("scores.py", "return np.lexsort((ids, -np.asarray(s, dtype=np.float64)))[:K]",
     "return np.lexsort((-ids, -np.asarray(s, dtype=np.float64)))[:K]"),
    ("gradient.py", "M[:n, n:] = np.outer(np.asarray(g, dtype=np.float64), np.ones(n))",
     "M[:n, n:] = np.outer(np.ones(n), np.asarray(g, dtype=np.float64))"),
    ("gradient.py", "return U @ (F * np.outer(a, b)) @ U.T", "return U @ (F * np.outer(b, a)) @ U.T"),
    ("dense.py", "return U @ (np.exp(lam) * c)", "return U.T @ (np.exp(lam) * c)"),
    ("taylor.py", "acc = [acc[i] + Fraction(walks[i], fact) for i in range(n)]",
     "acc = [acc[i] + Fraction(walks[i], fact * l) for i in range(n)]"),
    # Saad's relative estimate: the normalisation dropped, the 1-norm, the first component
    ("tridiag.py", "return float(beta_last * abs(y[-1]) / ny) if ny > 0 else 0.0",
     "return float(beta_last * abs(y[-1])) if ny > 0 else 0.0"),
    ("tridiag.py", "ny = float(np.linalg.norm(y))", "ny = float(np.linalg.norm(y, 1))"),
    ("tridiag.py", "return float(beta_last * abs(y[-1]) / ny) if ny > 0 else 0.0",
     "return float(beta_last * abs(y[0]) / ny) if ny > 0 else 0.0"),
    ("lanczos.py", "est = 0.0 if flags & FLAG_BREAKDOWN else tridiag.saad_estimate(y, beta[k - 1])",
     "est = 0.0 if flags & FLAG_BREAKDOWN else tridiag.saad_estimate(y, beta[k - 2])"),
]


def load_copy(tmp_path, mutation=None, tag="m"):
    dst = tmp_path / f"oracle_{tag}"
    shutil.copytree(ORACLE_DIR, dst, ignore=shutil.ignore_patterns("__pycache__"))
    if mutation is not None:
        fname, old, new = mutation
        p = dst / fname
        text = p.read_text()
        assert text.count(old) >= 1, f"mutation anchor not found in {fname}: {old!r}"
        p.write_text(text.replace(old, new, 1))
    name = f"oracle_{tag}"
    spec = importlib.util.spec_from_file_location(name, dst / "__init__.py", submodule_search_locations=[str(dst)])
    mod = importlib.util.module_from_spec(spec)
    sys.modules[name] = mod
    try:
        spec.loader.exec_module(mod)
    finally:
        pass
    return mod


def battery(o) -> list[str]:
    """Return the list of failed pins for an oracle package object."""
    fails = []

    def rel(a, b):
        return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))

    def check(name, fn):
        try:
            if not fn():
                fails.append(name)
        except Exception:  # a crash counts as a failed pin
            fails.append(name)

    n = 12
    a = math.sqrt(n - 1)
    star_ref = np.array([math.cosh(a) + a * math.sinh(a)] + [math.cosh(a) + math.sinh(a) / a] * (n - 1))
    star = gs.bipartite(1, n - 1)
    K6 = gs.complete(6)
    check("dense-star", lambda: rel(o.dense.ebtc_eigh(star), star_ref) < 1e-13)
    check("lanczos-K6", lambda: (lambda r: rel(np.exp(r.theta) * r.u, np.full(6, math.exp(5))) < 1e-13)(
        o.lanczos.lanczos_expv(sp.csr_matrix(K6), m=10)))
    check("lanczos-star", lambda: (lambda r: rel(np.exp(r.theta) * r.u, star_ref) < 1e-13)(
        o.lanczos.lanczos_expv(sp.csr_matrix(star), m=10)))
    A = gs.random_graph(120, 0.08, 5)
    ref = sla.expm(A) @ np.ones(120)
    check("lanczos-vs-expm", lambda: (lambda r: rel(np.exp(r.theta) * r.u, ref) < 1e-11)(
        o.lanczos.lanczos_expv(sp.csr_matrix(A), m=40)))
    check("tridiag-theta-is-max", lambda: abs(o.tridiag.expv_e1([1.0, 3.0, -2.0], [0.5, 0.5])[1]
                                              - np.linalg.eigvalsh(o.tridiag.tridiag_dense([1.0, 3.0, -2.0], [0.5, 0.5]))[-1]) < 1e-12)
    B = gs.random_graph(7, 0.5, 9)
    check("taylor-vs-pade", lambda: rel([float(x) for x in o.taylor.ebtc_taylor_exact(B)], sla.expm(B) @ np.ones(7)) < 1e-13)

    class _B:
        def __init__(self, mats):
            self.mats = [sp.csr_matrix(M) for M in mats]
            self.graph_of = np.zeros(len(mats), int)
            self.R = len(mats)

        def csr(self, r):
            M = self.mats[r]
            return M.shape[0], M.indptr, M.indices, M.data

    reals = [gs.random_graph(40, 0.1 + 0.1 * k, 60 + k) for k in range(3)]
    check("sum-vs-plain", lambda: (lambda g: rel(np.exp(g.log_scale) * g.s, sum(sla.expm(M) @ np.ones(40) for M in reals)) < 1e-12)(
        o.scores.batch_scores(_B(reals), m=40)[0]))
    check("topk-ties", lambda: o.scores.topk(np.array([1.0, 2.0, 2.0, 0.5, 2.0]), 2).tolist() == [1, 2])
    W = gs.random_graph(20, 0.3, 4, weighted=True)
    g = np.random.default_rng(2).normal(size=20)
    i, j = [int(x[0]) for x in np.nonzero(np.triu(W, 1))]
    check("grad-vanloan-vs-frechet", lambda: (lambda G: abs(G[i, j] + G[j, i] - o.gradient.frechet_edge(W, g, i, j)) < 1e-9)(
        o.gradient.grad_vanloan(W, g)))
    check("grad-entry-vanloan", lambda: abs(o.gradient.grad_vanloan(W, g)[i, j]
                                            - o.gradient.frechet_edge(W, g, i, j, symmetric=False)) < 1e-9)
    check("grad-entry-divdiff", lambda: abs(o.gradient.grad_divdiff(W, g)[i, j]
                                            - o.gradient.frechet_edge(W, g, i, j, symmetric=False)) < 1e-9)
    check("grad-divdiff-vs-frechet", lambda: (lambda G: abs(G[i, j] + G[j, i] - o.gradient.frechet_edge(W, g, i, j)) < 1e-9)(
        o.gradient.grad_divdiff(W, g)))

    # Saad's estimate: P_5 at m = 2 by hand (alpha = 8/5, -4/15; beta = sqrt(6)/5, sqrt(5)/3), the
    # 2 x 2 exponential in closed form; invariance under A -> A + 3I without the shift; decay with
    # the true error on a lollipop graph
    def saad_p5():
        r = o.lanczos.lanczos_expv(sp.csr_matrix(gs.path(5)), m=2)
        a0, a1, b0, b1 = 8 / 5, -4 / 15, math.sqrt(6) / 5, math.sqrt(5) / 3
        mu, d = (a0 + a1) / 2, (a0 - a1) / 2
        rr = math.hypot(d, b0)
        y = np.array([math.cosh(rr) + d * math.sinh(rr) / rr, b0 * math.sinh(rr) / rr])
        return abs(r.est - b1 * abs(y[1]) / np.linalg.norm(y)) < 1e-14

    def saad_relative():
        L = gs.lollipop(8, 40)
        e = [o.lanczos.lanczos_expv(sp.csr_matrix(L + c * np.eye(48)), m=8, shift=False).est for c in (0.0, 3.0)]
        return abs(e[1] - e[0]) < 1e-9 * e[0]

    def saad_decays():
        L = gs.lollipop(8, 60)
        ex = sla.expm(L) @ np.ones(68)
        for m in (4, 8):
            r = o.lanczos.lanczos_expv(sp.csr_matrix(L), m=m)
            u = np.exp(r.theta) * r.u
            err = np.linalg.norm(u - ex) / np.linalg.norm(u)
            if not (err <= r.est <= 40.0 * err):
                return False
        return True

    check("saad-p5-by-hand", saad_p5)
    check("saad-relative", saad_relative)
    check("saad-decays", saad_decays)
    return fails


def test_unmodified_copy_passes(tmp_path):
    assert battery(load_copy(tmp_path, None, "clean")) == []


@pytest.mark.parametrize("idx", range(len(MUTATIONS)), ids=[f"{m[0]}:{i}" for i, m in enumerate(MUTATIONS)])
def test_planted_mistake_is_caught(tmp_path, idx):
    mod = load_copy(tmp_path, MUTATIONS[idx], f"mut{idx}")
    assert battery(mod), f"mutation {MUTATIONS[idx]} passed every pin"
