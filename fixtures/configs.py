"""Workload recipes and host-side batch assembly (seeded, synthetic).

Each recipe fixes the background family and size, the target pattern, the number of background
realizations N and the selection size K. The five workloads follow the experiments of the paper
(ER/SW/BA backgrounds with a sparse or complete target, many or one background) at the sizes the
benchmarks are quoted on:

  0  tiny plain method: ER n=200 p=0.1, N=20, 10-node ER(p=0.3) target, FP64, m=20, K=10
  1  batched realizations: ER n=1e5 degree 20, N=64, 50-node target (internal degree 4), FP32, m=30
  2  single background, three n=1e6 graphs (BA m=5, WS k=10 beta=0.1, ER degree 10), 30-clique, m=40
  3  differentiation: ER n=2e5 degree 16, N=16, 40-node target (internal degree 3), FP32, m=30
  4  uneven batch: 256 graphs, n ~ U{1e4..5e5}, family ~ U{ER, BA, WS}, degree ~ U[8, 32],
     target t ~ U{20..100} sparse ER(degree 3) or clique, N=8, adaptive m (tol 1e-6, cap 60)

No value here depends on the method's arithmetic.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

from . import graphs as G


@dataclass(frozen=True)
class GraphSpec:
    family: str          # "er" | "ws" | "ba"
    n: int
    bg: float            # ER: edge probability p; WS: lattice degree k; BA: edges per new node m
    target: str = "er"   # "er" (fixed random pattern), "sparse" (connected, hubs of degree 4) or "clique"
    t: int = 10          # target size
    int_p: float = 0.3   # internal edge probability of an "er" target pattern
    N: int = 1           # background realizations
    K: int = 10          # selection size (= target size in the paper's protocol)
    ws_beta: float = 0.1


@dataclass(frozen=True)
class Workload:
    ci: int
    name: str
    graphs: tuple
    dtype: str           # "f32" | "f64"
    m: int               # fixed Krylov dimension, 0 = adaptive
    tol: float = 0.0
    m_max: int = 0


def er_spec(n, degree, **kw):
    return GraphSpec("er", n, degree / (n - 1), **kw)


def workload(ci: int) -> Workload:
    if ci == 0:
        return Workload(0, "tiny-er-n200-N20", (GraphSpec("er", 200, 0.1, "er", 10, 0.3, 20, 10),), "f64", 20)
    if ci == 1:
        return Workload(1, "er-n1e5-d20-N64", (er_spec(100_000, 20.0, target="er", t=50, int_p=4 / 49, N=64, K=50),),
                        "f32", 30)
    if ci == 2:
        n = 1_000_000
        return Workload(2, "single-bg-n1e6-ba-ws-er", (
            GraphSpec("ba", n, 5, "clique", 30, 1.0, 1, 30),
            GraphSpec("ws", n, 10, "clique", 30, 1.0, 1, 30, ws_beta=0.1),
            er_spec(n, 10.0, target="clique", t=30, int_p=1.0, N=1, K=30)), "f32", 40)
    if ci == 3:
        return Workload(3, "er-n2e5-d16-N16-grad", (er_spec(200_000, 16.0, target="er", t=40, int_p=3 / 39, N=16, K=40),),
                        "f32", 30)
    if ci == 4:
        rng = G.rng_for(4, 1 << 20, 0)
        specs = []
        for _ in range(256):
            n = int(rng.integers(10_000, 500_001))
            fam = ("er", "ba", "ws")[int(rng.integers(0, 3))]
            d = float(rng.uniform(8.0, 32.0))
            t = int(rng.integers(20, 101))
            sparse = bool(rng.random() < 0.5)
            tgt = dict(target="er" if sparse else "clique", t=t, int_p=3.0 / (t - 1) if sparse else 1.0, N=8, K=t)
            if fam == "er":
                specs.append(GraphSpec("er", n, d / (n - 1), **tgt))
            elif fam == "ba":
                specs.append(GraphSpec("ba", n, max(1, int(round(d / 2))), **tgt))
            else:
                specs.append(GraphSpec("ws", n, 2 * max(1, int(round(d / 2))), **tgt))
        return Workload(4, "uneven-256-graphs-N8-adaptive", tuple(specs), "f32", 0, 1e-6, 60)
    raise ValueError(f"no workload {ci}")


def scaled(w: Workload, n: int | None = None, N: int | None = None, graphs: slice | None = None) -> Workload:
    """The same recipe at a smaller size (degree and target kept; ER p rescaled to keep the degree)."""
    specs = list(w.graphs[graphs] if graphs is not None else w.graphs)
    out = []
    for s in specs:
        kw = {}
        if n is not None:
            kw["n"] = n
            if s.family == "er":
                kw["bg"] = s.bg * (s.n - 1) / (n - 1)
        if N is not None:
            kw["N"] = N
        out.append(dataclasses.replace(s, **kw))
    return dataclasses.replace(w, graphs=tuple(out))


@dataclass
class GraphDraw:
    spec: GraphSpec
    targets: np.ndarray      # int64 global ids, in pattern order
    pattern: np.ndarray      # local keys (a * t + b)


def draw_graph(ci: int, g: int, spec: GraphSpec) -> GraphDraw:
    rng = G.rng_for(ci, g, 0)
    targets = rng.choice(spec.n, size=spec.t, replace=False).astype(np.int64)
    if spec.target == "clique":
        pattern = G.complete_pattern(spec.t)
    elif spec.target == "sparse":  # int_p carries the average internal degree; hubs of degree 4
        pattern = G.sparse_target_keys(spec.t, int(round(spec.int_p * spec.t / 2)), 4, rng)
    else:
        pattern = G.er_keys(spec.t, spec.int_p, rng)
    return GraphDraw(spec, targets, pattern)


def background(ci: int, g: int, k: int, spec: GraphSpec) -> np.ndarray:
    rng = G.rng_for(ci, g, 1 + k)
    if spec.family == "er":
        return G.er_keys(spec.n, spec.bg, rng)
    if spec.family == "ws":
        return G.ws_keys(spec.n, int(spec.bg), spec.ws_beta, rng)
    if spec.family == "ba":
        return G.ba_keys(spec.n, int(spec.bg), rng)
    raise ValueError(spec.family)


def realization(ci: int, g: int, k: int, draw: GraphDraw) -> tuple[np.ndarray, np.ndarray]:
    """CSR (row_ptr, col_idx) of realization k of graph g: background k with the target embedded."""
    keys = G.embed(background(ci, g, k, draw.spec), draw.spec.n, draw.targets, draw.pattern)
    return G.csr_from_keys(keys, draw.spec.n)


@dataclass
class HostBatch:
    """Concatenated per-realization CSR arrays (realizations ordered by graph, then by k)."""
    dtype: np.dtype
    n: np.ndarray            # int32 [G]
    nreal: np.ndarray        # int32 [G]
    K: np.ndarray            # int32 [G]
    targets: list
    row_ptr: np.ndarray      # int32 [sum_r (n_r + 1)]
    col_idx: np.ndarray      # int32 [sum_r z_r]
    values: np.ndarray | None
    rowptr_off: np.ndarray   # int64 [R]
    nnz_off: np.ndarray      # int64 [R + 1]
    graph_of: np.ndarray = field(default=None)  # int32 [R]

    @property
    def R(self) -> int:
        return int(self.rowptr_off.size)

    def csr(self, r: int):
        g = int(self.graph_of[r])
        n = int(self.n[g])
        rp = self.row_ptr[self.rowptr_off[r]: self.rowptr_off[r] + n + 1]
        a, b = int(self.nnz_off[r]), int(self.nnz_off[r + 1])
        ci = self.col_idx[a:b]
        v = None if self.values is None else self.values[a:b]
        return n, rp, ci, v


def assemble(parts: list, dtype, with_values: bool = True) -> HostBatch:
    """parts: list over graphs of (spec, targets, [ (row_ptr, col_idx), ... per realization ])."""
    dt = np.dtype(np.float64 if dtype in ("f64", np.float64) else np.float32)
    rps, cis, ro, no, gof = [], [], [], [0], []
    rtot = 0
    ztot = 0
    for g, (spec, _t, reals) in enumerate(parts):
        for rp, ci in reals:
            ro.append(rtot)
            rps.append(rp)
            cis.append(ci)
            rtot += rp.size
            ztot += ci.size
            no.append(ztot)
            gof.append(g)
    col = np.concatenate(cis) if cis else np.empty(0, np.int32)
    return HostBatch(
        dtype=dt,
        n=np.array([p[0].n for p in parts], np.int32),
        nreal=np.array([len(p[2]) for p in parts], np.int32),
        K=np.array([p[0].K for p in parts], np.int32),
        targets=[p[1] for p in parts],
        row_ptr=np.concatenate(rps) if rps else np.empty(0, np.int32),
        col_idx=col,
        values=np.ones(col.size, dt) if with_values else None,
        rowptr_off=np.array(ro, np.int64),
        nnz_off=np.array(no, np.int64),
        graph_of=np.array(gof, np.int32),
    )


def build(w: Workload, with_values: bool = True, realizations: int | None = None) -> HostBatch:
    """Generate and assemble the whole workload on the host."""
    parts = []
    for g, spec in enumerate(w.graphs):
        d = draw_graph(w.ci, g, spec)
        N = spec.N if realizations is None else min(spec.N, realizations)
        parts.append((spec, d.targets, [realization(w.ci, g, k, d) for k in range(N)]))
    return assemble(parts, w.dtype, with_values)


def _gen_one(args):
    ci, g, k, draw = args
    return realization(ci, g, k, draw)


def build_parallel(w: Workload, workers: int = 8, with_values: bool = True,
                   realizations: int | None = None, progress=None) -> HostBatch:
    """build() with the realizations generated by a process pool (same seeds, same result).
    progress(done, total), if given, is called after every twentieth of the realizations."""
    import multiprocessing as mp
    draws = [draw_graph(w.ci, g, spec) for g, spec in enumerate(w.graphs)]
    jobs = []
    for g, (spec, d) in enumerate(zip(w.graphs, draws)):
        N = spec.N if realizations is None else min(spec.N, realizations)
        jobs += [(w.ci, g, k, d) for k in range(N)]
    out = []
    every = max(1, len(jobs) // 20)
    if workers > 1 and len(jobs) > 1:
        with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
            for i, res in enumerate(pool.imap(_gen_one, jobs, chunksize=1)):
                out.append(res)
                if progress is not None and (i + 1) % every == 0:
                    progress(i + 1, len(jobs))
    else:
        for i, j in enumerate(jobs):
            out.append(_gen_one(j))
            if progress is not None and (i + 1) % every == 0:
                progress(i + 1, len(jobs))
    parts = []
    i = 0
    for g, (spec, d) in enumerate(zip(w.graphs, draws)):
        N = spec.N if realizations is None else min(spec.N, realizations)
        parts.append((spec, d.targets, out[i:i + N]))
        i += N
    return assemble(parts, w.dtype, with_values)
