"""Seeded synthetic graph generators: backgrounds, target patterns, the embedding, CSR assembly.

This module produces the inputs that both the oracle and the HIP path consume. It holds no part of
the communicability computation itself (no Krylov step, no exponential, no sum, no selection).

Paper anchors (Fioriti & Chinnici, arXiv 1409.5000):
  * backgrounds are Erdos-Renyi, small-world (Watts-Strogatz) or Barabasi-Albert graphs
    (Introduction; "Multiple backgrounds scenario"; "Single background scenario", Tables 1-3);
  * the target has a fixed topology, is placed on uniformly random nodes, and keeps its internal
    edges while its links to the background come from the background draw ("Multiple backgrounds
    scenario");
  * in the dynamic case N backgrounds are re-drawn on the same node set ("Signal processing on
    graphs", problem statement).

Readings of what the paper leaves open (each is listed in the design notes):
  * G(n, p) with p = d / (n - 1); the edge count is Binomial(n(n-1)/2, p) and, given the count, the
    edge set is uniform -- which is exactly the G(n, p) law;
  * Watts-Strogatz: ring lattice with k/2 neighbours on each side, every lattice edge's far end is
    re-drawn with probability beta to a uniform node, rejecting self-loops and duplicates;
  * Barabasi-Albert: seed star on m+1 nodes, each new node attaches m edges to endpoints drawn
    uniformly from the endpoint list of all earlier edges (degree-proportional choice, the
    Batagelj-Brandes construction); repeated picks by one node collapse to one edge;
  * embedding: background edges with both ends in the target set are removed and the fixed pattern
    is added; one placement per (configuration, graph) shared by all of its realizations.

Edges are handled as sorted unique int64 keys a*n + b with a < b.
"""
from __future__ import annotations

import numpy as np

ROOT_SEED = 14095000  # arXiv number 1409.5000


def rng_for(ci: int, g: int, slot: int) -> np.random.Generator:
    """Independent PCG64 stream for (configuration, graph, slot); slot 0 = target, 1+k = realization k."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=(ci, g, slot))))


def canon(i: np.ndarray, j: np.ndarray, n: int) -> np.ndarray:
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    return np.minimum(i, j) * n + np.maximum(i, j)


def er_keys(n: int, p: float, rng: np.random.Generator) -> np.ndarray:
    """Edge keys of G(n, p)."""
    total = n * (n - 1) // 2
    if total == 0 or p <= 0.0:
        return np.empty(0, np.int64)
    if p >= 1.0:
        a, b = np.triu_indices(n, 1)
        return canon(a, b, n)
    M = int(rng.binomial(total, p))
    keys = np.empty(0, np.int64)
    while keys.size < M:
        need = M - keys.size
        k = int(need * 1.05) + 64
        i = rng.integers(0, n, size=k)
        j = rng.integers(0, n, size=k)
        ok = i != j
        keys = np.union1d(keys, canon(i[ok], j[ok], n))
    if keys.size > M:
        keep = rng.choice(keys.size, size=M, replace=False)
        keys = np.sort(keys[keep])
    return keys


def ws_keys(n: int, k: int, beta: float, rng: np.random.Generator) -> np.ndarray:
    """Edge keys of a Watts-Strogatz small world: ring lattice of even degree k, rewiring prob beta."""
    half = k // 2
    if half < 1 or n < k + 2:
        raise ValueError("Watts-Strogatz needs k >= 2 and n > k + 1")
    src = np.repeat(np.arange(n, dtype=np.int64), half)
    dst = (src + np.tile(np.arange(1, half + 1, dtype=np.int64), n)) % n
    rew = rng.random(src.size) < beta
    keys = np.unique(canon(src[~rew], dst[~rew], n))
    s = src[rew]
    while s.size:
        t = rng.integers(0, n, size=s.size)
        cand = canon(s, t, n)
        ok = (s != t) & ~np.isin(cand, keys)
        idx_ok = np.flatnonzero(ok)
        _, first = np.unique(cand[idx_ok], return_index=True)
        accepted = np.zeros(s.size, dtype=bool)
        accepted[idx_ok[first]] = True
        keys = np.union1d(keys, cand[accepted])
        s = s[~accepted]
    return keys


def ba_keys(n: int, m: int, rng: np.random.Generator) -> np.ndarray:
    """Edge keys of a Barabasi-Albert graph with m edges per new node (seed: star on m + 1 nodes)."""
    if m < 1 or n < m + 2:
        raise ValueError("Barabasi-Albert needs m >= 1 and n >= m + 2")
    e0 = m  # seed star: centre 0, leaves 1..m
    n_new = n - (m + 1)
    E = e0 + n_new * m
    src = np.empty(E, np.int64)
    dst = np.empty(E, np.int64)
    src[:e0] = np.arange(1, m + 1)
    dst[:e0] = 0
    src[e0:] = np.repeat(np.arange(m + 1, n, dtype=np.int64), m)
    e_before = e0 + (src[e0:] - (m + 1)) * m  # edges that exist before this node arrives
    r = np.floor(rng.random(E - e0) * (2 * e_before)).astype(np.int64)
    np.minimum(r, 2 * e_before - 1, out=r)
    # Endpoint slot p: even 2e -> src[e]; odd 2e+1 -> dst[e]. dst of a non-seed edge is itself the
    # endpoint at slot r[e - e0], which is strictly earlier, so following the references ends.
    p = r.copy()
    out = np.full(E - e0, -1, np.int64)
    todo = np.arange(E - e0)
    while todo.size:
        pp = p[todo]
        e = pp >> 1
        odd = (pp & 1) == 1
        even_idx = todo[~odd]
        out[even_idx] = src[e[~odd]]
        seed_odd = odd & (e < e0)
        out[todo[seed_odd]] = dst[e[seed_odd]]
        chase = odd & (e >= e0)
        p[todo[chase]] = r[e[chase] - e0]
        todo = todo[chase]
    dst[e0:] = out
    return np.unique(canon(src, dst, n))


def complete_pattern(t: int) -> np.ndarray:
    """Local edge list (t x t keys) of the complete graph K_t."""
    a, b = np.triu_indices(t, 1)
    return canon(a, b, t)


def sparse_target_keys(t: int, edges: int, max_deg: int, rng: np.random.Generator) -> np.ndarray:
    """A connected t-node pattern with exactly `edges` edges, every degree <= max_deg and at least one
    node of degree max_deg (the sparse target of the multiple-backgrounds experiments: 20 nodes,
    average degree 2.1, hubs of degree 4; its exact topology is not published). A random tree grown
    by attaching nodes, in random order, to a uniform earlier node below the cap; then uniform extra
    edges below the cap; redrawn until some node reaches the cap."""
    if not (t - 1 <= edges <= t * max_deg // 2):
        raise ValueError("edge count out of range")
    while True:
        deg = np.zeros(t, np.int64)
        order = rng.permutation(t)
        keys = set()
        ok = True
        for idx in range(1, t):
            a = int(order[idx])
            cand = [int(b) for b in order[:idx] if deg[b] < max_deg]
            if not cand:
                ok = False
                break
            b = cand[int(rng.integers(len(cand)))]
            keys.add(min(a, b) * t + max(a, b))
            deg[a] += 1
            deg[b] += 1
        tries = 0
        while ok and len(keys) < edges and tries < 10000:
            tries += 1
            a, b = (int(v) for v in rng.integers(0, t, size=2))
            k = min(a, b) * t + max(a, b)
            if a == b or k in keys or deg[a] >= max_deg or deg[b] >= max_deg:
                continue
            keys.add(k)
            deg[a] += 1
            deg[b] += 1
        if ok and len(keys) == edges and deg.max() == max_deg:
            return np.array(sorted(keys), np.int64)


def embed(bg: np.ndarray, n: int, targets: np.ndarray, pattern_local: np.ndarray) -> np.ndarray:
    """Remove background edges inside the target set and add the fixed target pattern."""
    t = targets.size
    a = bg // n
    b = bg % n
    inside = np.zeros(n, dtype=bool)
    inside[targets] = True
    kept = bg[~(inside[a] & inside[b])]
    pa = targets[pattern_local // t]
    pb = targets[pattern_local % t]
    return np.union1d(kept, canon(pa, pb, n))


def csr_from_keys(keys: np.ndarray, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Symmetric CSR (row_ptr int32 [n+1], col_idx int32 [2E]) with sorted columns per row."""
    a = keys // n
    b = keys % n
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    order = np.argsort(rows * n + cols, kind="stable")
    rows = rows[order]
    cols = cols[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("a single realization needs fewer than 2^31 stored entries")
    return row_ptr.astype(np.int32), cols.astype(np.int32)
