"""Reference realization generator (test infrastructure: only the tests, the smoke check and the
benchmark's CPU leg use this package).

The step before the path: background graphs of the families in the paper's experiments
(Erdos-Renyi G(n, p), Watts-Strogatz small world, Barabasi-Albert: Introduction, "Multiple
backgrounds scenario", "Single background scenario", Tables 1-3), N independent draws on one node
set ("Signal processing on graphs": the dynamic background), the fixed target pattern embedded on
given nodes (edges among target nodes replaced by the pattern), as symmetric CSR with sorted columns
and no self-loops. Plain numpy; the device generator implements the same definitions.

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC 2011), key = the 64-bit seed (low word, high word), counter = (c0, c1, realization
index, family tag). Every draw is a pure function of its counter, so rows, edges and realizations
can be drawn in any order.

Definitions (realization r, n nodes):
  ER   row i visits the columns j > i by geometric skips: from j = i the next edge is at
       j + 1 + G, G = floor(ln U / ln(1 - p)), U = (w + 1/2) 2^-32, w the next word of row i's
       stream (counters (i, c, r, 1), c = 0, 1, ..., words w0..w3 in order); the row ends when the
       position would reach n. P(G >= g) = (1 - p)^g, so each pair is an edge independently with
       probability p. p = 1: every pair; p = 0 or 1 - p == 1 in FP64: no pair.
       ln is `exact_log`: frexp and the atanh series, with correctly rounded +, -, *, / only, so
       every IEEE double implementation of the same operations gets the same bits.
  WS   lattice edge e = (i, i + s mod n), i = e div h, s = 1 + e mod h, h = k / 2; with words of
       counter (e, 0, r, 2): rewired iff w0 < floor(beta 2^32), new far end
       (i + 1 + floor(w1 (n - 1) / 2^32)) mod n (uniform over the other n - 1 nodes); edges that
       coincide are kept once.
  BA   seed star: edges e < m join leaf e + 1 to centre 0; edge e >= m belongs to node
       u = m + 1 + (e - m) div m and picks endpoint slot R_e = floor(X (2 E_u) / 2^64) of the
       2 E_u slots of the E_u = m + (u - m - 1) m earlier edges (slot 2f: the new node of edge f,
       slot 2f + 1: the node edge f attached to), X = w0 2^32 + w1 from counter (e, 0, r, 3):
       degree-proportional choice (Batagelj and Brandes' construction). A node's repeated picks
       collapse to one edge.
  embedding  edges with both ends among the target nodes are dropped and the pattern's edges
       (local pairs mapped through `targets`) are added.
"""
from __future__ import annotations

import numpy as np

TAG_ER, TAG_WS, TAG_BA = 1, 2, 3
_M32 = np.uint64(0xFFFFFFFF)
_PHILOX_M = (np.uint64(0xD2511F53), np.uint64(0xCD9E8D57))
_PHILOX_W = (np.uint64(0x9E3779B9), np.uint64(0xBB67AE85))

SQRT_HALF = 0.70710678118654752440
LN2 = 0.69314718055994530942
LOG_TERMS = 11                                           # atanh series: s, s^3/3, ..., s^21/21
LOG_COEF = tuple(1.0 / (2 * k + 1) for k in range(LOG_TERMS))


def philox4x32_10(c0, c1, c2, c3, seed: int):
    """Philox4x32-10 of counters (c0, c1, c2, c3) (arrays or scalars < 2^32) under the 64-bit seed.
    Each round: (hi0, lo0) = M0 c0, (hi1, lo1) = M1 c2 (32 x 32 -> 64-bit products),
    c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key gains the Weyl increments between rounds."""
    c = [np.asarray(x, dtype=np.uint64) & _M32 for x in np.broadcast_arrays(c0, c1, c2, c3)]
    k0, k1 = np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _PHILOX_W[0]) & _M32
            k1 = (k1 + _PHILOX_W[1]) & _M32
        p0 = _PHILOX_M[0] * c[0]
        p1 = _PHILOX_M[1] * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & _M32, p1 & _M32, ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & _M32,
             p0 & _M32]
    return c


def exact_log(x):
    """Natural logarithm of x > 0: x = m 2^e with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s),
    s = (m - 1) / (m + 1), series in s^2 by Horner, then e ln 2 + (2 s) q. Only correctly rounded
    operations, in this order, with no fused multiply-add."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    low = m < SQRT_HALF
    m = np.where(low, m * 2.0, m)
    e = np.where(low, e - 1, e)
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    q = np.full_like(s, LOG_COEF[-1])
    for k in range(LOG_TERMS - 2, -1, -1):
        q = q * z
        q = q + LOG_COEF[k]
    return e.astype(np.float64) * LN2 + (2.0 * s) * q


def unit_from_word(w):
    """U = (w + 1/2) 2^-32 in (0, 1), exact in FP64."""
    return (np.asarray(w, dtype=np.uint64).astype(np.float64) + 0.5) * (2.0 ** -32)


def canon(a, b, n: int) -> np.ndarray:
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    return np.minimum(a, b) * n + np.maximum(a, b)


def er_keys(n: int, p: float, seed: int, r: int) -> np.ndarray:
    """Sorted edge keys a * n + b (a < b) of realization r of G(n, p)."""
    if n < 2 or p <= 0.0 or 1.0 - p == 1.0:
        return np.empty(0, np.int64)
    if p >= 1.0:
        a, b = np.triu_indices(n, 1)
        return canon(a, b, n)
    q = float(exact_log(np.float64(1.0 - p)))
    rows = np.arange(n - 1, dtype=np.int64)
    pos = rows.copy()                        # last visited column of each row
    active = np.ones(rows.size, bool)
    out = []
    c = 0
    while active.any():
        idx = np.flatnonzero(active)
        words = philox4x32_10(rows[idx], c, r, TAG_ER, seed)
        for w in words:                      # w0, w1, w2, w3 in order
            live = active[idx]
            g = np.floor(exact_log(unit_from_word(w)) / q)
            room = (n - 1 - pos[idx]).astype(np.float64)
            ok = live & (g < room)
            stop = live & ~ok
            active[idx[stop]] = False
            sel = idx[ok]
            pos[sel] = pos[sel] + 1 + g[ok].astype(np.int64)
            out.append(rows[sel] * n + pos[sel])
        c += 1
    return np.sort(np.concatenate(out)) if out else np.empty(0, np.int64)


def ws_keys(n: int, k: int, beta: float, seed: int, r: int) -> np.ndarray:
    """Sorted unique edge keys of realization r of the Watts-Strogatz small world (even k)."""
    h = k // 2
    if h < 1 or n < k + 2:
        raise ValueError("Watts-Strogatz needs an even k >= 2 and n >= k + 2")
    e = np.arange(n * h, dtype=np.int64)
    i = e // h
    far = (i + 1 + e % h) % n
    w = philox4x32_10(e, 0, r, TAG_WS, seed)
    thr = int(np.floor(beta * 4294967296.0))
    rew = w[0].astype(np.int64) < thr
    new = (i + 1 + ((w[1] * np.uint64(n - 1)) >> np.uint64(32)).astype(np.int64)) % n
    return np.unique(canon(i, np.where(rew, new, far), n))


def mulhi_range(w0, w1, R):
    """floor(X R / 2^64) for X = w0 2^32 + w1 and 0 < R < 2^32 (exact in 64-bit integers)."""
    R = np.asarray(R, dtype=np.uint64)
    lo = (np.asarray(w1, np.uint64) * R) >> np.uint64(32)
    return ((np.asarray(w0, np.uint64) * R + lo) >> np.uint64(32)).astype(np.int64)


def ba_keys(n: int, m: int, seed: int, r: int) -> np.ndarray:
    """Sorted unique edge keys of realization r of the Barabasi-Albert graph (m edges per new node)."""
    if m < 1 or n < m + 2:
        raise ValueError("Barabasi-Albert needs m >= 1 and n >= m + 2")
    E = m + (n - m - 1) * m
    e = np.arange(E, dtype=np.int64)
    new_node = np.where(e < m, e + 1, m + 1 + (e - m) // m)
    e_before = np.where(e < m, 0, m + (new_node - m - 1) * m)   # edges present when edge e is drawn
    w = philox4x32_10(e, 0, r, TAG_BA, seed)
    slot = mulhi_range(w[0], w[1], 2 * e_before)      # meaningful for e >= m
    end = np.full(E, -1, np.int64)
    end[:m] = 0                                       # seed star: leaves attach to the centre
    todo = np.arange(m, E)
    cur = slot[todo].copy()
    while todo.size:
        f = cur >> 1
        even = (cur & 1) == 0
        end[todo[even]] = new_node[f[even]]           # slot 2f: the new node of edge f
        seed_odd = ~even & (f < m)
        end[todo[seed_odd]] = 0                       # slot 2f + 1 of a seed edge: the centre
        chase = ~even & (f >= m)                      # slot 2f + 1: where edge f attached, its own slot
        cur = slot[f[chase]]
        todo = todo[chase]
    return np.unique(canon(new_node, end, n))


def embed(keys: np.ndarray, n: int, targets, pattern) -> np.ndarray:
    """Drop edges with both ends in `targets`, add the pattern's edges (local pairs (a, b))."""
    targets = np.asarray(targets, dtype=np.int64)
    if targets.size == 0:
        return keys
    inside = np.zeros(n, bool)
    inside[targets] = True
    kept = keys[~(inside[keys // n] & inside[keys % n])]
    pat = np.asarray(pattern, dtype=np.int64).reshape(-1, 2)
    return np.unique(np.concatenate([kept, canon(targets[pat[:, 0]], targets[pat[:, 1]], n)]))


def csr(keys: np.ndarray, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Symmetric CSR (row_ptr int32 [n + 1], col_idx int32) with sorted columns."""
    a, b = keys // n, keys % n
    directed = np.sort(np.concatenate([a * n + b, b * n + a]))
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(directed // n, minlength=n), out=row_ptr[1:])
    return row_ptr.astype(np.int32), (directed % n).astype(np.int32)


def realization(family: str, n: int, seed: int, r: int, p: float = 0.0, k: int = 0, beta: float = 0.0,
                targets=(), pattern=()) -> tuple[np.ndarray, np.ndarray]:
    """CSR of realization r: the background of `family` ("er", "ws", "ba") with the target embedded."""
    if family == "er":
        keys = er_keys(n, p, seed, r)
    elif family == "ws":
        keys = ws_keys(n, k, beta, seed, r)
    elif family == "ba":
        keys = ba_keys(n, k, seed, r)
    else:
        raise ValueError(family)
    return csr(embed(keys, n, targets, pattern), n)
