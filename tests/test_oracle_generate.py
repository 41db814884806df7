"""Pins of the reference realization generator (oracle/generate.py) against what does not depend on
it: Philox4x32-10's published known-answer vectors, the library logarithm, brute-force pair
frequencies of G(n, p), the ring lattice, a sequential Batagelj-Brandes construction, closed forms."""
import math

import numpy as np
import pytest

from oracle import generate as gen

SEED = 0x1409_5000_5EED


@pytest.mark.parametrize("ctr,key,want", [
    ((0, 0, 0, 0), 0, (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, 0xFFFFFFFF_FFFFFFFF, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0x299F31D0 << 32) | 0xA4093822,
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
])
def test_philox_known_answers(ctr, key, want):
    # the known-answer vectors published with Philox4x32-10 (counter words 0..3, key words 0..1)
    assert tuple(int(x) for x in gen.philox4x32_10(*ctr, key)) == want


def test_exact_log_is_the_logarithm():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.random(20000), np.exp(rng.uniform(-700, 700, 20000)), [1.0, 0.5, 2.0 ** -32, 0.75]])
    got = gen.exact_log(x)
    ref = np.array([math.log(v) for v in x])
    assert np.all(np.abs(got - ref) <= 4 * np.spacing(np.abs(ref)) + 1e-300)
    assert gen.exact_log(np.float64(1.0)) == 0.0
    assert gen.exact_log(np.float64(2.0 ** 10)) == 10 * gen.LN2


def test_unit_from_word_open_interval():
    u = gen.unit_from_word(np.array([0, 1, 0xFFFFFFFF], np.uint64))
    assert u[0] == 2.0 ** -33 and u[1] == 1.5 * 2.0 ** -32 and u[2] == 1.0 - 2.0 ** -33


def test_er_pair_frequencies_and_independence():
    # every pair an edge with probability p, independently (brute force over many realizations)
    n, p, R = 8, 0.3, 3000
    A = np.zeros((R, n, n), bool)
    for r in range(R):
        k = gen.er_keys(n, p, SEED, r)
        A[r, k // n, k % n] = True
    iu = np.triu_indices(n, 1)
    freq = A[:, iu[0], iu[1]].sum(0)
    sd = math.sqrt(R * p * (1 - p))
    assert np.all(np.abs(freq - R * p) < 5 * sd)
    sd2 = math.sqrt(R * p * p * (1 - p * p))
    for (a, b), (c, d) in [((0, 1), (0, 2)), ((0, 1), (1, 2)), ((2, 3), (2, 7)), ((0, 7), (6, 7))]:
        both = int((A[:, a, b] & A[:, c, d]).sum())
        assert abs(both - R * p * p) < 5 * sd2, ((a, b), (c, d), both)


def test_er_edge_count_binomial():
    n = 20000
    p = 10.0 / (n - 1)
    N2 = n * (n - 1) // 2
    sd = math.sqrt(N2 * p * (1 - p))
    for r in range(4):
        k = gen.er_keys(n, p, SEED, r)
        assert abs(k.size - N2 * p) < 5 * sd
        a, b = k // n, k % n
        assert np.all(a < b) and np.all(np.diff(k) > 0)


def test_er_limits_and_reproducibility():
    n = 9
    assert gen.er_keys(n, 1.0, SEED, 0).size == n * (n - 1) // 2
    assert gen.er_keys(n, 0.0, SEED, 0).size == 0
    assert gen.er_keys(n, 1e-17, SEED, 0).size == 0
    a = gen.er_keys(500, 0.05, SEED, 3)
    assert np.array_equal(a, gen.er_keys(500, 0.05, SEED, 3))
    assert not np.array_equal(a, gen.er_keys(500, 0.05, SEED, 4))
    assert not np.array_equal(a, gen.er_keys(500, 0.05, SEED + 1, 3))


def test_ws_lattice_and_rewiring():
    n, k = 200, 6
    lat = gen.ws_keys(n, k, 0.0, SEED, 0)
    want = np.unique(gen.canon(np.repeat(np.arange(n), 3), (np.repeat(np.arange(n), 3) + np.tile([1, 2, 3], n)) % n, n))
    assert np.array_equal(lat, want)
    beta, tot, R = 0.3, 0, 20
    for r in range(R):
        kk = gen.ws_keys(n, k, beta, SEED, r)
        tot += np.setdiff1d(kk, want).size        # edges off the lattice
        a, b = kk // n, kk % n
        assert np.all(a != b) and kk.size <= n * 3
    E = R * n * 3
    # a rewired edge lands off the lattice unless its new end is one of the 2h lattice neighbours
    mean = E * beta * (1 - (k - 1) / (n - 1))
    assert abs(tot - mean) < 5 * math.sqrt(E * beta * (1 - beta)) + 0.01 * mean


def test_ba_chase_equals_sequential_construction():
    # Batagelj-Brandes with the same slot draws, built slot by slot in order
    n, m = 300, 3
    for r in range(3):
        E = m + (n - m - 1) * m
        e = np.arange(E)
        u = np.where(e < m, e + 1, m + 1 + (e - m) // m)
        eb = np.where(e < m, 0, m + (u - m - 1) * m)
        w = gen.philox4x32_10(e, 0, r, gen.TAG_BA, SEED)
        M = []
        for f in range(E):
            if f < m:
                M += [f + 1, 0]
            else:
                X = (int(w[0][f]) << 32) | int(w[1][f])
                slot = (X * 2 * int(eb[f])) >> 64
                M += [int(u[f]), M[slot]]
        want = np.unique(gen.canon(M[0::2], M[1::2], n))
        assert np.array_equal(gen.ba_keys(n, m, SEED, r), want)


def test_ba_tree_and_first_attachment():
    n = 400
    k = gen.ba_keys(n, 1, SEED, 0)
    assert k.size == n - 1
    parent = np.arange(n)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for a, b in zip(k // n, k % n):
        parent[find(a)] = find(b)
    assert len({find(v) for v in range(n)}) == 1
    # node m + 1's first edge picks the centre (degree m of 2m endpoint slots) with probability 1/2
    m, R = 4, 4000
    e = np.full(R, m)
    w = gen.philox4x32_10(e, 0, np.arange(R), gen.TAG_BA, SEED)
    slots = gen.mulhi_range(w[0], w[1], np.full(R, 2 * m))
    hits = int(np.sum(slots % 2 == 1))
    assert abs(hits - R / 2) < 5 * math.sqrt(R / 4)
    assert np.all((slots >= 0) & (slots < 2 * m))


def test_embedding_and_csr():
    n = 60
    keys = gen.er_keys(n, 0.2, SEED, 1)
    targets = np.array([5, 17, 42, 3])
    pattern = np.array([[0, 1], [1, 2], [2, 3]])
    out = gen.embed(keys, n, targets, pattern)
    inside = np.isin(out // n, targets) & np.isin(out % n, targets)
    assert np.array_equal(np.sort(out[inside]), np.sort(gen.canon([5, 17, 42], [17, 42, 3], n)))
    outside_before = keys[~(np.isin(keys // n, targets) & np.isin(keys % n, targets))]
    assert np.array_equal(out[~inside], outside_before)
    rp, ci = gen.csr(out, n)
    D = np.zeros((n, n), bool)
    D[out // n, out % n] = True
    D |= D.T
    assert rp[-1] == 2 * out.size
    for i in range(n):
        row = ci[rp[i]:rp[i + 1]]
        assert np.array_equal(row, np.flatnonzero(D[i]))
