"""GPU realization generator (ebtc_generate_count / ebtc_generate_fill) against the reference
generator: every drawn realization's row pointers and columns equal bit for bit (integer work), for
the three families, with and without an embedded target, at small sizes, at the edge cases, and on
sampled realizations of the n=1e5 degree-20 batch of 64 realizations; a generated batch scores like
the same CSR uploaded from the host."""
import numpy as np
import pytest

from fixtures import configs as C
from oracle import generate as ogen
from tests.test_gpu_parity import api, torch_mod

pytestmark = pytest.mark.gpu

SEED = 0x1409_5000_0F1


def check_against_oracle(family, n, count, first=0, sample=None, **kw):
    rp, ci, nnz = api().generate(family, n, count, SEED, first=first, **kw)
    rp = rp.cpu().numpy().reshape(count, n + 1)
    ci = ci.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(nnz)])
    for r in (range(count) if sample is None else sample):
        want_rp, want_ci = ogen.realization(family, n, SEED, first + r, **kw)
        assert nnz[r] == want_ci.size, (family, r, nnz[r], want_ci.size)
        assert np.array_equal(rp[r], want_rp), (family, r)
        assert np.array_equal(ci[off[r]:off[r + 1]], want_ci), (family, r)
    return rp, ci, nnz


def test_er_with_target_bitwise(gpu_lib):
    t = np.array([3, 2999, 1500, 77, 2048, 5, 6, 7, 1024, 2047, 100, 2500])
    pattern = [[i, (i + 1) % 12] for i in range(12)] + [[0, 6], [3, 9]]
    check_against_oracle("er", 3000, 4, first=7, p=0.004, targets=t, pattern=pattern)


@pytest.mark.parametrize("n,passes", [(9, 1), (10, 2), (147, 2), (148, 3)])
def test_sort_pass_boundaries_bitwise(gpu_lib, n, passes):
    # the keys (realization, a, b) take the bits of count n^2 - 1: 3 n^2 = 243, 300, 64827, 65712
    # give 8, 9, 16 and 17 bits, i.e. one, two, two and three 8-bit passes of the radix sort
    assert ((3 * n * n | 1).bit_length() + 7) // 8 == passes
    check_against_oracle("er", n, 3, p=0.3)


@pytest.mark.parametrize("n,p", [(60, 1.0), (10, 0.0), (1, 0.5), (2, 0.5), (500, 1e-17), (257, 0.9)])
def test_er_limits_bitwise(gpu_lib, n, p):
    _, _, nnz = check_against_oracle("er", n, 3, p=p)
    if p == 1.0:
        assert np.all(nnz == n * (n - 1))
    if p == 0.0 or n == 1 or p == 1e-17:
        assert np.all(nnz == 0)


@pytest.mark.parametrize("beta", [0.0, 0.1, 1.0])
def test_ws_bitwise(gpu_lib, beta):
    _, _, nnz = check_against_oracle("ws", 2000, 3, k=6, beta=beta)
    if beta == 0.0:
        assert np.all(nnz == 2000 * 6)


@pytest.mark.parametrize("m", [1, 5])
def test_ba_bitwise(gpu_lib, m):
    t = np.arange(40, 60)
    clique = [[a, b] for a in range(20) for b in range(a + 1, 20)]
    _, _, nnz = check_against_oracle("ba", 2000, 3, k=m, targets=t, pattern=clique)
    if m == 1:
        # a tree, except inside the target, which becomes a clique
        assert np.all(nnz <= 2 * (1999 + 190))


def test_benchmark_batch_sampled_bitwise(gpu_lib):
    # the n=1e5 degree-20 ER batch of 64 realizations with its 50-node target, drawn in one call
    w = C.workload(1)
    spec = w.graphs[0]
    draw = C.draw_graph(w.ci, 0, spec)
    pattern = np.stack([draw.pattern // spec.t, draw.pattern % spec.t], 1)
    _, _, nnz = check_against_oracle("er", spec.n, 64, sample=[0, 17, 63], p=spec.bg, targets=draw.targets,
                                     pattern=pattern)
    mean = spec.bg * spec.n * (spec.n - 1)
    assert abs(nnz.mean() - mean) < 0.01 * mean


def test_chunked_calls_equal_one_call(gpu_lib):
    rp1, ci1, nnz1 = api().generate("ba", 3000, 6, SEED, k=3)
    parts = [api().generate("ba", 3000, 3, SEED, first=f, k=3) for f in (0, 3)]
    assert np.array_equal(rp1.cpu().numpy(), np.concatenate([p[0].cpu().numpy() for p in parts]))
    assert np.array_equal(ci1.cpu().numpy(), np.concatenate([p[1].cpu().numpy() for p in parts]))


def test_generated_batch_scores_like_host_upload(gpu_lib):
    torch = torch_mod()
    graphs = [dict(family="er", n=5000, count=4, seed=SEED, p=12 / 4999, targets=[1, 2, 3, 4], pattern=[[0, 1], [1, 2], [2, 3]]),
              dict(family="ws", n=3000, count=2, seed=SEED + 1, k=8, beta=0.2),
              dict(family="ba", n=4000, count=3, seed=SEED + 2, k=4)]
    b = api().generated_batch(graphs, dtype="f64", chunk=2)
    assert b.R == 9 and list(b.graph_n) == [5000, 3000, 4000]
    host = api().Batch(b.graph_n, b.graph_nreal, b.rowptr_off, b.nnz_off, b.row_ptr.cpu().numpy(),
                       b.col_idx.cpu().numpy(), None, "f64")
    s1 = b.scores(m=20)
    s2 = host.scores(m=20)
    torch.cuda.synchronize()
    assert np.array_equal(s1.scores.cpu().numpy(), s2.scores.cpu().numpy())
    assert b.validate() < 0
    # and the generated realization 1 of graph 0 is the reference's
    r = 1
    rp = b.row_ptr[int(b.rowptr_off[r]):int(b.rowptr_off[r]) + 5001].cpu().numpy()
    ci = b.col_idx[int(b.nnz_off[r]):int(b.nnz_off[r + 1])].cpu().numpy()
    want_rp, want_ci = ogen.realization("er", 5000, SEED, 1, p=12 / 4999, targets=[1, 2, 3, 4],
                                        pattern=[[0, 1], [1, 2], [2, 3]])
    assert np.array_equal(rp, want_rp) and np.array_equal(ci, want_ci)
