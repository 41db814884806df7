"""GPU parity of the column-segmented SpMV form against the CSR-stream form and the FP64 oracle.

The segmented form adds each row's products segment by segment, in entry order inside a segment;
for rows stored with ascending columns (every fixture here) that is the stream form's order, so
the whole Lanczos path must agree with the stream form bit for bit -- scores, log-scales, m_used.
Row blocks the sort cannot take (more than 65535 entries, or a row with more than 255 entries in
one segment) run the stream arithmetic inside the same kernel and must agree bit for bit as well.
"""
import dataclasses

import numpy as np
import pytest

from fixtures import configs as C, graphs as G
from tests.test_gpu_parity import api, check_against_oracle, torch_mod

pytestmark = pytest.mark.gpu


def symmetric_weights(hb, seed=0):
    """Deterministic symmetric weights in [0.5, 1.5): w(i, j) depends on the unordered pair only."""
    vals = np.empty(hb.col_idx.size, np.float64)
    for r in range(hb.R):
        n, rp, ci, _ = hb.csr(r)
        rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
        lo, hi = np.minimum(rows, ci), np.maximum(rows, ci)
        h = (lo * 1_000_003 + hi * 7919 + seed) % 1024
        a = int(hb.nnz_off[r])
        vals[a:a + ci.size] = 0.5 + h / 1024.0
    return vals.astype(hb.dtype)


def seg_eligible(hb, seg_len, dtype):
    """Fraction of row blocks that take the sorted path, by the rules of the prepare kernel: its entries
    and the padding of its wave bands (up to 3 slots per band) within 65535 slots, 255 entries of one
    row in one segment, and a wave band's (128 rows') entries in one segment, padded to a multiple of
    four, within its product slots (768 FP32 / 384 FP64)."""
    seg = seg_len or (6144 if dtype == "f64" else 12288)
    wcap = 384 if dtype == "f64" else 768
    ok = tot = 0
    for r in range(hb.R):
        n, rp, ci, _ = hb.csr(r)
        rows_of = np.repeat(np.arange(n), np.diff(rp))
        for b0 in range(0, n, 2048):
            b1 = min(n, b0 + 2048)
            sl = slice(int(rp[b0]), int(rp[b1]))
            tot += 1
            S = (n + seg - 1) // seg
            if rp[b1] - rp[b0] + 3 * 16 * S > 65535:
                continue
            sg, rw = ci[sl] // seg, rows_of[sl] - b0
            per_row = np.bincount(sg * 2048 + rw, minlength=S * 2048)
            per_band = np.bincount(sg * 16 + rw // 128, minlength=S * 16)
            ok += int(per_row.max(initial=0) <= 255 and ((per_band + 3) // 4 * 4).max(initial=0) <= wcap)
    return ok / tot


def run_pair(hb, m, **seg_kw):
    torch = torch_mod()
    b = api().Batch.from_host(hb)
    ref = b.scores(m=m, spmv="stream")
    seg = b.scores(m=m, spmv="segmented", **seg_kw)
    torch.cuda.synchronize()
    return b, ref, seg


def assert_bitwise(ref, seg):
    assert np.array_equal(ref.scores.cpu().numpy(), seg.scores.cpu().numpy())
    assert np.array_equal(ref.log_scale.cpu().numpy(), seg.log_scale.cpu().numpy())
    dr, ds = ref.diag_numpy(), seg.diag_numpy()
    assert np.array_equal(dr["m_used"], ds["m_used"]) and np.array_equal(dr["flags"], ds["flags"])


@pytest.mark.parametrize("dtype,seg_len", [("f32", 500), ("f32", 1000), ("f32", 4096), ("f32", 0), ("f64", 400),
                                           ("f64", 777), ("f64", 0)])
@pytest.mark.parametrize("weighted", [False, True])
def test_segmented_equals_stream_bitwise(gpu_lib, dtype, seg_len, weighted):
    # n = 9000: four full row blocks and a ragged one of 808 rows; seg_len 500 / 1000 / 400 / 777
    # give 18 / 9 / 23 / 12 segments with a ragged last one, every block sorted; 4096 and the
    # defaults put up to 2560 entries of a wave's rows into one segment, beyond its product slots:
    # every block runs the stream arithmetic inside the segmented kernel
    w = dataclasses.replace(C.scaled(C.workload(1), n=9000, N=3), dtype=dtype)
    hb = C.build(w, with_values=weighted)
    if weighted:
        hb.values = symmetric_weights(hb)
    assert seg_eligible(hb, seg_len, dtype) == (1.0 if seg_len in (500, 1000, 400, 777) else 0.0)
    b, ref, seg = run_pair(hb, w.m, seg_len=seg_len)
    assert_bitwise(ref, seg)
    if seg_len == 0:
        check_against_oracle(hb, seg, b, w.m, dtype, K=50)


@pytest.mark.parametrize("seg_len", [1001, 2003])
def test_segmented_fp32_ragged_slices_bitwise(gpu_lib, seg_len):
    # FP32 with an odd n and segment lengths that are not multiples of four: the vector slice loads
    # and stores one element at a time, the last block (809 rows) is odd, its pad row counts nothing
    w = dataclasses.replace(C.scaled(C.workload(1), n=9001, N=2), dtype="f32")
    hb = C.build(w, with_values=True)
    hb.values = symmetric_weights(hb, seed=3)
    assert seg_eligible(hb, seg_len, "f32") == 1.0
    b, ref, seg = run_pair(hb, w.m, seg_len=seg_len)
    assert_bitwise(ref, seg)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_segmented_rows_not_ascending(gpu_lib, dtype):
    # rows stored with their columns in no order: the sort keeps each row's stored order within a
    # segment, so the sums (segment by segment) differ from the stream form's in their order only and
    # agree with it and with the oracle to the working precision
    w = dataclasses.replace(C.scaled(C.workload(1), n=9000, N=2), dtype=dtype)
    hb = C.build(w, with_values=True)
    hb.values = symmetric_weights(hb, seed=7)
    rng = np.random.default_rng(5)
    for r in range(hb.R):
        n, rp, ci, _ = hb.csr(r)
        a = int(hb.nnz_off[r])
        for i in range(n):
            k0, k1 = a + int(rp[i]), a + int(rp[i + 1])
            perm = k0 + rng.permutation(k1 - k0)
            hb.col_idx[k0:k1] = hb.col_idx[perm]
            hb.values[k0:k1] = hb.values[perm]
    b, ref, seg = run_pair(hb, w.m, seg_len=1000)
    tol = 1e-12 if dtype == "f64" else 1e-5
    r_, s_ = ref.scores.cpu().numpy(), seg.scores.cpu().numpy()
    assert np.max(np.abs(r_ - s_)) <= tol * np.max(np.abs(r_))
    check_against_oracle(hb, seg, b, w.m, dtype, K=50)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_segmented_large_segments_prefetched_bitwise(gpu_lib, dtype):
    # n = 40000, degree 8: the default segment (12288 FP32 / 6144 FP64 columns, two LDS buffers)
    # holds about 315 / 157 entries of a wave's 128 rows, within its product slots
    spec = C.er_spec(40000, 8.0, target="er", t=50, int_p=4 / 49, N=2, K=50)
    w = C.Workload(92, "segmented-large", (spec,), dtype, 20)
    hb = C.build(w)
    assert seg_eligible(hb, 0, dtype) == 1.0
    b, ref, seg = run_pair(hb, w.m)
    assert_bitwise(ref, seg)


def test_segmented_fallback_blocks_bitwise(gpu_lib):
    # graph 0: BA hubs put hundreds of one row's entries into one segment (those blocks fall back);
    # graph 1: ER degree ~34 puts more than 65535 entries into a full row block (falls back) while
    # its ragged last block (1904 rows) stays under the limit and is sorted
    specs = (C.GraphSpec("ba", 20000, 10, "clique", 20, N=2, K=20),
             C.er_spec(6000, 34.0, target="er", t=20, int_p=0.2, N=2, K=20))
    w = C.Workload(91, "segmented-fallback", specs, "f32", 25)
    hb = C.build(w, with_values=False)
    deg = np.diff(hb.csr(0)[1])
    assert deg.max() > 255
    rp1 = hb.csr(2)[1]
    assert rp1[2048] - rp1[0] > 65535 and rp1[6000] - rp1[4096] <= 65535
    assert 0.0 < seg_eligible(hb, 4096, "f32") < 1.0
    b, ref, seg = run_pair(hb, w.m, seg_len=4096)
    assert_bitwise(ref, seg)
    check_against_oracle(hb, seg, b, w.m, "f32", K=20)


@pytest.mark.parametrize("schedule,hipgraph", [("plain", False), ("batched", True)])
def test_segmented_schedules_and_replays(gpu_lib, schedule, hipgraph):
    torch = torch_mod()
    w = C.scaled(C.workload(1), n=12000, N=4)
    hb = C.build(w)
    b = api().Batch.from_host(hb)
    ref = b.scores(m=w.m, spmv="stream", schedule="batched", hipgraph=False)
    run = b.run(m=w.m, spmv="segmented", seg_len=3000, schedule=schedule, hipgraph=hipgraph)
    outs = []
    for _ in range(3):  # replays with eager work between them
        o = run.launch()
        torch.cuda.synchronize()
        outs.append(o.scores.cpu().numpy().copy())
        torch.zeros(1 << 20, device="cuda").sum().item()
    r = ref.scores.cpu().numpy()
    for o in outs:
        assert np.array_equal(o, r)


def test_segmented_adaptive_and_uneven(gpu_lib):
    # adaptive m with early stops: stopped realizations skip the step inside the segmented kernel too
    w = C.scaled(C.workload(4), graphs=slice(0, 3))
    specs = [dict(n=2500, N=2), dict(n=1100, N=3), dict(n=4097, N=1)]
    w = dataclasses.replace(w, graphs=tuple(dataclasses.replace(s, **kw) if s.family != "er" else
                                            dataclasses.replace(s, bg=s.bg * (s.n - 1) / (kw["n"] - 1), **kw)
                                            for s, kw in zip(w.graphs, specs)))
    hb = C.build(w)
    torch = torch_mod()
    b = api().Batch.from_host(hb)
    ref = b.scores(m=0, tol=w.tol, m_max=w.m_max, spmv="stream")
    seg = b.scores(m=0, tol=w.tol, m_max=w.m_max, spmv="segmented", seg_len=1024)
    torch.cuda.synchronize()
    assert_bitwise(ref, seg)


def test_segmented_backward_equals_stream(gpu_lib):
    torch = torch_mod()
    w = C.scaled(C.workload(3), n=6000, N=3)
    hb = C.build(w)
    hb.values = symmetric_weights(hb, seed=5)
    b = api().Batch.from_host(hb)
    fwd = b.scores(m=w.m)
    g = torch.linspace(-1.0, 1.0, fwd.scores.numel(), device="cuda", dtype=fwd.scores.dtype)
    g_ref = b.scores_backward(fwd.log_scale, g, m=w.m, spmv="stream").cpu().numpy()
    g_seg = b.scores_backward(fwd.log_scale, g, m=w.m, spmv="segmented", seg_len=2000).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(g_ref, g_seg)


def test_segmented_rejects_too_many_segments(gpu_lib):
    from paper_1409_5000_amd import _abi as A
    w = C.scaled(C.workload(1), n=9000, N=1)
    b = api().Batch.from_host(C.build(w))
    with pytest.raises(A.EbtcError, match="segments"):
        b.scores(m=5, spmv="segmented", seg_len=256)  # 36 segments > 32
