"""The paneled SpMV form (entries sorted by column panel once per call; a products pass with one vector
slice in LDS per panel and group of row blocks, then a row-sum pass in entry order) against the
CSR-stream form, bit for bit, through the whole Lanczos path, and against the FP64 oracle.

Covers ragged sizes (n not a multiple of the panel or of the 2048-row block), weighted and
pattern-only graphs in FP32 and FP64, batches of graphs of different sizes, the plain, batched and
replayed schedules, adaptive m, the adjoint, and the row blocks the form leaves unsorted (more entries
than the row-sum pass holds, or a row beyond the stream form's capacity), which take the stream
arithmetic inside the row-sum pass.
"""
import dataclasses

import numpy as np
import pytest

from fixtures import configs as C, graphs as G
from tests.test_gpu_parity import check_against_oracle

pytestmark = pytest.mark.gpu


def api():
    from paper_1409_5000_amd import api as _api
    return _api


def torch_mod():
    import torch
    return torch


def outputs(b, **kw):
    torch = torch_mod()
    out = b.scores(**kw)
    torch.cuda.synchronize()
    return out.scores.cpu().numpy().tobytes(), out.log_scale.cpu().numpy().tobytes(), out.diag_numpy().tobytes()


def uneven(dtype="f32", values=True, N=2):
    w = C.workload(4)
    pick = [s for f in ("er", "ba", "ws") for s in [t for t in w.graphs if t.family == f][:1]]
    sizes = [30000, 70001, 150000]
    specs = tuple(dataclasses.replace(s, n=nn, N=N, bg=(s.bg * (s.n - 1) / (nn - 1) if s.family == "er" else s.bg))
                  for s, nn in zip(pick, sizes))
    return C.build(dataclasses.replace(w, graphs=specs, dtype=dtype), with_values=values)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("values", [True, False])
def test_paneled_equals_stream_uneven(gpu_lib, dtype, values):
    hb = uneven(dtype, values)
    b = api().Batch.from_host(hb)
    ref = outputs(b, m=30, schedule="batched", spmv="stream")
    for kw in (dict(schedule="batched", hipgraph=False), dict(schedule="batched", hipgraph=True),
               dict(schedule="plain")):
        assert outputs(b, m=30, spmv="paneled", **kw) == ref
    # a narrower panel: more panels per realization and ragged last panels
    assert outputs(b, m=30, spmv="paneled", seg_len=4000, schedule="batched") == ref


def test_paneled_adaptive_and_oracle(gpu_lib):
    hb = uneven("f32", True, N=2)
    b = api().Batch.from_host(hb)
    ref = outputs(b, m=0, tol=1e-6, m_max=60, schedule="batched", spmv="stream")
    out = b.scores(m=0, tol=1e-6, m_max=60, schedule="batched", spmv="paneled")
    torch_mod().cuda.synchronize()
    assert (out.scores.cpu().numpy().tobytes(), out.log_scale.cpu().numpy().tobytes(),
            out.diag_numpy().tobytes()) == ref
    check_against_oracle(hb, out, b, 0, "f32", K=20, tol=1e-6, m_max=60, check_m=False, workers=8)


def test_paneled_unsorted_blocks(gpu_lib):
    # hub rows of 7000 entries (beyond the stream form's 6144-product capacity) and a dense region
    # whose row blocks exceed the row-sum pass's 32768 products: those blocks stay unsorted
    n = 60000
    rng = np.random.default_rng(9)
    keys = G.er_keys(n, 6.0 / (n - 1), G.rng_for(12, 1, 1))
    extra = [G.canon(np.full(7000, h), rng.choice(n, 7000, replace=False), n) for h in (5, 7001, 59999)]
    dense = rng.integers(20480, 22528, size=(60000, 2))  # about 30 entries per row in one row block
    extra.append(G.canon(dense[:, 0], dense[:, 1], n))
    keys = np.unique(np.concatenate([keys] + extra))
    keys = keys[(keys // n) != (keys % n)]
    rp, ci = G.csr_from_keys(keys, n)

    class HB:
        pass
    hb = HB()
    hb.dtype = np.float32
    hb.n = np.array([n], np.int32)
    hb.nreal = np.array([1], np.int32)
    hb.row_ptr = rp.astype(np.int32)
    hb.col_idx = ci.astype(np.int32)
    hb.values = (0.5 + rng.random(ci.size)).astype(np.float32)
    hb.rowptr_off = np.zeros(1, np.int64)
    hb.nnz_off = np.array([0, ci.size], np.int64)
    hb.graph_of = np.zeros(1, np.int32)
    hb.csr = lambda r: (n, hb.row_ptr, hb.col_idx, hb.values)
    assert np.max(np.diff(rp)) > 6144
    b = api().Batch.from_host(hb)
    ref = outputs(b, m=20, schedule="batched", spmv="stream")
    assert outputs(b, m=20, schedule="batched", spmv="paneled") == ref


def test_paneled_adjoint_equals_stream(gpu_lib):
    torch = torch_mod()
    hb = uneven("f32", True, N=1)
    b = api().Batch.from_host(hb)
    g = torch.as_tensor(np.random.default_rng(4).normal(size=int(hb.n.sum()))).to("cuda")
    grads = []
    for form in ("stream", "paneled"):
        out = b.scores(m=24, schedule="batched", spmv=form)
        grads.append(b.scores_backward(out.log_scale, g, m=24, spmv=form).cpu().numpy().tobytes())
    torch.cuda.synchronize()
    assert grads[0] == grads[1]


def test_tuner_times_the_paneled_form(gpu_lib):
    hb = uneven("f32", True, N=1)
    b = api().Batch.from_host(hb)
    api().tune_cache_clear()  # time every bucket afresh
    t = b.tune(m=30)
    assert "paneled" in t["ms_per_launch"] and t["ms_per_launch"]["paneled"] > 0
