"""The single-kernel schedule (one workgroup runs a realization's whole Lanczos process) against the
per-phase schedules, bit for bit, and against the FP64 oracle.

The single-kernel solve calls the per-phase kernels' own device functions with their thread layouts,
so scores, log-scales, diagnostics and checkpoints must equal those of the batched (one launch per
phase) and plain (one realization at a time) schedules exactly: with fixed and adaptive m, every
dot window (8, 16, 32 and 64 basis vectors), weighted and pattern-only graphs, FP32 and FP64, ragged
sizes up to the 2048-node limit and the breakdown cases of eq. (4) on regular, bipartite and empty
graphs. A graph's bits must not depend on which schedule its batch takes.
"""
import dataclasses

import numpy as np
import pytest

from fixtures import configs as C
from oracle import dense as odense
from tests import graphs_small as gs
from tests.test_gpu_parity import DenseBatch, check_against_oracle

pytestmark = pytest.mark.gpu


def api():
    from paper_1409_5000_amd import api as _api
    return _api


def torch_mod():
    import torch
    return torch


def outputs(b, **kw):
    torch = torch_mod()
    out = b.scores(ckpt=True, **kw)
    torch.cuda.synchronize()
    return (out.scores.cpu().numpy().copy(), out.log_scale.cpu().numpy().copy(), out.diag_numpy().copy(),
            out.ckpt.cpu().numpy().copy())


def assert_same(x, y):
    for a, b in zip(x, y):
        assert a.dtype == b.dtype and a.shape == b.shape
        assert a.tobytes() == b.tobytes()


def weighted(hb, seed):
    vals = np.empty(hb.col_idx.size, np.float64)
    for r in range(hb.R):
        n, rp, ci, _ = hb.csr(r)
        rows = np.repeat(np.arange(n), np.diff(rp))
        lo, hi = np.minimum(rows, ci), np.maximum(rows, ci)
        h = (lo.astype(np.int64) * 2654435761 + hi * 40503 + seed) % 1000
        vals[hb.nnz_off[r]:hb.nnz_off[r + 1]] = 0.5 + h / 1000.0
    hb.values = vals.astype(hb.dtype)
    return hb


def test_tiny_workload_schedules_bitwise_and_oracle(gpu_lib):
    # the plain-method workload (20 x n=200, FP64, m=20): single, batched (eager and replayed), plain
    w = C.workload(0)
    hb = C.build(w)
    b = api().Batch.from_host(hb)
    ref = outputs(b, m=w.m, schedule="batched", hipgraph=False)
    for kw in (dict(schedule="single", hipgraph=False), dict(schedule="single", hipgraph=True),
               dict(schedule="auto"), dict(schedule="plain")):
        assert_same(outputs(b, m=w.m, **kw), ref)
    out = b.scores(m=w.m, schedule="single")
    check_against_oracle(hb, out, b, w.m, "f64", K=10)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("valued", [False, True])
def test_every_window_ragged_sizes(gpu_lib, dtype, valued):
    # m = 40 crosses the 8-, 16-, 32- and 64-vector dot windows; sizes up to the 2048-row limit
    torch = torch_mod()
    sizes = [2048, 1999, 513, 64]
    graphs = [[gs.random_graph(n, min(0.5, 12.0 / n), 100 + n + k) for k in range(2)] for n in sizes]
    hb = DenseBatch(graphs, dtype, weighted=valued)
    if valued:
        weighted(hb, 3)
    b = api().Batch.from_host(hb)
    ref = outputs(b, m=40, schedule="batched", hipgraph=False)
    assert_same(outputs(b, m=40, schedule="single"), ref)
    assert_same(outputs(b, m=40, schedule="plain"), ref)
    for form in ("stream", "segmented", "balanced"):
        assert_same(outputs(b, m=40, schedule="batched", hipgraph=False, spmv=form), ref)
    out = b.scores(m=40, schedule="single")
    torch.cuda.synchronize()
    check_against_oracle(hb, out, b, 40, dtype, K=20)


def test_adaptive_breakdown_and_cap(gpu_lib):
    # adaptive stop (tol 1e-8, cap 60), the cap (tol 1e-14, m_max 9) and early breakdowns: a regular
    # graph and the empty graph stop after one step, a complete bipartite graph after two, the path
    # P_41 after 21
    mats = [[gs.random_graph(300, 0.05, 7), gs.random_graph(300, 0.06, 8)], [gs.complete(90)], [gs.cycle(500)],
            [gs.bipartite(7, 30)], [np.zeros((40, 40))], [gs.path(41)]]
    hb = DenseBatch(mats, "f64")
    b = api().Batch.from_host(hb)
    for kw in (dict(m=0, tol=1e-8, m_max=60), dict(m=0, tol=1e-14, m_max=9), dict(m=30)):
        ref = outputs(b, schedule="batched", hipgraph=False, **kw)
        assert_same(outputs(b, schedule="single", **kw), ref)
        d = ref[2]
        assert d["m_used"][2:6].tolist() == [1, 1, 2, 1]
        assert d["flags"][2:6].tolist() == [1, 1, 1, 1]
        if kw["m"] == 30:
            assert d["m_used"][6] == 21 and d["flags"][6] == 1
        if kw.get("m_max") == 9:
            assert d["m_used"][6] == 9 and d["flags"][6] == 2
        check_against_oracle(hb, b.scores(schedule="single", **kw), b, kw["m"], "f64", K=5,
                             tol=kw.get("tol", 0.0), m_max=kw.get("m_max", 60),
                             check_m=True if kw["m"] or kw["m_max"] == 9 else False)


def test_graph_bits_do_not_depend_on_the_batch(gpu_lib):
    # a small graph scored alone (auto: single kernel) and next to a 3000-node graph (auto: one launch
    # per phase, the fused dots-and-update kernel not applicable) gives the same bits; FP32, m = 40
    torch = torch_mod()
    small = [gs.random_graph(700, 0.02, 31), gs.random_graph(700, 0.02, 32)]
    big = [gs.random_graph(3000, 0.004, 33)]
    alone = api().Batch.from_host(DenseBatch([small], "f32"))
    mixed = api().Batch.from_host(DenseBatch([small, big], "f32"))
    a = alone.scores(m=40)
    m = mixed.scores(m=40)
    torch.cuda.synchronize()
    assert a.scores.cpu().numpy().tobytes() == m.scores[:700].cpu().numpy().tobytes()
    assert a.log_scale.cpu().numpy()[0] == m.log_scale.cpu().numpy()[0]


def test_hipgraph_replays_with_eager_work_between(gpu_lib):
    torch = torch_mod()
    hb = C.build(C.scaled(C.workload(0), N=6))
    b = api().Batch.from_host(hb)
    eager = outputs(b, m=20, schedule="single", hipgraph=False)
    run = b.run(m=20, schedule="single", hipgraph=True)
    for _ in range(4):
        out = run.launch()
        torch.cuda.synchronize()
        assert out.scores.cpu().numpy().tobytes() == eager[0].tobytes()
        _ = torch.ones(1000, device="cuda").sum().item()


def test_adjoint_after_single_kernel_forward(gpu_lib):
    # the backward recomputes the basis with the per-phase kernels; after a single-kernel forward the
    # gradient must equal the one after a per-phase forward (same log-scales, bit for bit)
    torch = torch_mod()
    hb = weighted(DenseBatch([[gs.random_graph(400, 0.03, 41), gs.random_graph(400, 0.03, 42)]], "f64",
                             weighted=True), 5)
    b = api().Batch.from_host(hb)
    g = torch.as_tensor(np.random.default_rng(3).normal(size=400)).to("cuda")
    grads = []
    for sched in ("single", "batched"):
        out = b.scores(m=24, schedule=sched)
        grads.append(b.scores_backward(out.log_scale, g, m=24).cpu().numpy().copy())
    torch.cuda.synchronize()
    assert grads[0].tobytes() == grads[1].tobytes()


def test_single_schedule_refuses_what_it_cannot_run(gpu_lib):
    hb = DenseBatch([[gs.random_graph(2049, 0.004, 1)]], "f32")
    b = api().Batch.from_host(hb)
    with pytest.raises(Exception):
        b.scores(m=10, schedule="single")
    small = api().Batch.from_host(DenseBatch([[gs.random_graph(100, 0.1, 2)]], "f32"))
    for kw in (dict(reorth=2), dict(reorth=0), dict(spmv="lanes")):
        with pytest.raises(Exception):
            small.scores(m=10, schedule="single", **kw)
        small.scores(m=10, schedule="auto", **kw)  # auto falls back to the per-phase schedule
