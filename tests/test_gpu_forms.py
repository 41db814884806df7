"""SpMV forms recorded per graph, and the autotuner's buckets and process-wide cache.

Several forms in one launch sequence (one SpMV launch per form over its graphs' row blocks) are
switched off: the first eager pass of a six-graph batch on six forms did not complete and its cause is
not found. The tests of that path stay here, skipped, for when it is enabled again: every form computes
the CSR-stream form's sums, so a batch of mixed forms must give the stream form's results bit for bit,
on every schedule, in FP32 and FP64, weighted and pattern-only, with adaptive m, the memory-bounded
two-pass form, the adjoint and the entry point that allocates nothing.
"""
import dataclasses

import numpy as np
import pytest

from fixtures import configs as C

pytestmark = pytest.mark.gpu
MIXED_OFF = pytest.mark.skip(reason="several SpMV forms in one batch are switched off: the first eager pass of "
                                    "this batch did not complete on the GPU and the cause is not found")

MIXED = ["segmented", "balanced", "paneled", "staged", ("lanes", 16, 0), "stream"]


def api():
    from paper_1409_5000_amd import api as _api
    return _api


def torch_mod():
    import torch
    return torch


def outputs(b, **kw):
    torch = torch_mod()
    print("  scores", kw, flush=True)
    out = b.scores(**kw)
    torch.cuda.synchronize()
    return out.scores.cpu().numpy().tobytes(), out.log_scale.cpu().numpy().tobytes(), out.diag_numpy().tobytes()


def six_graphs(dtype="f32", values=True, N=2, sizes=(30000, 70001, 150000, 9000, 20001, 4100)):
    """Two graphs of each family of the uneven workload, at ragged sizes (ER degree kept)."""
    w = C.workload(4)
    pick = [t for f in ("er", "ba", "ws") for t in [s for s in w.graphs if s.family == f][:2]]
    specs = tuple(dataclasses.replace(s, n=nn, N=N, bg=(s.bg * (s.n - 1) / (nn - 1) if s.family == "er" else s.bg))
                  for s, nn in zip(pick, sizes))
    return C.build(dataclasses.replace(w, graphs=specs, dtype=dtype), with_values=values)


@MIXED_OFF
@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("values", [True, False])
def test_mixed_forms_equal_stream(gpu_lib, dtype, values):
    print("  building the batch", flush=True)
    hb = six_graphs(dtype, values)
    b = api().Batch.from_host(hb)
    print("  uploaded", flush=True)
    ref = outputs(b, m=30, schedule="batched", spmv="stream")
    b.set_forms(MIXED)
    assert [f[0] for f in b.tuned_forms()] == ["segmented", "balanced", "paneled", "staged", "lanes", "stream"]
    for kw in (dict(schedule="batched", hipgraph=False), dict(schedule="batched", hipgraph=True),
               dict(schedule="plain")):
        assert outputs(b, m=30, **kw) == ref, kw
    assert outputs(b, m=30, schedule="batched") == ref  # a replay of the captured graph
    # a form named in the options overrides the recorded ones
    assert outputs(b, m=30, schedule="batched", spmv="balanced") == ref


@MIXED_OFF
def test_mixed_forms_adaptive_and_two_pass(gpu_lib):
    hb = six_graphs("f32", True)
    b = api().Batch.from_host(hb)
    ref_a = outputs(b, m=0, tol=1e-6, m_max=60, schedule="batched", spmv="stream")
    ref_2 = outputs(b, m=30, reorth=0, schedule="batched", spmv="stream")
    b.set_forms(MIXED[::-1])
    assert outputs(b, m=0, tol=1e-6, m_max=60, schedule="batched") == ref_a
    assert outputs(b, m=30, reorth=0, schedule="batched") == ref_2


@MIXED_OFF
def test_mixed_forms_adjoint(gpu_lib):
    torch = torch_mod()
    hb = six_graphs("f32", True, N=1)
    b = api().Batch.from_host(hb)
    g = torch.as_tensor(np.random.default_rng(8).normal(size=int(hb.n.sum()))).to("cuda")
    out = b.scores(m=24, schedule="batched", spmv="stream")
    ref = b.scores_backward(out.log_scale, g, m=24, spmv="stream").cpu().numpy().tobytes()
    b.set_forms(MIXED)
    out2 = b.scores(m=24, schedule="batched")
    got = b.scores_backward(out2.log_scale, g, m=24).cpu().numpy().tobytes()
    torch.cuda.synchronize()
    assert got == ref


@MIXED_OFF
def test_mixed_forms_noalloc(gpu_lib):
    torch = torch_mod()
    hb = six_graphs("f32", True, N=1, sizes=(12000, 9001, 15000, 5000, 7001, 3000))
    b = api().Batch.from_host(hb)
    b.set_forms(MIXED)
    ref = b.scores(m=16, schedule="batched", hipgraph=False)
    got = b.scores_noalloc(m=16, schedule="batched")
    torch.cuda.synchronize()
    assert np.array_equal(ref.scores.cpu().numpy(), got.scores.cpu().numpy())
    assert np.array_equal(ref.log_scale.cpu().numpy(), got.log_scale.cpu().numpy())


def test_tuner_cache_by_batch_composition(gpu_lib):
    # the batch's composition (its buckets: two ER graphs of one n-octave and degree, and a BA graph
    # whose rows reach far above its mean degree) keys one cache line; a second tune of the batch, or
    # of an equal batch after the cache text is restored, times nothing and keeps the form
    torch = torch_mod()
    _api = api()
    w = C.workload(4)
    er = [s for s in w.graphs if s.family == "er"][0]
    ba = [s for s in w.graphs if s.family == "ba"][0]
    specs = (dataclasses.replace(er, n=30000, N=2, bg=20.0 / 29999), dataclasses.replace(er, n=31001, N=2, bg=20.0 / 31000),
             dataclasses.replace(ba, n=70001, N=2))
    hb = C.build(dataclasses.replace(w, graphs=specs, dtype="f32"), with_values=True)
    b = _api.Batch.from_host(hb)
    ref = outputs(b, m=30, schedule="batched", spmv="stream")
    _api.tune_cache_clear()
    t = b.tune(m=30)
    assert t["form"] != "mixed" and len(set(t["graph_forms"])) == 1
    assert len(t["ms_per_launch"]) >= 5 and all(v > 0 for v in t["ms_per_launch"].values())
    text = _api.tune_cache_text()
    lines = text.splitlines()
    assert len(lines) == 1
    buckets = lines[0].split()[0].split("+")
    hub = sorted(int(k.split("-h")[1].split("-")[0]) for k in buckets)
    assert len(buckets) == 2 and hub[1] - hub[0] >= 3  # ER rows reach about twice the mean, BA's far more
    assert outputs(b, m=30, schedule="batched") == ref  # every form gives the stream form's bits
    t2 = b.tune(m=30)
    assert t2["ms_per_launch"] == {} and t2["graph_forms"] == t["graph_forms"]
    _api.tune_cache_clear()
    _api.tune_cache_add(text)
    b2 = _api.Batch.from_host(hb)
    t3 = b2.tune(m=30)
    assert t3["ms_per_launch"] == {} and t3["graph_forms"] == t["graph_forms"]
    assert outputs(b2, m=30, schedule="batched") == ref
    torch.cuda.synchronize()
    _api.tune_cache_clear()


def test_mixed_forms_refused(gpu_lib):
    hb = six_graphs("f32", True, N=1, sizes=(12000, 9001, 15000, 5000, 7001, 3000))
    b = api().Batch.from_host(hb)
    b.set_forms(MIXED)
    with pytest.raises(Exception, match="several SpMV forms"):
        b.scores(m=16, schedule="batched")
    b.set_forms(["balanced"] * 6)
    ref = outputs(b, m=16, schedule="batched", spmv="stream")
    assert outputs(b, m=16, schedule="batched") == ref
