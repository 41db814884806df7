"""ebtc_scores_noalloc (the library's fixed device array as the workspace) against ebtc_scores with a
caller workspace, through the C ABI: the same launches on different memory, so the outputs must agree
bit for bit (scores, log-scales, diagnostics, checkpoint), on two calls in a row with the second one
smaller, for the single-kernel and the per-phase schedules; and a batch whose workspace exceeds the
array is refused before anything runs.
"""
import ctypes

import numpy as np
import pytest

from fixtures import configs as C
from tests import graphs_small as gs
from tests.test_gpu_parity import DenseBatch, check_against_oracle

pytestmark = pytest.mark.gpu


def api():
    from paper_1409_5000_amd import api as _api
    return _api


def host(out):
    return (out.scores.cpu().numpy().copy(), out.log_scale.cpu().numpy().copy(),
            out.raw_diag.cpu().numpy().copy())


def compare(b, **kw):
    import torch
    ref = b.scores(**kw)
    torch.cuda.synchronize()
    r = host(ref)
    got = b.scores_noalloc(**kw)
    torch.cuda.synchronize()
    g = host(got)
    for x, y in zip(r, g):
        assert x.tobytes() == y.tobytes()
    return got


def test_noalloc_equals_workspace_call_twice_second_smaller(gpu_lib):
    # call 1: the plain-method workload (20 x n=200, FP64, single-kernel schedule), then a smaller batch
    # (3 x n=150): the array keeps the first call's contents, which must not leak into the second
    hb1 = C.build(C.workload(0))
    b1 = api().Batch.from_host(hb1)
    out1 = compare(b1, m=20)
    check_against_oracle(hb1, out1, b1, 20, "f64", K=10)
    hb2 = DenseBatch([[gs.random_graph(150, 0.08, 3 + k) for k in range(3)]], "f64")
    b2 = api().Batch.from_host(hb2)
    out2 = compare(b2, m=20)
    check_against_oracle(hb2, out2, b2, 20, "f64", K=10)


def test_noalloc_per_phase_schedule_and_adaptive(gpu_lib):
    # graphs beyond one row block take the per-phase schedule; FP32, adaptive m, then a smaller batch
    w = C.scaled(C.workload(1), n=9000, N=4)
    hb = C.build(w)
    b = api().Batch.from_host(hb)
    compare(b, m=0, tol=1e-6, m_max=60)
    hb2 = C.build(C.scaled(C.workload(1), n=5000, N=2))
    compare(api().Batch.from_host(hb2), m=30)


def test_noalloc_refuses_a_batch_beyond_the_array(gpu_lib):
    import torch
    from paper_1409_5000_amd import _abi as A
    w = C.scaled(C.workload(1), n=100_000, N=3)  # at m = 64: 65 basis vectors of 400 kB per realization
    hb = C.build(w)
    b = api().Batch.from_host(hb)
    ws = ctypes.c_size_t()
    opts = api().make_opts(m=64)
    A.check(A.lib().ebtc_plan(b.handle, ctypes.byref(opts), ctypes.byref(ws), None))
    assert ws.value > A.NOALLOC_WS_BYTES
    with pytest.raises(A.EbtcError) as e:
        b.scores_noalloc(m=64)
    assert e.value.status == A.EBTC_EWORKSPACE
    assert "static scratch" in str(e.value)
    torch.cuda.synchronize()
