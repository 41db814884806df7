"""GPU parity at the workloads' full sizes, in the launch configuration the benchmark times: the batch
as one batched launch sequence replayed from a hipGraph, SpMV form chosen by the tuner (ebtc_tune).

Every realization of the batched (64 x n=1e5), single-background (3 x n=1e6) and differentiation
(16 x n=2e5) workloads is checked against the FP64 oracle, which finishes them in seconds on the
host's cores. The uneven workload's 2048 realizations (about 1e10 stored entries) take minutes to
generate on the host, so a slice of its graphs -- the largest of each family, at full size and
with all 8 realizations -- stands in for it.
"""
import dataclasses
import os

import numpy as np
import pytest

from fixtures import configs as C
from tests.parity import TOL, topk_consistent
from tests.test_gpu_parity import api, check_against_oracle, torch_mod

pytestmark = pytest.mark.gpu


def workers() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return 1


def run_tuned(hb, m, tol=1e-6, m_max=60):
    torch = torch_mod()
    b = api().Batch.from_host(hb)
    api().tune_cache_clear()  # time every bucket afresh
    t = b.tune(m=m, tol=tol, m_max=m_max)
    run = b.run(m=m, tol=tol, m_max=m_max)  # batched, hipGraph, the tuned form
    run.launch()
    out = run.launch()  # a replay
    torch.cuda.synchronize()
    return b, out, t


def check_topk(b, out, ref, K):
    idx, _ = b.topk(out.scores, K)
    idx = idx.cpu().numpy()
    off = 0
    for g, gsc in enumerate(ref):
        k = int(K[g]) if np.ndim(K) else int(K)
        ok, _ = topk_consistent(idx[off:off + k], gsc.s, k, TOL["f32"])
        assert ok, f"graph {g}: top-{k} set differs from the oracle's"
        off += k


def test_full_batched_er_n1e5_N64(gpu_lib):
    w = C.workload(1)
    hb = C.build_parallel(w, workers=workers())
    b, out, t = run_tuned(hb, w.m)
    ref, rep = check_against_oracle(hb, out, b, w.m, "f32", K=50, workers=workers())
    check_topk(b, out, ref, hb.K)
    assert out.diag_numpy()["flags"].max() == 0


def test_full_single_background_n1e6(gpu_lib):
    w = C.workload(2)
    hb = C.build_parallel(w, workers=min(3, workers()))
    b, out, t = run_tuned(hb, w.m)
    ref, rep = check_against_oracle(hb, out, b, w.m, "f32", K=30, workers=min(3, workers()))
    check_topk(b, out, ref, hb.K)


def test_full_differentiation_forward_n2e5_N16(gpu_lib):
    w = C.workload(3)
    hb = C.build_parallel(w, workers=workers())
    b, out, t = run_tuned(hb, w.m)
    ref, rep = check_against_oracle(hb, out, b, w.m, "f32", K=40, workers=workers())
    check_topk(b, out, ref, hb.K)


def test_full_uneven_slice_adaptive(gpu_lib):
    # the two largest graphs of each family of the uneven workload, at full size, N = 8, adaptive m
    w = C.workload(4)
    pick = []
    for fam in ("er", "ba", "ws"):
        idx = sorted((i for i, g in enumerate(w.graphs) if g.family == fam), key=lambda i: -w.graphs[i].n)
        pick += idx[:2]
    w = dataclasses.replace(w, graphs=tuple(w.graphs[i] for i in sorted(pick)))
    hb = C.build_parallel(w, workers=workers())
    assert hb.R == 6 * 8 and int(hb.n.max()) > 480_000
    b, out, t = run_tuned(hb, 0, tol=w.tol, m_max=w.m_max)
    ref, rep = check_against_oracle(hb, out, b, 0, "f32", K=100, tol=w.tol, m_max=w.m_max, check_m=False,
                                    workers=workers())
    d = out.diag_numpy()
    assert d["m_used"].max() <= w.m_max and (d["flags"] & 4).max() == 0  # no non-finite results
    check_topk(b, out, ref, hb.K)


def test_full_uneven_span_adaptive(gpu_lib):
    # thirty graphs of the uneven workload at their full sizes with their eight realizations, ten per
    # family spread over its n range (evenly spaced in the family's graphs sorted by n: n from about 1e4
    # to 5e5, degrees 8 to 32, clique and sparse targets); adaptive m against the oracle graph by graph
    # (scores, flags, theta*, Saad's estimate) and the top-K sets
    w = C.workload(4)
    pick = []
    for fam in ("er", "ba", "ws"):
        idx = sorted((i for i, g in enumerate(w.graphs) if g.family == fam), key=lambda i: w.graphs[i].n)
        pick += [idx[round(k * (len(idx) - 1) / 9)] for k in range(10)]
    w = dataclasses.replace(w, graphs=tuple(w.graphs[i] for i in sorted(pick)))
    hb = C.build_parallel(w, workers=workers())
    n = np.asarray(hb.n)
    assert hb.R == 240 and n.min() < 30_000 and n.max() > 450_000
    b, out, t = run_tuned(hb, 0, tol=w.tol, m_max=w.m_max)
    ref, rep = check_against_oracle(hb, out, b, 0, "f32", K=100, tol=w.tol, m_max=w.m_max, check_m=False,
                                    workers=workers())
    d = out.diag_numpy()
    assert d["m_used"].max() <= w.m_max and (d["flags"] & 4).max() == 0
    check_topk(b, out, ref, hb.K)

