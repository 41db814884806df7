"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every function the header
declares, validates descriptors and options with the documented status codes, reports workspace
sizes that match the documented layout, and keeps ebtc_last_error in step. No compute call is made.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1409_5000_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE_DEV = 0x7F0000000000  # never dereferenced by host-only calls


def header_functions():
    text = open(os.path.join(ROOT, "include", "ebtc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ebtc_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = A.lib()
    names = header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), f"{name} declared in ebtc.h but not exported"
    assert sorted(A.EXPORTED) == names


def test_version_and_status_strings():
    a, b = ctypes.c_int(), ctypes.c_int()
    assert A.lib().ebtc_version(ctypes.byref(a), ctypes.byref(b)) == 0 and (a.value, b.value) == (0, 1)
    assert A.lib().ebtc_version(None, None) == A.EBTC_EINVAL
    for s in range(6):
        assert A.lib().ebtc_status_str(s)
    assert A.lib().ebtc_status_str(99) == b"unknown status"


def make_desc(G=1, nreal=(3,), n=(10,), nnz=(20, 20, 20), dtype=A.EBTC_F32, keep=None):
    keep = [] if keep is None else keep
    gn = np.array(n, np.int32)
    gr = np.array(nreal, np.int32)
    R = int(gr.sum())
    ro = np.zeros(R, np.int64)
    acc = 0
    r = 0
    for g in range(G):
        for _ in range(gr[g]):
            ro[r] = acc
            acc += gn[g] + 1
            r += 1
    no = np.concatenate([[0], np.cumsum(np.array(nnz, np.int64))]).astype(np.int64)
    keep += [gn, gr, ro, no]
    i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    d = A.BatchDesc(dtype, G, R, gn.ctypes.data_as(i32p), gr.ctypes.data_as(i32p), ro.ctypes.data_as(i64p),
                    no.ctypes.data_as(i64p), FAKE_DEV, FAKE_DEV + 4096, None)
    return d, keep


def create(d):
    h = ctypes.c_void_p()
    rc = A.lib().ebtc_batch_create(ctypes.byref(d), ctypes.byref(h))
    return rc, h


def test_batch_create_ok_and_destroy_null_safe():
    d, keep = make_desc()
    rc, h = create(d)
    assert rc == 0 and h.value
    A.lib().ebtc_batch_destroy(h)
    A.lib().ebtc_batch_destroy(None)


@pytest.mark.parametrize("mutate,code,text", [
    (lambda d: setattr(d, "dtype", 7), A.EBTC_EINVAL, "dtype"),
    (lambda d: setattr(d, "num_graphs", 0), A.EBTC_EINVAL, "num_graphs"),
    (lambda d: setattr(d, "num_realizations", 0), A.EBTC_EINVAL, "num_realizations"),
    (lambda d: setattr(d, "num_realizations", 4), A.EBTC_EBADGRAPH, "sum of graph_nreal"),
    (lambda d: setattr(d, "row_ptr", None), A.EBTC_EINVAL, "row_ptr"),
    (lambda d: setattr(d, "graph_n", None), A.EBTC_EINVAL, "host array"),
])
def test_batch_create_rejects(mutate, code, text):
    d, keep = make_desc()
    mutate(d)
    rc, h = create(d)
    assert rc == code and not h.value
    assert text in A.lib().ebtc_last_error().decode()


def test_batch_create_rejects_bad_counts():
    d, keep = make_desc(n=(0,))
    assert create(d)[0] == A.EBTC_EINVAL
    d, keep = make_desc(nnz=(20, -5, 20))
    assert create(d)[0] == A.EBTC_EBADGRAPH
    d, keep = make_desc(nnz=(20, 2 ** 31, 20))
    assert create(d)[0] == A.EBTC_EBADGRAPH


def test_int64_offsets_beyond_2_31_accepted():
    # three realizations of 2^30 entries each: batch offsets pass 2^31 while each realization stays < 2^31
    d, keep = make_desc(n=(1000,), nnz=(2 ** 30, 2 ** 30, 2 ** 30))
    rc, h = create(d)
    assert rc == 0
    A.lib().ebtc_batch_destroy(h)


def plan(h, **kw):
    o = A.default_opts(**kw)
    ws, ck = ctypes.c_size_t(), ctypes.c_size_t()
    rc = A.lib().ebtc_plan(h, ctypes.byref(o), ctypes.byref(ws), ctypes.byref(ck))
    return rc, ws.value, ck.value


def align(x):
    return (x + 255) // 256 * 256


def expected_ws(G, nreal, n, m_slots, es, rstate_bytes):
    R = sum(nreal)
    blocks = sum(((ng + 2047) // 2048) * nr for ng, nr in zip(n, nreal))
    rows = sum(ng * nr for ng, nr in zip(n, nreal))
    off = align(80 * R)  # realization records
    off = align(off + 24 * G)
    off = align(off + 4 * blocks)
    off = align(off + rstate_bytes * R)
    off = align(off + 8 * A.M_LIMIT * blocks)  # dot partials: one per basis vector and row block
    off = align(off + 8 * blocks)
    off = align(off + 4 * A.M_LIMIT)  # realizations still running after each step (adaptive runs)
    off = align(off + es * m_slots * rows)
    off = align(off + es * rows)
    off = align(off + es * rows)
    return off


M = A.M_LIMIT
RSTATE_BYTES = 8 * (M + M + (M + 1) + M + M + 4) + 4 * 4  # alpha, beta, s, y, scal; 4 scalars; 4 ints


@pytest.mark.parametrize("dtype,es", [(A.EBTC_F32, 4), (A.EBTC_F64, 8)])
def test_plan_workspace_arithmetic(dtype, es):
    d, keep = make_desc(G=2, nreal=(2, 3), n=(3000, 70), nnz=(10, 10, 10, 10, 10), dtype=dtype)
    rc, h = create(d)
    assert rc == 0
    rc, ws, ck = plan(h, m=30)
    assert rc == 0
    assert ws == expected_ws(2, (2, 3), (3000, 70), 31, es, RSTATE_BYTES)
    assert ck == 5 * A.CKPT_DOUBLES * 8
    rc, ws2, _ = plan(h, m=0, m_max=60, tol=1e-6)
    assert rc == 0 and ws2 == expected_ws(2, (2, 3), (3000, 70), 61, es, RSTATE_BYTES)
    rc, ws3, _ = plan(h, m=30, reorth=0)  # memory-bounded: three basis slots whatever m
    assert rc == 0 and ws3 == expected_ws(2, (2, 3), (3000, 70), 3, es, RSTATE_BYTES)
    A.lib().ebtc_batch_destroy(h)


@pytest.mark.parametrize("seg_len,per", [(0, 4096), (8192, 8192), (300, 300)])
def test_plan_balanced_workspace_arithmetic(seg_len, per):
    # the entry-balanced form appends its shares (16 bytes each: one per `per` entries of a
    # realization, at least one) and the first share of each realization (int64, R + 1); a small
    # batch takes the smallest default share size (4096)
    nnz = (10, 9000, 8192, 8193, 0)
    d, keep = make_desc(G=2, nreal=(2, 3), n=(3000, 70), nnz=nnz)
    rc, h = create(d)
    assert rc == 0
    rc, ws, _ = plan(h, m=30, spmv=5, seg_len=seg_len)
    assert rc == 0
    shares = sum(max(1, -(-z // per)) for z in nnz)
    off = expected_ws(2, (2, 3), (3000, 70), 31, 4, RSTATE_BYTES)
    off = align(off + 16 * shares)
    off = align(off + 8 * (5 + 1))
    assert ws == off
    rc, _, _ = plan(h, m=30, spmv=5, seg_len=100)
    assert rc == A.EBTC_EINVAL and "shares of 256" in A.lib().ebtc_last_error().decode()
    A.lib().ebtc_batch_destroy(h)


def test_plan_segmented_workspace_arithmetic():
    # the column-segmented form appends: block flags (int32), per-(segment, row) counts (8 bits,
    # max segments x 2048 per block), wave-band offsets (16 bits, max segments x 17 per block),
    # 64-byte block descriptors, in-segment columns (16 bits per slot: the entries, then per block
    # 3 x 16 x 32 + 8 slots for the zero padding of the wave bands' runs and the alignment of the
    # block's first slot); no value copy for a pattern-only batch
    d, keep = make_desc(G=2, nreal=(2, 3), n=(3000, 70), nnz=(10, 10, 10, 10, 10))
    rc, h = create(d)
    rc, ws, _ = plan(h, m=30, spmv=4, seg_len=1000)
    assert rc == 0
    blocks = 2 * 2 + 3 * 1
    off = expected_ws(2, (2, 3), (3000, 70), 31, 4, RSTATE_BYTES)
    off = align(off + 4 * blocks)
    off = align(off + 3 * 2048 * blocks)      # per-(segment, row) counts
    off = align(off + 2 * 3 * 17 * blocks)    # per-(segment, wave band) entry offsets (16 bits)
    off = align(off + 64 * blocks)            # block descriptors
    off = align(off + 2 * (50 + blocks * (3 * 16 * 32 + 8) + 8))
    assert ws == off
    rc, _, _ = plan(h, m=30, spmv=4, seg_len=50)  # 60 segments
    assert rc == A.EBTC_EINVAL and "segments" in A.lib().ebtc_last_error().decode()
    A.lib().ebtc_batch_destroy(h)


def set_forms(h, forms, lanes=None, seg=None):
    f = np.array(forms, np.int32)
    l = None if lanes is None else np.array(lanes, np.int32)
    q = None if seg is None else np.array(seg, np.int32)
    return A.lib().ebtc_set_forms(h, f.ctypes.data, None if l is None else l.ctypes.data,
                                  None if q is None else q.ctypes.data), (f, l, q)


def test_set_forms_records_and_plans():
    # one form recorded for every graph is the plain single-form plan; a form named in the options
    # overrides it; graphs on different forms are refused (several forms in one launch sequence are
    # not supported)
    d, keep = make_desc(G=2, nreal=(2, 3), n=(3000, 70), nnz=(10, 10, 10, 10, 10))
    rc, h = create(d)
    assert rc == 0
    rc, _ = set_forms(h, [5, 5])
    assert rc == 0
    assert plan(h, m=30)[1] == plan(h, m=30, spmv=5)[1]
    assert plan(h, m=30, spmv=1)[1] == expected_ws(2, (2, 3), (3000, 70), 31, 4, RSTATE_BYTES)
    rc, _ = set_forms(h, [4, 5], seg=[1000, 0])
    assert rc == 0
    f = np.zeros(2, np.int32)
    l = np.zeros(2, np.int32)
    q = np.zeros(2, np.int32)
    assert A.lib().ebtc_tuned_forms(h, f.ctypes.data, l.ctypes.data, q.ctypes.data) == 0
    assert f.tolist() == [4, 5] and q.tolist() == [1000, 0]
    rc, _, _ = plan(h, m=30)
    assert rc == A.EBTC_ENOTSUPPORTED and "several SpMV forms" in A.lib().ebtc_last_error().decode()
    assert plan(h, m=30, spmv=4, seg_len=1000)[0] == 0  # a named form still plans
    A.lib().ebtc_batch_destroy(h)


@pytest.mark.parametrize("forms,lanes,seg,text", [
    ([7, 1], None, None, "unknown spmv form"),
    ([1, 0], None, None, "unknown spmv form"),
    ([2, 2], [4, 5], None, "lanes must be"),
    ([4, 1], None, [-1, 0], "seg_len must be"),
])
def test_set_forms_rejects(forms, lanes, seg, text):
    d, keep = make_desc(G=2, nreal=(2, 3), n=(3000, 70), nnz=(10, 10, 10, 10, 10))
    rc, h = create(d)
    assert rc == 0
    rc, _ = set_forms(h, forms, lanes, seg)
    assert rc == A.EBTC_EINVAL and text in A.lib().ebtc_last_error().decode()
    assert A.lib().ebtc_set_forms(h, None, None, None) == A.EBTC_EINVAL
    assert A.lib().ebtc_set_forms(None, np.zeros(2, np.int32).ctypes.data, None, None) == A.EBTC_EINVAL
    f = np.full(2, 9, np.int32)
    assert A.lib().ebtc_tuned_forms(h, f.ctypes.data, None, None) == 0 and f.tolist() == [0, 0]  # nothing recorded
    A.lib().ebtc_batch_destroy(h)


def test_tune_cache_text_roundtrip_and_errors():
    L = A.lib()
    assert L.ebtc_tune_cache_clear() == 0
    n = ctypes.c_size_t(99)
    assert L.ebtc_tune_cache_get(None, 0, ctypes.byref(n)) == 0 and n.value == 0
    text = b"f32v-n16-d8-h2-s4 4 0 12288\nf32p-n19-d6-h9-s5 5 0 8192\n"
    assert L.ebtc_tune_cache_put(text) == 0
    assert L.ebtc_tune_cache_get(None, 0, ctypes.byref(n)) == 0
    buf = ctypes.create_string_buffer(n.value + 1)
    assert L.ebtc_tune_cache_get(buf, n.value + 1, ctypes.byref(n)) == 0
    assert sorted(buf.value.decode().splitlines()) == sorted(text.decode().splitlines())
    small = ctypes.create_string_buffer(4)
    assert L.ebtc_tune_cache_get(small, 4, ctypes.byref(n)) == A.EBTC_EINVAL
    # later lines win; malformed lines are refused whole
    assert L.ebtc_tune_cache_put(b"f32v-n16-d8-h2-s4 1 0 0\n") == 0
    assert "f32v-n16-d8-h2-s4 1 0 0" in _cache_text()
    for bad in (b"key 9 0 0", b"key 4 0", b"key 4 -1 0", b"key x 0 0", b"key 1 3 0", b"key 1 64 0"):
        assert L.ebtc_tune_cache_put(bad) == A.EBTC_EINVAL and "tune-cache line" in L.ebtc_last_error().decode()
    assert L.ebtc_tune_cache_put(None) == A.EBTC_EINVAL
    assert L.ebtc_tune_cache_get(None, 0, None) == A.EBTC_EINVAL
    assert L.ebtc_tune_cache_clear() == 0 and _cache_text() == ""


def _cache_text():
    n = ctypes.c_size_t()
    A.lib().ebtc_tune_cache_get(None, 0, ctypes.byref(n))
    buf = ctypes.create_string_buffer(n.value + 1)
    A.lib().ebtc_tune_cache_get(buf, n.value + 1, ctypes.byref(n))
    return buf.value.decode()


@pytest.mark.parametrize("kw,text", [
    (dict(m=129), "m must be"), (dict(m=-1), "m must be"), (dict(m=0, m_max=0), "m_max"),
    (dict(m=0, m_max=129), "m_max"),
    (dict(m=0, tol=0.0), "tol"), (dict(reorth=3), "reorth"), (dict(schedule=9), "schedule"),
    (dict(lanes_per_row=5), "lanes_per_row"), (dict(hub_threshold=-1), "hub_threshold"),
    (dict(seg_len=-1), "seg_len"), (dict(spmv=7), "spmv form"), (dict(spmv=-1), "spmv form"),
])
def test_plan_rejects_bad_opts(kw, text):
    d, keep = make_desc()
    rc, h = create(d)
    rc, _, _ = plan(h, **kw)
    assert rc == A.EBTC_EINVAL and text in A.lib().ebtc_last_error().decode()
    A.lib().ebtc_batch_destroy(h)


def test_scores_rejects_before_enqueue():
    d, keep = make_desc()
    rc, h = create(d)
    o = A.default_opts(m=10)
    # NULL outputs and a too-small workspace fail on the host before any HIP call
    rc = A.lib().ebtc_scores(h, ctypes.byref(o), FAKE_DEV, 1 << 40, None, None, None, None, None)
    assert rc == A.EBTC_EINVAL
    rc = A.lib().ebtc_scores(h, ctypes.byref(o), FAKE_DEV, 16, FAKE_DEV, FAKE_DEV, None, None, None)
    assert rc == A.EBTC_EWORKSPACE and "need" in A.lib().ebtc_last_error().decode()
    rc = A.lib().ebtc_scores(h, ctypes.byref(o), FAKE_DEV + 8, 1 << 40, FAKE_DEV, FAKE_DEV, None, None, None)
    assert rc == A.EBTC_EINVAL and "aligned" in A.lib().ebtc_last_error().decode()
    A.lib().ebtc_batch_destroy(h)


def test_scores_backward_rejects_before_enqueue():
    d, keep = make_desc()
    rc, h = create(d)
    o = A.default_opts(m=10)
    L = A.lib()
    args = (h, ctypes.byref(o), FAKE_DEV, FAKE_DEV, FAKE_DEV, FAKE_DEV, 1 << 40)
    assert L.ebtc_scores_backward(h, ctypes.byref(o), None, FAKE_DEV, FAKE_DEV, FAKE_DEV, 1 << 40, None, None,
                                  None) == A.EBTC_EINVAL
    # a checkpoint to compare needs the mismatch counter
    assert L.ebtc_scores_backward(*args, FAKE_DEV, None, None) == A.EBTC_EINVAL
    assert "ckpt_mismatch" in L.ebtc_last_error().decode()
    o2 = A.default_opts(m=10, reorth=0)
    assert L.ebtc_scores_backward(h, ctypes.byref(o2), FAKE_DEV, FAKE_DEV, FAKE_DEV, FAKE_DEV, 1 << 40, None, None,
                                  None) == A.EBTC_ENOTSUPPORTED
    o3 = A.default_opts(m=41)
    assert L.ebtc_scores_backward(h, ctypes.byref(o3), FAKE_DEV, FAKE_DEV, FAKE_DEV, FAKE_DEV, 1 << 40, None, None,
                                  None) == A.EBTC_ENOTSUPPORTED
    A.lib().ebtc_batch_destroy(h)


def test_scores_noalloc_rejects_before_enqueue():
    # NULL outputs, a batch whose workspace exceeds the static array, and a schedule the batch cannot
    # take all fail on the host, before any HIP call (the scratch address is looked up only after them)
    d, keep = make_desc()
    rc, h = create(d)
    o = A.default_opts(m=10)
    assert A.lib().ebtc_scores_noalloc(h, ctypes.byref(o), None, None, None, None, None) == A.EBTC_EINVAL
    A.lib().ebtc_batch_destroy(h)
    d, keep = make_desc(nreal=(4,), n=(1_000_000,), nnz=(10_000_000,) * 4)
    rc, h = create(d)
    ws, _ = ctypes.c_size_t(), None
    assert A.lib().ebtc_plan(h, ctypes.byref(o), ctypes.byref(ws), None) == A.EBTC_OK
    assert ws.value > A.NOALLOC_WS_BYTES
    rc = A.lib().ebtc_scores_noalloc(h, ctypes.byref(o), FAKE_DEV, FAKE_DEV, None, None, None)
    assert rc == A.EBTC_EWORKSPACE and "static scratch" in A.lib().ebtc_last_error().decode()
    o = A.default_opts(m=10, schedule=A.SCHED_SINGLE, m_max=60)
    d2, keep2 = make_desc(nreal=(1,), n=(3000,), nnz=(20,))
    rc, h2 = create(d2)
    rc = A.lib().ebtc_scores_noalloc(h2, ctypes.byref(o), FAKE_DEV, FAKE_DEV, None, None, None)
    assert rc == A.EBTC_ENOTSUPPORTED and "single-kernel" in A.lib().ebtc_last_error().decode()
    A.lib().ebtc_batch_destroy(h)
    A.lib().ebtc_batch_destroy(h2)


def test_topk_rejects_bad_k():
    d, keep = make_desc(n=(10,))
    rc, h = create(d)
    ws = ctypes.c_size_t()
    assert A.lib().ebtc_topk_ws_bytes(h, ctypes.byref(ws)) == 0 and ws.value > 0
    for k, code in ((11, A.EBTC_EINVAL), (-1, A.EBTC_EINVAL)):
        kv = (ctypes.c_int32 * 1)(k)
        rc = A.lib().ebtc_topk(h, FAKE_DEV, kv, FAKE_DEV, None, FAKE_DEV, ws.value, None)
        assert rc == code
    rc = A.lib().ebtc_topk(h, FAKE_DEV, (ctypes.c_int32 * 1)(3), FAKE_DEV, None, FAKE_DEV, 1, None)
    assert rc == A.EBTC_EWORKSPACE
    A.lib().ebtc_batch_destroy(h)


def test_component_entry_points_validate():
    L = A.lib()
    assert L.ebtc_spmv(5, 10, FAKE_DEV, FAKE_DEV, None, FAKE_DEV, FAKE_DEV + 64, 0, 0, 0, None) == A.EBTC_EINVAL
    assert L.ebtc_spmv(0, 0, FAKE_DEV, FAKE_DEV, None, FAKE_DEV, FAKE_DEV + 64, 0, 0, 0, None) == A.EBTC_EINVAL
    assert L.ebtc_spmv(0, 10, FAKE_DEV, FAKE_DEV, None, FAKE_DEV, FAKE_DEV, 0, 0, 0, None) == A.EBTC_EINVAL
    assert L.ebtc_spmv(0, 10, FAKE_DEV, FAKE_DEV, None, FAKE_DEV, FAKE_DEV + 64, 6, 0, 0, None)
    assert L.ebtc_spmv(0, 10, FAKE_DEV, FAKE_DEV, None, FAKE_DEV, FAKE_DEV + 64, 0, 0, -2, None) == A.EBTC_EINVAL
    assert L.ebtc_tridiag_expv(1, A.M_LIMIT + 1, FAKE_DEV, FAKE_DEV, FAKE_DEV, FAKE_DEV, 1, None) == A.EBTC_EINVAL
    assert L.ebtc_tridiag_expv(-1, 5, FAKE_DEV, FAKE_DEV, FAKE_DEV, FAKE_DEV, 1, None) == A.EBTC_EINVAL
    assert L.ebtc_tridiag_expv(0, 5, None, None, None, None, 1, None) == A.EBTC_OK


def test_tune_validates_before_any_launch():
    d, keep = make_desc()
    rc, h = create(d)
    o = A.default_opts(m=10)
    L = A.lib()
    assert L.ebtc_tune(None, ctypes.byref(o), FAKE_DEV, 1 << 40, None, None, None, None, None) == A.EBTC_EINVAL
    assert L.ebtc_tune(h, ctypes.byref(o), None, 1 << 40, None, None, None, None, None) == A.EBTC_EINVAL
    assert L.ebtc_tune(h, ctypes.byref(o), FAKE_DEV, 16, None, None, None, None, None) == A.EBTC_EWORKSPACE
    o.spmv = 9
    assert L.ebtc_tune(h, ctypes.byref(o), FAKE_DEV, 1 << 40, None, None, None, None, None) == A.EBTC_EINVAL
    A.lib().ebtc_batch_destroy(h)


def test_last_error_cleared_on_success():
    d, keep = make_desc()
    d.dtype = 9
    assert create(d)[0] != 0 and A.lib().ebtc_last_error()
    d2, keep2 = make_desc()
    rc, h = create(d2)
    assert rc == 0 and A.lib().ebtc_last_error() == b""
    A.lib().ebtc_batch_destroy(h)


def test_subgraph_centrality_validates_and_sizes():
    L = A.lib()
    ws = ctypes.c_size_t()
    assert L.ebtc_subgraph_centrality_ws_bytes(0, 5000, 3, 20, ctypes.byref(ws)) == 0 and ws.value > 0
    w1 = ws.value
    assert L.ebtc_subgraph_centrality_ws_bytes(0, 5000, 6, 20, ctypes.byref(ws)) == 0 and ws.value > w1
    for args, text in [((7, 10, 1, 5), "dtype"), ((0, 0, 1, 5), "n must"), ((0, 10, 0, 5), "count"),
                       ((0, 10, 1, 0), "m must"), ((0, 10, 1, A.M_LIMIT + 1), "m must")]:
        assert L.ebtc_subgraph_centrality_ws_bytes(*args, ctypes.byref(ws)) == A.EBTC_EINVAL
        assert text in L.ebtc_last_error().decode()
    assert L.ebtc_subgraph_centrality(0, 10, None, FAKE_DEV, None, 1, FAKE_DEV, 5, FAKE_DEV, FAKE_DEV, 1 << 30,
                                      None) == A.EBTC_EINVAL
    assert L.ebtc_subgraph_centrality(0, 10, FAKE_DEV, FAKE_DEV, None, 1, FAKE_DEV, 5, FAKE_DEV, FAKE_DEV, 16,
                                      None) == A.EBTC_EWORKSPACE


@pytest.mark.parametrize("kw,code,text", [
    (dict(family="ws", n=1000, k=7), A.EBTC_EINVAL, "even k"),
    (dict(family="ws", n=6, k=6), A.EBTC_EINVAL, "n >= k + 2"),
    (dict(family="ws", n=100, k=4, beta=1.5), A.EBTC_EINVAL, "beta"),
    (dict(family="er", n=100, p=1.5), A.EBTC_EINVAL, "p must be"),
    (dict(family="er", n=0, p=0.1), A.EBTC_EINVAL, "n >= 1"),
    (dict(family="ba", n=5, k=4), A.EBTC_EINVAL, "n >= k + 2"),
    (dict(family="ba", n=50, k=0), A.EBTC_EINVAL, "k >= 1"),
    (dict(family="er", n=100, p=0.1, targets=[1, 1]), A.EBTC_EINVAL, "repeated target"),
    (dict(family="er", n=100, p=0.1, targets=[1, 100]), A.EBTC_EINVAL, "out of range"),
    (dict(family="er", n=100, p=0.1, targets=[1, 2], pattern=[[0, 2]]), A.EBTC_EINVAL, "pattern edge"),
    (dict(family="er", n=100, p=0.1, targets=[1, 2], pattern=[[1, 1]]), A.EBTC_EINVAL, "pattern edge"),
    (dict(family="er", n=100, p=0.1, count=0), A.EBTC_EINVAL, "count"),
    (dict(family="er", n=100, p=0.1, first=(1 << 32) - 1, count=2), A.EBTC_EINVAL, "2^32"),
    (dict(family="er", n=2_000_000_000, p=1e-9, count=4), A.EBTC_ENOTSUPPORTED, "2^63"),
])
def test_generate_plan_validates(kw, code, text):
    # the spec is checked before anything touches a device
    from paper_1409_5000_amd.api import _gen_spec
    kw = {"count": 1, "seed": 7, **kw}
    spec, keep = _gen_spec(**kw)
    ws = ctypes.c_size_t()
    assert A.lib().ebtc_generate_plan(ctypes.byref(spec), ctypes.byref(ws)) == code
    assert text in A.lib().ebtc_last_error().decode()
    assert A.lib().ebtc_generate_plan(ctypes.byref(spec), None) == A.EBTC_EINVAL


def test_generate_plan_needs_no_device():
    # the workspace, the sort's and scan's temporary storage included, follows from the spec alone;
    # it grows with the realizations per call
    from paper_1409_5000_amd.api import _gen_spec
    sizes = []
    for count in (1, 4):
        spec, keep = _gen_spec(family="er", n=20000, p=1e-3, count=count, seed=7)
        ws = ctypes.c_size_t()
        assert A.lib().ebtc_generate_plan(ctypes.byref(spec), ctypes.byref(ws)) == 0
        sizes.append(ws.value)
    assert 0 < sizes[0] < sizes[1]


def test_generate_spec_layout():
    # the C struct: int32 family, n; double p; int32 k, count; double beta; uint64 seed; int64 first;
    # int32 t, pattern_edges; two pointers
    f = {name: getattr(A.GenSpec, name).offset for name, _ in A.GenSpec._fields_}
    assert (f["p"], f["k"], f["beta"], f["seed"], f["first"], f["t"], f["targets"], f["pattern"]) == \
        (8, 16, 24, 32, 40, 48, 56, 64)
    assert ctypes.sizeof(A.GenSpec) == 72
