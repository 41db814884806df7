"""ctypes declarations of the C ABI in include/ebtc.h (argument marshalling only).

The library is libebtc.so next to this file, built by paper_1409_5000_amd.build. Importing the
binding never falls back to anything else: if the library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libebtc.so")

EBTC_OK, EBTC_EINVAL, EBTC_EBADGRAPH, EBTC_EWORKSPACE, EBTC_EHIP, EBTC_ENOTSUPPORTED = range(6)
EBTC_F32, EBTC_F64 = 0, 1
SCHED_AUTO, SCHED_PLAIN, SCHED_BATCHED, SCHED_SINGLE = 0, 1, 2, 3
FLAG_BREAKDOWN, FLAG_CAPPED, FLAG_NONFINITE = 1, 2, 4
M_LIMIT = 128
TOPK_LIMIT = 4096
CKPT_DOUBLES = 2 * M_LIMIT + 4
NOALLOC_WS_BYTES = 64 << 20  # EBTC_NOALLOC_WS_BYTES

EXPORTED = [
    "ebtc_version", "ebtc_status_str", "ebtc_last_error", "ebtc_default_opts", "ebtc_batch_create",
    "ebtc_batch_destroy", "ebtc_plan", "ebtc_scores", "ebtc_scores_noalloc", "ebtc_topk_ws_bytes", "ebtc_topk",
    "ebtc_spmv", "ebtc_tridiag_expv", "ebtc_validate_ws_bytes", "ebtc_validate", "ebtc_profile_phases", "ebtc_plan_backward",
    "ebtc_scores_backward", "ebtc_tune", "ebtc_subgraph_centrality_ws_bytes", "ebtc_subgraph_centrality",
    "ebtc_generate_plan", "ebtc_generate_count", "ebtc_generate_fill", "ebtc_tuned_forms", "ebtc_set_forms",
    "ebtc_tune_cache_get", "ebtc_tune_cache_put", "ebtc_tune_cache_clear",
]
GEN_FAMILIES = {"er": 0, "ws": 1, "ba": 2}
SPMV_FORMS = {"auto": 0, "stream": 1, "lanes": 2, "staged": 3, "segmented": 4, "balanced": 5, "paneled": 6}
TUNE_SLOTS = 10  # entries of ebtc_tune's ms_out
PHASES = ["start", "spmv", "dots", "update", "tridiag", "combine", "sum", "prepare", "first", "solve"]


class BatchDesc(ctypes.Structure):
    _fields_ = [
        ("dtype", c_int32), ("num_graphs", c_int32), ("num_realizations", c_int64),
        ("graph_n", POINTER(c_int32)), ("graph_nreal", POINTER(c_int32)),
        ("rowptr_off", POINTER(c_int64)), ("nnz_off", POINTER(c_int64)),
        ("row_ptr", c_void_p), ("col_idx", c_void_p), ("values", c_void_p),
    ]


class Opts(ctypes.Structure):
    _fields_ = [
        ("m", c_int32), ("m_max", c_int32), ("tol", c_double), ("reorth", c_int32), ("schedule", c_int32),
        ("use_hipgraph", c_int32), ("shift", c_int32), ("spmv", c_int32), ("lanes_per_row", c_int32),
        ("hub_threshold", c_int32), ("seg_len", c_int32),
    ]


class GenSpec(ctypes.Structure):
    _fields_ = [
        ("family", c_int32), ("n", c_int32), ("p", c_double), ("k", c_int32), ("count", c_int32),
        ("beta", c_double), ("seed", ctypes.c_uint64), ("first", c_int64), ("t", c_int32),
        ("pattern_edges", c_int32), ("targets", POINTER(c_int32)), ("pattern", POINTER(c_int32)),
    ]


class Diag(ctypes.Structure):
    _fields_ = [("m_used", c_int32), ("flags", c_int32), ("theta", c_double), ("est", c_double)]


class EbtcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ebtc status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1409_5000_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz = c_void_p, c_size_t
    sig = {
        "ebtc_version": (c_int, [POINTER(c_int), POINTER(c_int)]),
        "ebtc_status_str": (c_char_p, [c_int]),
        "ebtc_last_error": (c_char_p, []),
        "ebtc_default_opts": (None, [POINTER(Opts)]),
        "ebtc_batch_create": (c_int, [POINTER(BatchDesc), POINTER(vp)]),
        "ebtc_batch_destroy": (None, [vp]),
        "ebtc_plan": (c_int, [vp, POINTER(Opts), POINTER(sz), POINTER(sz)]),
        "ebtc_scores": (c_int, [vp, POINTER(Opts), vp, sz, vp, vp, vp, vp, vp]),
        "ebtc_scores_noalloc": (c_int, [vp, POINTER(Opts), vp, vp, vp, vp, vp]),
        "ebtc_topk_ws_bytes": (c_int, [vp, POINTER(sz)]),
        "ebtc_topk": (c_int, [vp, vp, POINTER(c_int32), vp, vp, vp, sz, vp]),
        "ebtc_spmv": (c_int, [c_int32, c_int32, vp, vp, vp, vp, vp, c_int32, c_int32, c_int32, vp]),
        "ebtc_tridiag_expv": (c_int, [c_int32, c_int32, vp, vp, vp, vp, c_int32, vp]),
        "ebtc_validate_ws_bytes": (c_int, [vp, POINTER(sz)]),
        "ebtc_validate": (c_int, [vp, vp, sz, POINTER(c_int64), vp]),
        "ebtc_profile_phases": (c_int, [vp, POINTER(Opts), vp, sz, vp, vp, POINTER(c_double), POINTER(c_int64), vp]),
        "ebtc_plan_backward": (c_int, [vp, POINTER(Opts), POINTER(sz)]),
        "ebtc_scores_backward": (c_int, [vp, POINTER(Opts), vp, vp, vp, vp, sz, vp, vp, vp]),
        "ebtc_tune": (c_int, [vp, POINTER(Opts), vp, sz, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                              POINTER(c_double), vp]),
        "ebtc_tuned_forms": (c_int, [vp, vp, vp, vp]),
        "ebtc_set_forms": (c_int, [vp, vp, vp, vp]),
        "ebtc_tune_cache_get": (c_int, [ctypes.c_char_p, sz, POINTER(sz)]),
        "ebtc_tune_cache_put": (c_int, [ctypes.c_char_p]),
        "ebtc_tune_cache_clear": (c_int, []),
        "ebtc_subgraph_centrality_ws_bytes": (c_int, [c_int32, c_int32, c_int32, c_int32, POINTER(sz)]),
        "ebtc_subgraph_centrality": (c_int, [c_int32, c_int32, vp, vp, vp, c_int32, vp, c_int32, vp, vp, sz, vp]),
        "ebtc_generate_plan": (c_int, [POINTER(GenSpec), POINTER(sz)]),
        "ebtc_generate_count": (c_int, [POINTER(GenSpec), vp, sz, vp, vp, vp]),
        "ebtc_generate_fill": (c_int, [POINTER(GenSpec), vp, sz, POINTER(c_int64), vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status: int) -> None:
    if status != EBTC_OK:
        raise EbtcError(status, lib().ebtc_last_error().decode())


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().ebtc_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o
