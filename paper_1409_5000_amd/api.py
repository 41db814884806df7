"""Python face of the EBTC library: device batches, summed communicability scores, top-K.

Everything computational runs in the HIP library through the C ABI (paper_1409_5000_amd._abi);
this module only allocates device memory with torch, marshals pointers and picks the stream.

    b = Batch.from_host(host_batch)                 # CSR realizations copied to the GPU
    out = b.scores(m=30)                             # S~ per graph (scaled), log-scales, diagnostics
    idx, val = b.topk(out.scores, k=[50])            # candidate target nodes per graph

The summed score of graph g (eq. (5) of the paper: the plain sum over realizations of
exp(A_k) 1, eq. (4)) is exp(log_scale[g]) * scores[g-block].
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _abi as A

_DT = {"f32": (A.EBTC_F32, torch.float32, np.float32), "f64": (A.EBTC_F64, torch.float64, np.float64)}
_SCHED = {"auto": A.SCHED_AUTO, "plain": A.SCHED_PLAIN, "batched": A.SCHED_BATCHED, "single": A.SCHED_SINGLE}


def _vp(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def current_stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_opts(m: int = 30, tol: float = 1e-6, m_max: int = 60, reorth: int = 1, schedule: str = "auto",
              hipgraph: bool = True, shift: bool = True, spmv: str = "auto", lanes: int = 0, hub: int = 0,
              seg_len: int = 0) -> A.Opts:
    """Options of one call. schedule: "auto" (the single-kernel form when every graph has at most 2048
    nodes and reorth is 1, else "batched"), "batched" (one launch per phase over all realizations),
    "single" (one launch runs every realization's whole process) or "plain" (one realization at a
    time). spmv: "auto" (the tuned form, else "stream"), "stream", "lanes" (lanes per row, default 8),
    "staged" (segment length seg_len, default the largest that fits in LDS), "segmented" (seg_len
    columns per segment, default 12288 FP32 / 6144 FP64), "balanced" (seg_len entries per share) or
    "paneled" (seg_len columns per panel, default 12288 FP32 / 6144 FP64)."""
    return A.default_opts(m=m, tol=tol, m_max=m_max, reorth=reorth, schedule=_SCHED[schedule],
                          use_hipgraph=int(hipgraph), shift=int(shift), spmv=A.SPMV_FORMS[spmv], lanes_per_row=lanes,
                          hub_threshold=hub, seg_len=seg_len)


@dataclass
class ScoreResult:
    scores: torch.Tensor     # [sum_g n_g] dtype: S~ per graph, concatenated
    log_scale: torch.Tensor  # [G] float64: Sigma_g
    diag: torch.Tensor | None  # [R, 3] float64 view: (m_used, flags, theta, est) via diag_numpy()
    ckpt: torch.Tensor | None
    raw_diag: torch.Tensor | None = None

    def diag_numpy(self) -> np.ndarray:
        """Structured host copy of the per-realization diagnostics."""
        if self.raw_diag is None:
            return None
        host = self.raw_diag.cpu().numpy().tobytes()
        return np.frombuffer(host, dtype=np.dtype([("m_used", "<i4"), ("flags", "<i4"), ("theta", "<f8"),
                                                   ("est", "<f8")]))


class Run:
    """Workspace and output buffers for repeated ebtc_scores calls with fixed options.

    Reusing a Run keeps every device pointer fixed, so the batched schedule replays its captured
    hipGraph instead of re-capturing it."""

    def __init__(self, batch: "Batch", opts: A.Opts, diag: bool = True, ckpt: bool = False):
        self.batch = batch
        self.opts = opts
        ws = ctypes.c_size_t()
        ck = ctypes.c_size_t()
        A.check(A.lib().ebtc_plan(batch.handle, ctypes.byref(opts), ctypes.byref(ws), ctypes.byref(ck)))
        dev = batch.device
        self.ws_bytes = ws.value
        self.ws = torch.empty(max(1, ws.value), dtype=torch.uint8, device=dev)
        self.scores = torch.empty(batch.total_scores, dtype=batch.tdtype, device=dev)
        self.log_scale = torch.empty(batch.G, dtype=torch.float64, device=dev)
        self.raw_diag = torch.empty(batch.R * ctypes.sizeof(A.Diag), dtype=torch.uint8, device=dev) if diag else None
        self.ckpt = torch.empty(max(1, ck.value) // 8, dtype=torch.float64, device=dev) if ckpt else None

    def launch(self) -> ScoreResult:
        A.check(A.lib().ebtc_scores(self.batch.handle, ctypes.byref(self.opts), _vp(self.ws), self.ws_bytes,
                                    _vp(self.scores), _vp(self.log_scale), _vp(self.ckpt), _vp(self.raw_diag),
                                    current_stream()))
        return ScoreResult(self.scores, self.log_scale, None, self.ckpt, self.raw_diag)


    def profile(self) -> dict:
        """Eager run with a HIP event pair around every launch: {phase: (total_ms, launches)}."""
        ms = (ctypes.c_double * len(A.PHASES))()
        cnt = (ctypes.c_int64 * len(A.PHASES))()
        A.check(A.lib().ebtc_profile_phases(self.batch.handle, ctypes.byref(self.opts), _vp(self.ws), self.ws_bytes,
                                            _vp(self.scores), _vp(self.log_scale), ms, cnt, current_stream()))
        return {p: (ms[i], cnt[i]) for i, p in enumerate(A.PHASES)}


class BackwardRun:
    """Workspace and output for repeated ebtc_scores_backward calls with fixed options."""

    def __init__(self, batch: "Batch", opts: A.Opts):
        self.batch = batch
        self.opts = opts
        ws = ctypes.c_size_t()
        A.check(A.lib().ebtc_plan_backward(batch.handle, ctypes.byref(opts), ctypes.byref(ws)))
        self.ws_bytes = ws.value
        self.ws = torch.empty(max(1, ws.value), dtype=torch.uint8, device=batch.device)
        self.grad = torch.empty(max(1, int(batch.nnz_off[-1])), dtype=batch.tdtype, device=batch.device)

    def launch(self, log_scale: torch.Tensor, grad_scores: torch.Tensor, ckpt: torch.Tensor | None = None):
        """The gradient; with the forward call's checkpoint also the number of realizations whose
        recomputed forward process differs from it (a device int32 tensor: 0 when the recomputation
        is the forward's, bit for bit)."""
        g = grad_scores.to(self.batch.tdtype).contiguous()
        mism = torch.empty(1, dtype=torch.int32, device=self.batch.device) if ckpt is not None else None
        A.check(A.lib().ebtc_scores_backward(self.batch.handle, ctypes.byref(self.opts), _vp(log_scale), _vp(g),
                                             _vp(self.grad), _vp(self.ws), self.ws_bytes, _vp(ckpt), _vp(mism),
                                             current_stream()))
        grad = self.grad[: int(self.batch.nnz_off[-1])]
        return grad if ckpt is None else (grad, mism)


class Batch:
    """G graphs x N_g realizations as device CSR arrays (borrowed by the native batch handle)."""

    def __init__(self, graph_n, graph_nreal, rowptr_off, nnz_off, row_ptr, col_idx, values=None, dtype: str = "f32",
                 device: str = "cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("the EBTC library needs a GPU")
        self.dtype = dtype
        self.code, self.tdtype, self.ndtype = _DT[dtype]
        self.device = torch.device(device)
        self.graph_n = np.ascontiguousarray(graph_n, dtype=np.int32)
        self.graph_nreal = np.ascontiguousarray(graph_nreal, dtype=np.int32)
        self.rowptr_off = np.ascontiguousarray(rowptr_off, dtype=np.int64)
        self.nnz_off = np.ascontiguousarray(nnz_off, dtype=np.int64)
        self.G = int(self.graph_n.size)
        self.R = int(self.rowptr_off.size)
        self.total_scores = int(self.graph_n.sum())
        def dev(x, np_dtype, t_dtype):  # host arrays are copied; device tensors are used as they are
            if isinstance(x, torch.Tensor):
                return x.to(device=self.device, dtype=t_dtype).contiguous()
            return torch.as_tensor(np.ascontiguousarray(x, dtype=np_dtype)).to(self.device)
        self.row_ptr = dev(row_ptr, np.int32, torch.int32)
        self.col_idx = dev(col_idx, np.int32, torch.int32)
        self.values = None if values is None else dev(values, self.ndtype, self.tdtype)
        i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
        desc = A.BatchDesc(
            self.code, self.G, self.R,
            self.graph_n.ctypes.data_as(i32p), self.graph_nreal.ctypes.data_as(i32p),
            self.rowptr_off.ctypes.data_as(i64p), self.nnz_off.ctypes.data_as(i64p),
            self.row_ptr.data_ptr(), self.col_idx.data_ptr(), 0 if self.values is None else self.values.data_ptr())
        h = ctypes.c_void_p()
        A.check(A.lib().ebtc_batch_create(ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        self.score_off = np.concatenate([[0], np.cumsum(self.graph_n.astype(np.int64))])

    @classmethod
    def from_csr(cls, graphs: list, dtype: str = "f32", device: str = "cuda") -> "Batch":
        """From per-realization CSR arrays: graphs[g] is a list of (row_ptr, col_idx) or
        (row_ptr, col_idx, values) tuples, one per realization of graph g, all with n_g rows (local
        row pointers starting at 0, symmetric pattern, sorted columns, no self-loops). Values are
        taken from every realization or from none (pattern-only: all ones)."""
        gn, gr, rps, cis, vals, ro, no = [], [], [], [], [], [], [0]
        roff = 0
        for reals in graphs:
            if not reals:
                raise ValueError("every graph needs at least one realization")
            n = int(np.asarray(reals[0][0]).size) - 1
            gn.append(n)
            gr.append(len(reals))
            for real in reals:
                rp, ci = np.asarray(real[0], np.int64), np.asarray(real[1], np.int32)
                if rp.size != n + 1:
                    raise ValueError("the realizations of a graph must have the same number of rows")
                ro.append(roff)
                roff += n + 1
                rps.append(rp.astype(np.int32))
                cis.append(ci)
                no.append(no[-1] + ci.size)
                vals.append(None if len(real) < 3 or real[2] is None else np.asarray(real[2]))
        if any(v is None for v in vals) and not all(v is None for v in vals):
            raise ValueError("give values for every realization or for none")
        values = None if vals[0] is None else np.concatenate(vals)
        return cls(gn, gr, ro, no, np.concatenate(rps), np.concatenate(cis), values, dtype, device)

    @classmethod
    def from_host(cls, hb, device: str = "cuda", with_values: bool | None = None) -> "Batch":
        """From a host batch object (fields n, nreal, rowptr_off, nnz_off, row_ptr, col_idx, values, dtype)."""
        dtype = "f64" if np.dtype(hb.dtype) == np.float64 else "f32"
        vals = hb.values if (with_values is None or with_values) else None
        return cls(hb.n, hb.nreal, hb.rowptr_off, hb.nnz_off, hb.row_ptr, hb.col_idx, vals, dtype, device)

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            A.lib().ebtc_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def graph_slice(self, g: int) -> slice:
        return slice(int(self.score_off[g]), int(self.score_off[g + 1]))

    def run(self, diag: bool = True, ckpt: bool = False, **kw) -> Run:
        return Run(self, make_opts(**kw), diag=diag, ckpt=ckpt)

    def scores(self, diag: bool = True, ckpt: bool = False, **kw) -> ScoreResult:
        """Fresh output buffers on every call (see Run for repeated calls)."""
        return self.run(diag=diag, ckpt=ckpt, **kw).launch()

    def scores_noalloc(self, out: ScoreResult | None = None, **kw) -> ScoreResult:
        """ebtc_scores_noalloc: the library's fixed device array as the workspace (no allocation by the
        library). Outputs are allocated here unless `out` (a previous result) supplies them."""
        opts = make_opts(**kw)
        if out is None:
            out = ScoreResult(torch.empty(self.total_scores, dtype=self.tdtype, device=self.device),
                              torch.empty(self.G, dtype=torch.float64, device=self.device), None, None,
                              torch.empty(self.R * ctypes.sizeof(A.Diag), dtype=torch.uint8, device=self.device))
        A.check(A.lib().ebtc_scores_noalloc(self.handle, ctypes.byref(opts), _vp(out.scores), _vp(out.log_scale),
                                            _vp(out.ckpt), _vp(out.raw_diag), current_stream()))
        return out

    def topk(self, scores: torch.Tensor, k) -> tuple[torch.Tensor, torch.Tensor]:
        kv = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (self.G,)))
        ws = ctypes.c_size_t()
        A.check(A.lib().ebtc_topk_ws_bytes(self.handle, ctypes.byref(ws)))
        wst = torch.empty(max(1, ws.value), dtype=torch.uint8, device=self.device)
        tot = int(kv.sum())
        idx = torch.empty(max(1, tot), dtype=torch.int32, device=self.device)
        val = torch.empty(max(1, tot), dtype=self.tdtype, device=self.device)
        A.check(A.lib().ebtc_topk(self.handle, _vp(scores), kv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  _vp(idx), _vp(val), _vp(wst), ws.value, current_stream()))
        return idx[:tot], val[:tot]

    def tune(self, **kw) -> dict:
        """Times the SpMV forms bucket by bucket of similar graphs (ebtc_tune) and keeps each graph's
        fastest for spmv="auto" calls; buckets in the process-wide tune cache are not timed again. Plan
        Runs after tuning: the chosen forms set their workspace size. Returns the form (or "mixed"), the
        per-slot ms summed over the timed buckets, and each graph's form."""
        opts = make_opts(**kw)
        ws = ctypes.c_size_t()
        small = 3072 if self.dtype == "f64" else 6144
        # workspace for the largest candidate: the segmented form with the shorter segment length that
        # applies (more segments, more counts), the entry-balanced form, else the plan of the others
        A.check(A.lib().ebtc_plan(self.handle, ctypes.byref(opts), ctypes.byref(ws), None))
        need = ws.value
        for q in (small, 2 * small):
            seg = make_opts(**{**kw, "spmv": "segmented", "seg_len": q})
            if A.lib().ebtc_plan(self.handle, ctypes.byref(seg), ctypes.byref(ws), None) == A.EBTC_OK:
                need = max(need, ws.value)
                break
        for alt in ("balanced", "paneled"):
            o2 = make_opts(**{**kw, "spmv": alt})
            if A.lib().ebtc_plan(self.handle, ctypes.byref(o2), ctypes.byref(ws), None) == A.EBTC_OK:
                need = max(need, ws.value)
        wst = torch.empty(max(1, need), dtype=torch.uint8, device=self.device)
        form, lanes, segl = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ms = (ctypes.c_double * A.TUNE_SLOTS)()
        A.check(A.lib().ebtc_tune(self.handle, ctypes.byref(opts), _vp(wst), need, ctypes.byref(form),
                                  ctypes.byref(lanes), ctypes.byref(segl), ms, current_stream()))
        names = {v: k for k, v in A.SPMV_FORMS.items()}
        labels = ["stream", "lanes4", "lanes8", "lanes16", "lanes32", "staged", f"segmented{small}",
                  f"segmented{2 * small}", "balanced", "paneled"]
        return {"form": "mixed" if form.value == 0 else names[form.value], "lanes": lanes.value,
                "seg_len": segl.value, "ms_per_launch": {l: ms[i] for i, l in enumerate(labels) if ms[i] >= 0},
                "graph_forms": self.tuned_forms()}

    def tuned_forms(self) -> list:
        """Each graph's recorded SpMV form (ebtc_tuned_forms): [(form name, lanes, seg_len)]."""
        f = np.zeros(self.G, dtype=np.int32)
        l = np.zeros(self.G, dtype=np.int32)
        q = np.zeros(self.G, dtype=np.int32)
        A.check(A.lib().ebtc_tuned_forms(self.handle, f.ctypes.data, l.ctypes.data, q.ctypes.data))
        names = {v: k for k, v in A.SPMV_FORMS.items()}
        return [(names[int(a)], int(b), int(c)) for a, b, c in zip(f, l, q)]

    def set_forms(self, forms: list) -> None:
        """Records each graph's SpMV form for spmv="auto" calls (ebtc_set_forms): a list of form names
        or (name, lanes, seg_len) tuples, one per graph."""
        items = [(x, 0, 0) if isinstance(x, str) else tuple(x) for x in forms]
        if len(items) != self.G:
            raise ValueError(f"{len(items)} forms for {self.G} graphs")
        f = np.array([A.SPMV_FORMS[x[0]] for x in items], dtype=np.int32)
        l = np.array([x[1] for x in items], dtype=np.int32)
        q = np.array([x[2] for x in items], dtype=np.int32)
        A.check(A.lib().ebtc_set_forms(self.handle, f.ctypes.data, l.ctypes.data, q.ctypes.data))

    def backward_run(self, **kw) -> "BackwardRun":
        return BackwardRun(self, make_opts(**kw))

    def scores_backward(self, log_scale: torch.Tensor, grad_scores: torch.Tensor, ckpt: torch.Tensor | None = None,
                        **kw) -> torch.Tensor:
        """Gradient of sum_g <grad_scores_g, S~_g> with respect to every stored CSR entry (log-scales
        fixed); `kw` are the options of the forward call. With the forward call's checkpoint (a
        ScoreResult's ckpt, from scores(ckpt=True)) the recomputed forward process must equal it bit
        for bit, else RuntimeError (the values or the options are not the forward's)."""
        out = self.backward_run(**kw).launch(log_scale, grad_scores, ckpt)
        if ckpt is None:
            return out
        grad, mism = out
        bad = int(mism.item())
        if bad:
            raise RuntimeError(f"the backward's recomputed forward differs from the forward checkpoint in {bad} "
                               "realization(s): the batch's values or the options changed since the forward call")
        return grad

    def validate(self) -> int:
        ws = ctypes.c_size_t()
        A.check(A.lib().ebtc_validate_ws_bytes(self.handle, ctypes.byref(ws)))
        wst = torch.empty(max(1, ws.value), dtype=torch.uint8, device=self.device)
        bad = ctypes.c_int64()
        A.check(A.lib().ebtc_validate(self.handle, _vp(wst), ws.value, ctypes.byref(bad), current_stream()))
        return int(bad.value)


def tune_cache_text() -> str:
    """The autotuner's process-wide bucket decisions (ebtc_tune_cache_get): "<key> <form> <lanes> <seg_len>"
    lines."""
    n = ctypes.c_size_t()
    A.check(A.lib().ebtc_tune_cache_get(None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    A.check(A.lib().ebtc_tune_cache_get(buf, n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


def tune_cache_add(text: str) -> None:
    """Merges bucket decisions into the cache (ebtc_tune_cache_put)."""
    A.check(A.lib().ebtc_tune_cache_put(text.encode()))


def tune_cache_clear() -> None:
    A.check(A.lib().ebtc_tune_cache_clear())


def tune_cache_save(path: str) -> None:
    with open(path, "w") as f:
        f.write(tune_cache_text())


def tune_cache_load(path: str) -> None:
    with open(path) as f:
        tune_cache_add(f.read())


def _gen_spec(family: str, n: int, count: int, seed: int, first: int = 0, p: float = 0.0, k: int = 0,
              beta: float = 0.0, targets=None, pattern=None):
    tg = np.ascontiguousarray(np.asarray(targets if targets is not None else [], dtype=np.int32).ravel())
    pt = np.ascontiguousarray(np.asarray(pattern if pattern is not None else np.zeros((0, 2)), dtype=np.int32)
                              .reshape(-1, 2))
    i32p = ctypes.POINTER(ctypes.c_int32)
    spec = A.GenSpec(A.GEN_FAMILIES[family], int(n), float(p), int(k), int(count), float(beta),
                     int(seed) & 0xFFFFFFFFFFFFFFFF, int(first), int(tg.size), int(pt.shape[0]),
                     tg.ctypes.data_as(i32p) if tg.size else None, pt.ctypes.data_as(i32p) if pt.size else None)
    return spec, (tg, pt)


def generate(family: str, n: int, count: int, seed: int, first: int = 0, p: float = 0.0, k: int = 0,
             beta: float = 0.0, targets=None, pattern=None, device: str = "cuda"):
    """Draws `count` realizations on the device (ebtc_generate_count / ebtc_generate_fill): family "er"
    (edge probability p), "ws" (lattice degree k, rewiring beta) or "ba" (k edges per new node), with
    the target pattern (local pairs) embedded on `targets`. Realization r of the call is the family's
    realization first + r of `seed`. Returns (row_ptr int32 [count * (n + 1)], col_idx int32,
    nnz int64 numpy [count])."""
    spec, keep = _gen_spec(family, n, count, seed, first, p, k, beta, targets, pattern)
    ws = ctypes.c_size_t()
    A.check(A.lib().ebtc_generate_plan(ctypes.byref(spec), ctypes.byref(ws)))
    dev = torch.device(device)
    wst = torch.empty(max(1, ws.value), dtype=torch.uint8, device=dev)
    row_ptr = torch.empty(count * (n + 1), dtype=torch.int32, device=dev)
    nnz = torch.empty(count, dtype=torch.int64, device=dev)
    st = current_stream()
    A.check(A.lib().ebtc_generate_count(ctypes.byref(spec), _vp(wst), ws.value, _vp(row_ptr), _vp(nnz), st))
    nnz_h = nnz.cpu().numpy()
    if (nnz_h < 0).any():
        raise A.EbtcError(A.EBTC_EWORKSPACE, "a realization overflowed the candidate buffer or 2^31 entries")
    dest = np.ascontiguousarray(np.concatenate([[0], np.cumsum(nnz_h)[:-1]]).astype(np.int64))
    col = torch.empty(max(1, int(nnz_h.sum())), dtype=torch.int32, device=dev)
    A.check(A.lib().ebtc_generate_fill(ctypes.byref(spec), _vp(wst), ws.value,
                                       dest.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _vp(col), st))
    del keep
    return row_ptr, col[:int(nnz_h.sum())], nnz_h


def generated_batch(graphs: list, dtype: str = "f32", device: str = "cuda", chunk: int = 0,
                    values: bool = False) -> "Batch":
    """A Batch whose realizations are drawn on the device. graphs: dicts with the arguments of
    `generate` (family, n, count = realizations of the graph, seed, first, p / k / beta, targets,
    pattern). chunk > 0 draws at most that many realizations per call (bounds the workspace);
    values: store explicit unit weights (else the pattern-only form, values NULL)."""
    rps, cols, nnz_all, gn, gr = [], [], [], [], []
    for g in graphs:
        g = dict(g)
        count = int(g.pop("count"))
        first = int(g.pop("first", 0))
        step = chunk if chunk > 0 else count
        for c0 in range(0, count, step):
            rp, ci, nz = generate(count=min(step, count - c0), first=first + c0, device=device, **g)
            rps.append(rp)
            cols.append(ci)
            nnz_all.append(nz)
        gn.append(int(g["n"]))
        gr.append(count)
    nnz = np.concatenate(nnz_all)
    rowptr_off = np.concatenate([[0], np.cumsum(np.repeat(np.array(gn, np.int64) + 1, gr))[:-1]])
    nnz_off = np.concatenate([[0], np.cumsum(nnz)]).astype(np.int64)
    col = torch.cat(cols)
    vals = torch.ones(col.numel(), dtype=_DT[dtype][1], device=col.device) if values else None
    return Batch(gn, gr, rowptr_off, nnz_off, torch.cat(rps), col, vals, dtype, device)


def spmv(row_ptr: torch.Tensor, col_idx: torch.Tensor, values: torch.Tensor | None, x: torch.Tensor,
         lanes: int = 0, hub: int = 0, seg_len: int = 0) -> torch.Tensor:
    """y = A x for one CSR matrix on the device (the Krylov step's product); seg_len > 0 stages x in LDS."""
    code = A.EBTC_F64 if x.dtype == torch.float64 else A.EBTC_F32
    y = torch.empty_like(x)
    A.check(A.lib().ebtc_spmv(code, x.numel(), _vp(row_ptr), _vp(col_idx), _vp(values), _vp(x), _vp(y), lanes, hub,
                              seg_len, current_stream()))
    return y


def subgraph_centrality(row_ptr: torch.Tensor, col_idx: torch.Tensor, values: torch.Tensor | None,
                        nodes, m: int = 20, dtype: str = "f32") -> torch.Tensor:
    """[exp(A)]_ii for the given nodes of one graph (device CSR), by the m-point Gauss rule of the
    Lanczos process started at e_i (eq. 3); FP64 results on the device."""
    code = _DT[dtype][0]
    n = int(row_ptr.numel()) - 1
    dev = row_ptr.device
    nd = torch.as_tensor(np.asarray(nodes, dtype=np.int32)).to(dev)
    ws = ctypes.c_size_t()
    A.check(A.lib().ebtc_subgraph_centrality_ws_bytes(code, n, int(nd.numel()), m, ctypes.byref(ws)))
    wst = torch.empty(max(1, ws.value), dtype=torch.uint8, device=dev)
    out = torch.empty(int(nd.numel()), dtype=torch.float64, device=dev)
    A.check(A.lib().ebtc_subgraph_centrality(code, n, _vp(row_ptr), _vp(col_idx), _vp(values), int(nd.numel()),
                                             _vp(nd), m, _vp(out), _vp(wst), ws.value, current_stream()))
    return out


def tridiag_expv(alpha: torch.Tensor, beta: torch.Tensor, shift: bool = True) -> tuple[torch.Tensor, torch.Tensor]:
    """For a [count, k] stack of FP64 tridiagonals: (y = exp(T - theta I) e1 [count, k], theta [count])."""
    count, k = alpha.shape
    y = torch.empty_like(alpha)
    th = torch.empty(count, dtype=torch.float64, device=alpha.device)
    A.check(A.lib().ebtc_tridiag_expv(count, k, _vp(alpha), _vp(beta), _vp(y), _vp(th), int(shift), current_stream()))
    return y, th


class Communicability(torch.autograd.Function):
    """(S~, log_scale) = Communicability.apply(values, batch, opts) with values the batch's edge-weight
    tensor (the very tensor the batch was built on). Backward gives d<grad, S~>/d values through the
    hand-written adjoint (log_scale is treated as a constant)."""

    @staticmethod
    def forward(ctx, values, batch, opts):
        if batch.values is None or values.data_ptr() != batch.values.data_ptr():
            raise ValueError("values must be the tensor the batch was created on")
        out = batch.scores(diag=False, ckpt=True, **opts)
        ctx.batch = batch
        ctx.opts = dict(opts)
        ctx.save_for_backward(out.log_scale, out.ckpt)
        ctx.mark_non_differentiable(out.log_scale)
        return out.scores, out.log_scale

    @staticmethod
    def backward(ctx, grad_scores, _grad_log_scale):
        # the forward's checkpoint guards the recomputation: values changed in place between forward
        # and backward raise instead of giving the gradient of other weights
        log_scale, ckpt = ctx.saved_tensors
        g = ctx.batch.scores_backward(log_scale, grad_scores, ckpt=ckpt, **ctx.opts)
        return g, None, None
