// The whole Lanczos process of one realization in one workgroup (gfx950, 256 threads), for batches
// whose realizations each fit one row block (n <= kRowsPerBlock) and need at most 64 steps: the tiny
// plain-method workload and the identification-rate experiments (backgrounds of 1024-9000 nodes,
// "Multiple backgrounds scenario"), where each phase of the per-phase schedule is a launch over a few
// kilobytes and the run is launch latency.
//
// One launch replaces the per-phase sequence start, [SpMV, Gram-Schmidt dots and update, adaptive
// check] x m, small exponential, basis combination: workgroup barriers take the place of kernel
// boundaries, and the realization's working set stays in LDS -- the state, the partial sums, the row
// pointers, the gathered vector v_j and the product w always; the basis and the CSR entries when they
// fit the launch's LDS budget (the host decides per launch), else the workspace and the input arrays.
// Every phase calls the per-phase kernels' own device functions (step_device.h) with their thread
// layouts: the CSR-stream SpMV arithmetic (which the column-segmented and entry-balanced forms share
// bit for bit), the dot partials in the thread order of the dot kernel the window would get (1024 or
// 256 threads; a partial's bits do not depend on how many vectors one pass covers, so they are formed
// eight vectors at a time), the update and norm of the 256-thread update kernel, the same small
// exponential and combination. So a realization's results equal the per-phase schedule's bit for bit
// whichever schedule its batch takes; only where the data lives changes.
#include <algorithm>

#include "step_device.h"

namespace ebtc {
namespace {

constexpr int kSolveCap = kRowsPerBlock;  // product slots: every row of a simple graph on <= 2048 nodes fits
constexpr int kSolveRed = (kDotsThreads / 64) * 8;

// Dynamic LDS of one launch (byte offsets, host-computed from the largest realization).
struct SolveLds {
  int32_t x_off, w_off, rp_off;  // v_j, w (n_max elements each), row pointers (n_max + 1)
  int32_t v_off;                 // basis ((steps + 1) x n_max elements), or -1: in the workspace
  int32_t c_off, val_off;        // CSR columns and values (z_max each), or -1: read from the input
  int32_t z_max;
  int32_t bytes;
};

template <typename T, int NT>
__device__ inline void solve_dots(const T* V, int n, int j, const T* ws, double* part, double* red_d) {
  for (int c0 = 0; c0 <= j; c0 += 8) {
    block_dots<T, 8, NT, 0, kBlock>(V, n, c0, min(j, c0 + 7), 0, n, ws, nullptr, nullptr, part + c0, red_d);
    __syncthreads();  // red_d is reused by the next eight vectors
  }
}

__device__ inline void solve_tridiag(const LzArgs& a, RState* st, const double* npart, int64_t r, int mode, int j,
                                     int steps, int shift, double tol, ebtc_diag* diag, double* ckpt, double* chunks,
                                     double* ta, double* tb) {
  const TriPrep p = tridiag_prepare(a, st, npart, 1, r, mode, j, steps, diag, chunks);
  if (!p.exit) {
    if (threadIdx.x < 64) tridiag_load(st, p, ta, tb);
    __syncthreads();
    if (threadIdx.x < 64) tridiag_finish(a, st, r, mode, j, p, ta, tb, shift, tol, diag, ckpt);
  }
  __syncthreads();
}

// w = s_j A v_j with the realization's entries in LDS: one thread per row, the row's products in entry
// order, each rounded to T before its FP64 add -- the CSR-stream form's arithmetic (its products are
// staged in LDS before the sum) -- with the next four entries' loads issued ahead of the adds.
template <typename T, bool HAS_VAL>
__device__ inline void solve_spmv_lds(const int* rp_l, const int32_t* cl, const T* vl, const T* xs, int n, double sj,
                                      T* ws) {
  for (int row = threadIdx.x; row < n; row += kBlock) {
    double acc = 0.0;
    const int e1 = rp_l[row + 1];
    int k = rp_l[row];
    for (; k + 4 <= e1; k += 4) {
      T x[4], v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = xs[cl[k + u]];
        if constexpr (HAS_VAL) v[u] = vl[k + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if constexpr (HAS_VAL) {
          const T pr = v[u] * x[u];
          acc += (double)pr;
        } else {
          acc += (double)x[u];
        }
      }
    }
    for (; k < e1; ++k) {
      const T xv = xs[cl[k]];
      if constexpr (HAS_VAL) {
        const T pr = vl[k] * xv;
        acc += (double)pr;
      } else {
        acc += (double)xv;
      }
    }
    ws[row] = (T)(acc * sj);
  }
}

template <typename T, bool HAS_VAL, bool CSR_LDS>
__device__ inline void solve_spmv(int j, const int32_t* ci, const T* va, const T* xs, int n, double sj, int* rp_l,
                                  T* prod, T* ws, double* red) {
  if constexpr (CSR_LDS) {
    solve_spmv_lds<T, HAS_VAL>(rp_l, ci, va, xs, n, sj, ws);  // v_0 = 1: the row sums of the values
    return;
  }
  if (j == 0)  // A 1: each row's values summed in FP64 in entry order (the first-product kernels)
    spmv_stream_rows<T, HAS_VAL, kBlock, kSolveCap, true, true, !CSR_LDS>(nullptr, ci, va, xs, 0, n, sj, rp_l, prod,
                                                                          ws, red);
  else
    spmv_stream_rows<T, HAS_VAL, kBlock, kSolveCap, false, true, !CSR_LDS>(nullptr, ci, va, xs, 0, n, sj, rp_l, prod,
                                                                           ws, red);
}

template <typename T, bool HAS_VAL, bool CSR_LDS>
__global__ __launch_bounds__(kBlock) void k_solve_1(LzArgs a, SolveLds L, int steps, int shift, double tol,
                                                    ebtc_diag* diag, double* ckpt) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ T prod[kSolveCap];
  __shared__ double red_d[kSolveRed];
  __shared__ double cs[64];
  __shared__ double csum[64][kMaxChunks];
  __shared__ double red[kWaves];
  __shared__ double chunks[kMaxChunks];
  __shared__ double ta[kMLimit];
  __shared__ double tb[kMLimit];
  __shared__ double dcoef[kMLimit];
  __shared__ double part_l[kPartStride];
  __shared__ double npart_l[1];
  __shared__ RState st_l;
  const Ref ref = resolve(a);  // ref.blk == 0: one row block per realization
  const int64_t r = ref.task;
  const Task tk = a.tasks[r];
  const int n = tk.n, tid = threadIdx.x;
  T* xs = (T*)(dyn + L.x_off);
  T* ws = (T*)(dyn + L.w_off);
  int* rp_l = (int*)(dyn + L.rp_off);
  T* V = L.v_off >= 0 ? (T*)(dyn + L.v_off) : (T*)a.V + tk.vec_off;
  const int32_t* rp = a.row_ptr + tk.rowptr_off;
  for (int i = tid; i <= n; i += kBlock) rp_l[i] = rp[i];
  const int32_t* ci = a.col_idx + tk.nnz_off;
  const T* va = HAS_VAL ? (const T*)a.values + tk.nnz_off : nullptr;
  if constexpr (CSR_LDS) {  // the realization's entries, once, into LDS
    const int z = min(rp[n], L.z_max);
    int32_t* cl = (int32_t*)(dyn + L.c_off);
    for (int e = tid; e < z; e += kBlock) cl[e] = __builtin_nontemporal_load(ci + e);
    if constexpr (HAS_VAL) {
      T* vl = (T*)(dyn + L.val_off);
      for (int e = tid; e < z; e += kBlock) vl[e] = __builtin_nontemporal_load(va + e);
      va = vl;
    }
    ci = cl;
  }
  // start (k_start): raw v_0 = 1 with scale s_0 = 1/sqrt(n)
  for (int i = tid; i < n; i += kBlock) {
    V[i] = (T)1;
    xs[i] = (T)1;
  }
  RState* st = &st_l;
  if (tid == 0) {
    st->beta0 = sqrt((double)n);
    st->s[0] = 1.0 / st->beta0;
    st->theta = 0.0;
    st->est = 0.0;
    st->m_used = 0;
    st->flags = 0;
    st->done = 0;
  }
  __syncthreads();
  const StepMem<T> mem{st, V, part_l, npart_l};
  constexpr bool F64 = sizeof(T) == 8;
  for (int j = 0; j < steps; ++j) {
    double sj;
    if (!open_step(a, tk, st, 0, j, chunks, &sj, npart_l)) break;  // every thread gets the same answer
    solve_spmv<T, HAS_VAL, CSR_LDS>(j, ci, va, xs, n, sj, rp_l, prod, ws, red);
    __syncthreads();
    // the dot kernel's thread count for this window (dots_threads of its window class)
    const int cnt = j + 1, P = cnt <= 8 ? 8 : cnt <= 16 ? 16 : cnt <= 32 ? 32 : 64;
    if (dots_threads(P, F64 ? 8 : 4) == kDotsThreads) solve_dots<T, kDotsThreads>(V, n, j, ws, part_l, red_d);
    else solve_dots<T, kBlock>(V, n, j, ws, part_l, red_d);
    update_body<T, 64, 0>(a, tk, mem, 0, j, 1, 1, 0, cs, csum, red, ws, xs);
    __syncthreads();  // v~_{j+1} and the norm partial are complete
    if (a.m_fixed == 0) solve_tridiag(a, st, npart_l, r, 1, j, steps, shift, tol, nullptr, nullptr, chunks, ta, tb);
  }
  solve_tridiag(a, st, npart_l, r, 0, 0, steps, shift, tol, diag, ckpt, chunks, ta, tb);
  // combination (k_combine): u = sum_i (beta0 y_i s_i) Vraw_i, FP64, i ascending
  const int k = st->m_used;
  if (tid < k) dcoef[tid] = st->beta0 * st->y[tid] * st->s[tid];
  __syncthreads();
  T* u = (T*)a.U + tk.u_off;
  bool finite = true;
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int row = q * kBlock + tid;
    if (row < n) {
      double acc = 0.0;
      for (int i = 0; i < k; ++i) acc += dcoef[i] * (double)V[(size_t)i * n + row];
      const T out = (T)acc;
      u[row] = out;
      finite = finite && isfinite((double)out);
    }
  }
  if (__syncthreads_or(!finite) && tid == 0) {
    st->flags |= EBTC_FLAG_NONFINITE;
    if (diag) atomicOr(&diag[r].flags, EBTC_FLAG_NONFINITE);
  }
  __syncthreads();
  // the state to the workspace (the realization sum reads theta)
  const double* src = (const double*)st;
  double* dst = (double*)(a.state + r);
  static_assert(sizeof(RState) % sizeof(double) == 0, "state copy");
  for (int i = tid; i < (int)(sizeof(RState) / sizeof(double)); i += kBlock) dst[i] = src[i];
}

// Static LDS of an instantiation (queried once) and its opt-in to the rest of the 160 KB as dynamic LDS.
template <typename T, bool HAS_VAL, bool CSR_LDS>
size_t solve_static_bytes(hipError_t* err) {
  static size_t bytes = 0;
  static const hipError_t e = [] {
    hipFuncAttributes fa{};
    hipError_t r = hipFuncGetAttributes(&fa, (const void*)k_solve_1<T, HAS_VAL, CSR_LDS>);
    if (r != hipSuccess) return r;
    bytes = fa.sharedSizeBytes;
    return hipFuncSetAttribute((const void*)k_solve_1<T, HAS_VAL, CSR_LDS>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsBytes - bytes));
  }();
  *err = e;
  return bytes;
}

template <typename T, bool HAS_VAL>
hipError_t prepare_solve_t() {
  hipError_t e = hipSuccess;
  solve_static_bytes<T, HAS_VAL, true>(&e);
  if (e == hipSuccess) solve_static_bytes<T, HAS_VAL, false>(&e);
  return e;
}

size_t align16(size_t x) { return (x + 15) / 16 * 16; }

// LDS plan of a launch: v_j, w and the row pointers always; then the basis, then the CSR entries,
// each where it still fits next to what is placed.
SolveLds solve_lds(size_t es, bool has_val, int n_max, int64_t z_max, int steps, size_t budget) {
  SolveLds L{};
  size_t off = 0;
  L.x_off = (int32_t)off;
  off = align16(off + (size_t)n_max * es);
  L.w_off = (int32_t)off;
  off = align16(off + (size_t)n_max * es);
  L.rp_off = (int32_t)off;
  off = align16(off + (size_t)(n_max + 1) * 4);
  const size_t vb = (size_t)(steps + 1) * n_max * es;
  L.v_off = -1;
  if (off + vb <= budget) {
    L.v_off = (int32_t)off;
    off = align16(off + vb);
  }
  const size_t cb = align16((size_t)z_max * 4) + (has_val ? (size_t)z_max * es : 0);
  L.c_off = L.val_off = -1;
  if (off + cb <= budget) {
    L.c_off = (int32_t)off;
    off = align16(off + (size_t)z_max * 4);
    if (has_val) {
      L.val_off = (int32_t)off;
      off = align16(off + (size_t)z_max * es);
    }
  }
  L.z_max = (int32_t)std::min<int64_t>(z_max, INT32_MAX);
  L.bytes = (int32_t)off;
  return L;
}

template <typename T, bool HAS_VAL>
hipError_t solve_t(const LzArgs& a, int64_t count, int steps, int shift, double tol, ebtc_diag* diag, double* ckpt,
                   int n_max, int64_t z_max, hipStream_t s) {
  hipError_t e1 = hipSuccess, e2 = hipSuccess;
  const size_t st_csr = solve_static_bytes<T, HAS_VAL, true>(&e1);
  const size_t st_glob = solve_static_bytes<T, HAS_VAL, false>(&e2);
  if (e1 != hipSuccess) return e1;
  if (e2 != hipSuccess) return e2;
  const SolveLds L = solve_lds(sizeof(T), HAS_VAL, n_max, z_max, steps, kLdsBytes - std::max(st_csr, st_glob));
  const dim3 g((unsigned)count), b(kBlock);
  if (L.c_off >= 0)
    hipLaunchKernelGGL((k_solve_1<T, HAS_VAL, true>), g, b, (size_t)L.bytes, s, a, L, steps, shift, tol, diag, ckpt);
  else
    hipLaunchKernelGGL((k_solve_1<T, HAS_VAL, false>), g, b, (size_t)L.bytes, s, a, L, steps, shift, tol, diag, ckpt);
  return hipGetLastError();
}

}  // namespace

hipError_t prepare_solve_kernels() {
  static const hipError_t e = [] {
    hipError_t r = prepare_solve_t<float, true>();
    if (r == hipSuccess) r = prepare_solve_t<float, false>();
    if (r == hipSuccess) r = prepare_solve_t<double, true>();
    if (r == hipSuccess) r = prepare_solve_t<double, false>();
    return r;
  }();
  return e;
}

hipError_t launch_solve_1(int dtype, bool has_val, const LzArgs& a, int64_t count, int steps, int shift, double tol,
                          ebtc_diag* diag, double* ckpt, int n_max, int64_t z_max, hipStream_t s) {
  if (a.window != 0 || n_max < 1 || n_max > kRowsPerBlock || steps < 1 || steps > kDotsWindow)
    return hipErrorInvalidValue;
  if (dtype == EBTC_F64)
    return has_val ? solve_t<double, true>(a, count, steps, shift, tol, diag, ckpt, n_max, z_max, s)
                   : solve_t<double, false>(a, count, steps, shift, tol, diag, ckpt, n_max, z_max, s);
  return has_val ? solve_t<float, true>(a, count, steps, shift, tol, diag, ckpt, n_max, z_max, s)
                 : solve_t<float, false>(a, count, steps, shift, tol, diag, ckpt, n_max, z_max, s);
}

}  // namespace ebtc
