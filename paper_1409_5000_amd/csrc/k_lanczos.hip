// Lanczos streaming kernels for gfx950 (MI355X, wave64).
//
// One Lanczos step j of exp(A) 1 (Krylov approximation, "The total communicability", eq. (4)):
//   phase A  closes step j-1 (beta_{j-1} from the norm partials, breakdown test, scale 1/beta_{j-1}
//            of the unnormalised basis vector), then w = A v_j (CSR SpMV) and the per-workgroup
//            partial dot products <v_i, w>, i <= j;
//   phase B  reduces the dot partials, v~_{j+1} = w - sum_i h_i v_i (classical Gram-Schmidt against
//            the whole basis) and the per-workgroup partial squared norm.
// Workgroups never wait for each other inside a kernel and use no device-scope fences or atomics
// (the adaptive check alone counts the running realizations with an integer atomic, which the next
// step's kernels read): partial sums go to memory and the next kernel (after the launch boundary)
// reduces them. Every
// reader uses the same canonical summation order, so all of them see bit-identical totals.
// Every workgroup owns kRowsPerBlock consecutive rows of one realization. Launches either cover
// one realization (plain loop) or every realization of the batch at once (batched), in which case
// a table maps each workgroup to its realization.
//
// Memory layout: basis vectors are vector-major (V[i][0..n)), so every phase streams them with
// fully coalesced loads; the SpMV gathers from the one contiguous vector v_j.
#include <algorithm>

#include "step_device.h"

namespace ebtc {
namespace {


// k_dots_step: dot partials of w (written by the SpMV) against the window of Vraw_0..j, from its c0-th
// vector on (at most P of them: a window wider than kDotsWindow takes one launch per kDotsWindow).
template <typename T, int P, int RING>
__global__ __launch_bounds__(dots_threads(P, sizeof(T))) void k_dots_step(LzArgs a, int j, int c0) {
  if (all_stopped(a, j)) return;
  constexpr int NT = dots_threads(P, sizeof(T));
  __shared__ double red[(NT / 64) * P];
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  const RState* st = a.state + ref.task;
  if (step_skipped(a, st, j)) return;
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  const T* Vr = (const T*)a.V + tk.vec_off;
  const int lo = window_lo(a, j) + c0;
  block_dots<T, P, NT, RING>(Vr, n, lo, min(j, lo + P - 1), r0, r1, nullptr, (const T*)a.W + tk.w_off, nullptr,
                             a.part + tk.part_off + (size_t)ref.blk * kPartStride + c0, red);
}

// Second Gram-Schmidt pass: dots of the once-orthogonalised vector (stored in the slot of j+1).
template <typename T, int P, int RING>
__global__ __launch_bounds__(kBlock) void k_dots_again(LzArgs a, int j, int c0) {
  if (all_stopped(a, j)) return;
  __shared__ double red[kWaves * P];
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  const RState* st = a.state + ref.task;
  if (step_skipped(a, st, j)) return;
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  const T* Vr = (const T*)a.V + tk.vec_off;
  const int lo = window_lo(a, j) + c0;
  block_dots<T, P, kBlock, RING>(Vr, n, lo, min(j, lo + P - 1), r0, r1, nullptr, Vr + vslot(a, j + 1) * n,
                                 nullptr, a.part + tk.part_off + (size_t)ref.blk * kPartStride + c0, red);
}


template <typename T, int P, int RING>
__global__ __launch_bounds__(kBlock) void k_update(LzArgs a, int j, int from_w, int final_pass, int second) {
  if (all_stopped(a, j)) return;
  __shared__ double cs[P];
  __shared__ double csum[P][kMaxChunks];
  __shared__ double red[kWaves];
  const Ref ref = resolve(a);
  if (step_skipped(a, a.state + ref.task, j)) return;
  const Task tk = a.tasks[ref.task];
  update_body<T, P, RING>(a, tk, step_mem<T>(a, tk, ref.task), ref.blk, j, from_w, final_pass, second, cs, csum,
                          red);
}

// Dots and update of step j in one launch, for batches whose realizations each fit one row block
// (n <= kRowsPerBlock, one workgroup per realization): the workgroup's dot partials are then the
// realization's totals, so the update reads them back after a workgroup barrier instead of after a
// launch boundary. Same steps as k_dots_step followed by k_update (one Gram-Schmidt pass, full basis),
// with k_dots_step's thread order for the partials, so the bits do not depend on which of the two
// paths a batch takes.
template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_dots_update_1(LzArgs a, int j) {
  if (all_stopped(a, j)) return;
  constexpr int NT = dots_threads(P, sizeof(T));
  __shared__ double red_d[(NT / 64) * P];
  __shared__ double cs[P];
  __shared__ double csum[P][kMaxChunks];
  __shared__ double red[kWaves];
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  if (step_skipped(a, a.state + ref.task, j)) return;
  const int n = min(tk.n, kRowsPerBlock);
  block_dots<T, P, NT, 0, kBlock>((const T*)a.V + tk.vec_off, tk.n, 0, j, 0, n, nullptr, (const T*)a.W + tk.w_off,
                                  nullptr, a.part + tk.part_off, red_d);
  __syncthreads();  // the partials stored above (global) are read back by other threads of the workgroup
  update_body<T, P, 0>(a, tk, step_mem<T>(a, tk, ref.task), ref.blk, j, 1, 1, 0, cs, csum, red);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_start(LzArgs a) {
  if (a.live != nullptr && blockIdx.x == 0)
    for (int i = threadIdx.x; i < kMLimit; i += kBlock) a.live[i] = 0;
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  T* v0 = (T*)a.V + tk.vec_off;
  for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) v0[r] = (T)1;  // v_0 = s_0 * 1, s_0 = 1/sqrt(n)
  if (ref.blk == 0 && threadIdx.x == 0) {
    RState* st = a.state + ref.task;
    st->beta0 = sqrt((double)n);
    st->s[0] = 1.0 / st->beta0;
    st->theta = 0.0;
    st->est = 0.0;
    st->m_used = 0;
    st->flags = 0;
    st->done = 0;
  }
}

// Second pass of the memory-bounded form: the same start vector and scale as k_start, keeping
// theta, y, est, m_used and flags of the first pass.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restart(LzArgs a) {
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  T* v0 = (T*)a.V + tk.vec_off;
  for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) v0[r] = (T)1;
  if (ref.blk == 0 && threadIdx.x == 0) {
    RState* st = a.state + ref.task;
    st->s[0] = 1.0 / st->beta0;
    st->done = 0;
  }
}

// Before step j of the second pass: u = beta0 sum_{i <= j} y_i s_i Vraw_i, one term per step (the
// vector of step j is in its ring slot now and is overwritten three steps later), for j < m_used.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_accum(LzArgs a, int j) {
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  const RState* st = a.state + ref.task;
  if (st->done || j >= st->m_used) return;
  const double d = st->beta0 * st->y[j] * st->s[j];
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  const T* v = (const T*)a.V + tk.vec_off + vslot(a, j) * n;
  T* u = (T*)a.U + tk.u_off;
  for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock)
    u[r] = (T)((j == 0 ? 0.0 : (double)u[r]) + d * (double)v[r]);
}

// Start of the Gauss-quadrature processes of subgraph centrality: task r starts at e_{nodes[r]}
// (raw basis vector 0 = e_i with scale s_0 = 1, beta0 = ||e_i|| = 1). A node id outside [0, n)
// leaves v_0 = 0, which the first step closes as a breakdown; k_sc_out reports it as NaN.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_start_unit(LzArgs a, const int32_t* nodes) {
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  const int node = nodes[ref.task];
  T* v0 = (T*)a.V + tk.vec_off;
  for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) v0[r] = r == node ? (T)1 : (T)0;
  if (ref.blk == 0 && threadIdx.x == 0) {
    RState* st = a.state + ref.task;
    st->beta0 = 1.0;
    st->s[0] = 1.0;
    st->theta = 0.0;
    st->est = 0.0;
    st->m_used = 0;
    st->flags = 0;
    st->done = 0;
  }
}

// SC(i) ~ e1^T exp(T) e1 = e^{theta*} y_0 (eq. 3 by the Gauss rule of the process started at e_i).
__global__ __launch_bounds__(kBlock) void k_sc_out(const RState* state, const Task* tasks, const int32_t* nodes,
                                                   int64_t count, double* out) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= count) return;
  const RState* st = state + r;
  const int node = nodes[r];
  const bool ok = node >= 0 && node < tasks[r].n && st->m_used >= 1;
  out[r] = ok ? exp(st->theta) * st->y[0] : __builtin_nan("");
}

// u = beta0 * sum_i y_i v_i = sum_i (beta0 y_i s_i) Vraw_i, so exp(A) 1 ~ e^{theta*} u.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_combine(LzArgs a) {
  __shared__ double d[kMLimit];
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  const RState* st = a.state + ref.task;
  const int k = st->m_used;  // >= 1 once the steps ran
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  if ((int)threadIdx.x < k) d[threadIdx.x] = st->beta0 * st->y[threadIdx.x] * st->s[threadIdx.x];
  __syncthreads();
  const T* Vr = (const T*)a.V + tk.vec_off;
  T* u = (T*)a.U + tk.u_off;
  bool finite = true;
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int r = r0 + q * kBlock + (int)threadIdx.x;
    if (r < r1) {
      double acc = 0.0;
      for (int i = 0; i < k; ++i) acc += d[i] * (double)Vr[(size_t)i * n + r];
      const T out = (T)acc;
      u[r] = out;
      finite = finite && isfinite((double)out);
    }
  }
  // e.g. exp(A) 1 beyond the working range when the shift is switched off
  if (__syncthreads_or(!finite) && threadIdx.x == 0) {
    atomicOr(&a.state[ref.task].flags, EBTC_FLAG_NONFINITE);
    if (a.diag) atomicOr(&a.diag[ref.task].flags, EBTC_FLAG_NONFINITE);
  }
}

// eq. (5) in scaled form: S~_g = sum_k e^{theta_k - Sigma_g} u_k, k ascending, FP64 weights and
// accumulation; Sigma_g = max_k theta_k.
// One workgroup per kSumRows rows of a graph (one row per thread, so that a small batch of graphs
// still spreads over the CUs); each thread adds its row over the graph's realizations in order k,
// kSumU loads in flight at a time.
constexpr int kSumRows = kBlock;
constexpr int kSumU = 8;
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sum(const GraphInfo* graphs, const Task* tasks, const RState* state,
                                                 const T* U, T* scores, double* log_scale) {
  __shared__ double wk[kBlock];
  __shared__ int64_t uo[kBlock];
  __shared__ double sig;
  const GraphInfo gi = graphs[blockIdx.y];
  const int r0 = blockIdx.x * kSumRows;
  if (r0 >= gi.n) return;
  const int tid = threadIdx.x, r = r0 + tid;
  if (tid < 64) {
    double m = -INFINITY;
    for (int k = tid; k < gi.count; k += 64) m = fmax(m, state[gi.first + k].theta);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (tid == 0) sig = m;
  }
  __syncthreads();
  double acc = 0.0;
  for (int kb = 0; kb < gi.count; kb += kBlock) {
    const int cnt = min(kBlock, gi.count - kb);
    if (tid < cnt) {
      wk[tid] = exp(state[gi.first + kb + tid].theta - sig);
      uo[tid] = tasks[gi.first + kb + tid].u_off;
    }
    __syncthreads();
    if (r < gi.n) {
      for (int k0 = 0; k0 < cnt; k0 += kSumU) {
        T v[kSumU];
#pragma unroll
        for (int u = 0; u < kSumU; ++u) v[u] = k0 + u < cnt ? U[uo[k0 + u] + r] : (T)0;
#pragma unroll
        for (int u = 0; u < kSumU; ++u)
          if (k0 + u < cnt) acc += wk[k0 + u] * (double)v[u];
      }
    }
    __syncthreads();
  }
  if (r < gi.n) scores[gi.score_off + r] = (T)acc;
  if (blockIdx.x == 0 && tid == 0) log_scale[blockIdx.y] = sig;
}

// Largest row length of each realization (the autotuner's measure of hub rows), one workgroup each.
__global__ __launch_bounds__(kBlock) void k_row_max(const Task* tasks, const int32_t* row_ptr, int32_t* out) {
  __shared__ int red[kBlock / 64];
  const Task tk = tasks[blockIdx.x];
  const int32_t* rp = row_ptr + tk.rowptr_off;
  int m = 0;
  for (int r = threadIdx.x; r < tk.n; r += kBlock) m = max(m, rp[r + 1] - rp[r]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    int v = 0;
    for (int i = 0; i < kBlock / 64; ++i) v = max(v, red[i]);
    out[blockIdx.x] = v;
  }
}

__global__ void k_blkmap(const Task* tasks, int32_t* blkmap) {
  const Task tk = tasks[blockIdx.x];
  for (int b = threadIdx.x; b < tk.nblk; b += blockDim.x) blkmap[tk.blk_begin + b] = (int32_t)blockIdx.x;
}

}  // namespace

hipError_t launch_row_max(const Task* tasks, const int32_t* row_ptr, int64_t R, int32_t* out, hipStream_t s) {
  if (R < 1) return hipSuccess;
  hipLaunchKernelGGL(k_row_max, dim3((unsigned)R), dim3(kBlock), 0, s, tasks, row_ptr, out);
  return hipGetLastError();
}

hipError_t launch_blkmap(const Task* tasks, int64_t R, int32_t* blkmap, hipStream_t s) {
  hipLaunchKernelGGL(k_blkmap, dim3((unsigned)R), dim3(256), 0, s, tasks, blkmap);
  return hipGetLastError();
}

hipError_t launch_start(int dtype, const LzArgs& a, int64_t nb, hipStream_t s) {
  if (dtype == EBTC_F64)
    hipLaunchKernelGGL(k_start<double>, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_start<float>, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_start_unit(int dtype, const LzArgs& a, const int32_t* nodes, int64_t nb, hipStream_t s) {
  if (dtype == EBTC_F64)
    hipLaunchKernelGGL(k_start_unit<double>, dim3((unsigned)nb), dim3(kBlock), 0, s, a, nodes);
  else
    hipLaunchKernelGGL(k_start_unit<float>, dim3((unsigned)nb), dim3(kBlock), 0, s, a, nodes);
  return hipGetLastError();
}

hipError_t launch_sc_out(const RState* state, const Task* tasks, const int32_t* nodes, int64_t count, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_sc_out, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, state, tasks,
                     nodes, count, out);
  return hipGetLastError();
}

// Basis vectors in the Gram-Schmidt window of step j.
int window_count(const LzArgs& a, int j) { return a.window > 0 ? std::min(j + 1, (int)a.window) : j + 1; }

hipError_t launch_restart(int dtype, const LzArgs& a, int64_t nb, hipStream_t s) {
  if (dtype == EBTC_F64)
    hipLaunchKernelGGL(k_restart<double>, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_restart<float>, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_accum(int dtype, const LzArgs& a, int j, int64_t nb, hipStream_t s) {
  if (dtype == EBTC_F64)
    hipLaunchKernelGGL(k_accum<double>, dim3((unsigned)nb), dim3(kBlock), 0, s, a, j);
  else
    hipLaunchKernelGGL(k_accum<float>, dim3((unsigned)nb), dim3(kBlock), 0, s, a, j);
  return hipGetLastError();
}

// Gram-Schmidt kernels by basis window: the memory-bounded form (window 2, ring of three slots)
// takes the two-vector instantiation; the full basis takes 8, 16, 32 or 64 vectors per launch (WC:
// the vectors this launch covers) and the update 8 to 128.
#define EBTC_GS_LAUNCH(KERNEL, T, WC, ...)                                               \
  do {                                                                                   \
    if (a.window > 0) {                                                                  \
      if (a.window != 2) return hipErrorInvalidValue;                                    \
      hipLaunchKernelGGL((KERNEL<T, 2, 3>), g, b, 0, s, __VA_ARGS__);                    \
    } else if ((WC) <= 8) {                                                              \
      hipLaunchKernelGGL((KERNEL<T, 8, 0>), g, b, 0, s, __VA_ARGS__);                    \
    } else if ((WC) <= 16) {                                                             \
      hipLaunchKernelGGL((KERNEL<T, 16, 0>), g, b, 0, s, __VA_ARGS__);                   \
    } else if ((WC) <= 32) {                                                             \
      hipLaunchKernelGGL((KERNEL<T, 32, 0>), g, b, 0, s, __VA_ARGS__);                   \
    } else {                                                                             \
      hipLaunchKernelGGL((KERNEL<T, 64, 0>), g, b, 0, s, __VA_ARGS__);                   \
    }                                                                                    \
  } while (0)

// Window size class of a dot launch covering wc vectors.
int dots_p(const LzArgs& a, int wc) { return a.window > 0 ? 2 : wc <= 8 ? 8 : wc <= 16 ? 16 : (wc <= 32 ? 32 : 64); }

hipError_t launch_dots_step(int dtype, int j, const LzArgs& a, int64_t nb, hipStream_t s) {
  if (a.window > 0 && a.window != 2) return hipErrorInvalidValue;
  const int wc = window_count(a, j);
  for (int c0 = 0; c0 < wc; c0 += kDotsWindow) {
    const int wcc = std::min(kDotsWindow, wc - c0);
    const dim3 g((unsigned)nb), b(dots_threads(dots_p(a, wcc), dtype == EBTC_F64 ? 8 : 4));
    if (dtype == EBTC_F64) EBTC_GS_LAUNCH(k_dots_step, double, wcc, a, j, c0);
    else EBTC_GS_LAUNCH(k_dots_step, float, wcc, a, j, c0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_dots_again(int dtype, int j, const LzArgs& a, int64_t nb, hipStream_t s) {
  const int wc = window_count(a, j);
  for (int c0 = 0; c0 < wc; c0 += kDotsWindow) {
    const int wcc = std::min(kDotsWindow, wc - c0);
    const dim3 g((unsigned)nb), b(kBlock);
    if (dtype == EBTC_F64) EBTC_GS_LAUNCH(k_dots_again, double, wcc, a, j, c0);
    else EBTC_GS_LAUNCH(k_dots_again, float, wcc, a, j, c0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_update(int dtype, int j, bool from_w, bool final_pass, bool second_pass, const LzArgs& a,
                         int64_t nb, hipStream_t s) {
  const dim3 g((unsigned)nb), b(kBlock);
  const int fw = from_w ? 1 : 0, fp = final_pass ? 1 : 0, sp = second_pass ? 1 : 0;
  const int wc = window_count(a, j);
  if (a.window == 0 && wc > 64) {  // windows of 65 to 128 vectors
    if (dtype == EBTC_F64) hipLaunchKernelGGL((k_update<double, 128, 0>), g, b, 0, s, a, j, fw, fp, sp);
    else hipLaunchKernelGGL((k_update<float, 128, 0>), g, b, 0, s, a, j, fw, fp, sp);
    return hipGetLastError();
  }
  if (dtype == EBTC_F64) EBTC_GS_LAUNCH(k_update, double, wc, a, j, fw, fp, sp);
  else EBTC_GS_LAUNCH(k_update, float, wc, a, j, fw, fp, sp);
  return hipGetLastError();
}

hipError_t launch_dots_update_1(int dtype, int j, const LzArgs& a, int64_t nb, hipStream_t s) {
  if (a.window != 0) return hipErrorInvalidValue;
  const int wc = window_count(a, j);
  if (wc > kDotsWindow) return hipErrorInvalidValue;
  const dim3 g((unsigned)nb), b(kBlock);
#define EBTC_DU1(T)                                                                            \
  do {                                                                                         \
    if (wc <= 8) hipLaunchKernelGGL((k_dots_update_1<T, 8>), g, b, 0, s, a, j);                \
    else if (wc <= 16) hipLaunchKernelGGL((k_dots_update_1<T, 16>), g, b, 0, s, a, j);         \
    else if (wc <= 32) hipLaunchKernelGGL((k_dots_update_1<T, 32>), g, b, 0, s, a, j);         \
    else hipLaunchKernelGGL((k_dots_update_1<T, 64>), g, b, 0, s, a, j);                       \
  } while (0)
  if (dtype == EBTC_F64) EBTC_DU1(double);
  else EBTC_DU1(float);
#undef EBTC_DU1
  return hipGetLastError();
}

#undef EBTC_GS_LAUNCH

hipError_t launch_combine(int dtype, const LzArgs& a, int64_t nb, hipStream_t s) {
  if (dtype == EBTC_F64)
    hipLaunchKernelGGL(k_combine<double>, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_combine<float>, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sum(int dtype, const GraphInfo* graphs, int32_t G, int32_t max_blocks, const Task* tasks,
                      const RState* state, const void* U, void* scores, double* log_scale, hipStream_t s) {
  const dim3 g((unsigned)(max_blocks * (kRowsPerBlock / kSumRows)), (unsigned)G), b(kBlock);
  if (dtype == EBTC_F64)
    hipLaunchKernelGGL(k_sum<double>, g, b, 0, s, graphs, tasks, state, (const double*)U, (double*)scores, log_scale);
  else
    hipLaunchKernelGGL(k_sum<float>, g, b, 0, s, graphs, tasks, state, (const float*)U, (float*)scores, log_scale);
  return hipGetLastError();
}

}  // namespace ebtc
