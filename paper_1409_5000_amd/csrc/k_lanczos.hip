// Lanczos streaming kernels for gfx950 (MI355X, wave64).
//
// One Lanczos step j of exp(A) 1 (Krylov approximation, "The total communicability", eq. (4)):
//   phase A  closes step j-1 (beta_{j-1} from the norm partials, breakdown test, scale 1/beta_{j-1}
//            of the unnormalised basis vector), then w = A v_j (CSR SpMV) and the per-workgroup
//            partial dot products <v_i, w>, i <= j;
//   phase B  reduces the dot partials, v~_{j+1} = w - sum_i h_i v_i (classical Gram-Schmidt against
//            the whole basis) and the per-workgroup partial squared norm.
// Workgroups never wait for each other inside a kernel and use no device-scope fences or atomics:
// partial sums go to memory and the next kernel (after the launch boundary) reduces them. Every
// reader uses the same canonical summation order, so all of them see bit-identical totals.
// Every workgroup owns kRowsPerBlock consecutive rows of one realization. Launches either cover
// one realization (plain loop) or every realization of the batch at once (batched), in which case
// a table maps each workgroup to its realization.
//
// Memory layout: basis vectors are vector-major (V[i][0..n)), so every phase streams them with
// fully coalesced loads; the SpMV gathers from the one contiguous vector v_j.
#include <algorithm>

#include "device_common.h"

namespace ebtc {
namespace {

// Partial dots p_d = sum_rows Vraw_{lo+d}[r] * w[r] (d < cnt = j - lo + 1 <= P) of this workgroup's
// rows, reduced over the workgroup (NT threads) and stored to part_blk[d]. Basis loads are issued
// min(P, 8) vectors at a time (clamped to the last one, whose extra contributions are masked) so that
// many loads are in flight per thread. RING > 0: vector i lives in slot i % RING (the ring of the
// memory-bounded form). red: (NT / 64) * P doubles of LDS.
template <typename T, int P, int NT, int RING>
__device__ inline void block_dots(const T* __restrict__ Vr, int n, int lo, int j, int r0, int r1,
                                  const T* wsrc_lds, const T* wsrc_glob, T* wstore, double* part_blk, double* red) {
  static_assert(P == 2 || P == 8 || P == 16 || P == 32 || P == 64, "lane layout of ReduceScatter");
  constexpr int RPT = kRowsPerBlock / NT;
  constexpr int CH = P < 8 ? P : 8;
  const int tid = threadIdx.x, cnt = j - lo + 1;
  T p[P];
#pragma unroll
  for (int i = 0; i < P; ++i) p[i] = 0;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = r0 + q * NT + tid;
    if (r < r1) {
      const T wv = wsrc_lds ? wsrc_lds[r - r0] : wsrc_glob[r];
      if (wstore) wstore[r] = wv;
#pragma unroll
      for (int d0 = 0; d0 < P; d0 += CH) {
        if (d0 < cnt) {
          T v[CH];
#pragma unroll
          for (int c = 0; c < CH; ++c) {
            const int i = lo + min(d0 + c, cnt - 1);
            v[c] = Vr[(size_t)(RING ? i % RING : i) * n + r];
          }
#pragma unroll
          for (int c = 0; c < CH; ++c) p[d0 + c] += (d0 + c < cnt) ? v[c] * wv : (T)0;
        }
      }
    }
  }
  double pd[P];
#pragma unroll
  for (int i = 0; i < P; ++i) pd[i] = (double)p[i];
  const int lane = tid & 63, wave = tid >> 6;
  ReduceScatter<P, 32>::run(pd, lane);
  constexpr int LP = 64 / P;  // lanes per value after the reduce-scatter: lane l holds value l / LP
  if (lane % LP == 0) red[wave * P + lane / LP] = pd[0];
  __syncthreads();
  if (tid < P && tid < cnt) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w * P + tid];
    part_blk[tid] = s;
  }
}

// First basis vector of the Gram-Schmidt window of step j (all of v_0..v_j without a window).
__device__ inline int window_lo(const LzArgs& a, int j) { return a.window > 0 ? max(0, j - a.window + 1) : 0; }

// Workgroup size of the step's dot partials for windows of P vectors of es-byte elements: the
// two-vector ring, windows of up to 8 vectors and FP32 windows of up to 32 take kDotsThreads (two
// rows per thread, 64 registers, eight waves per SIMD); the rest 256 threads (their accumulators need
// the registers). The first steps use windows of 8 and 16 vectors: a 32-vector one would reduce and
// store 32 partials per workgroup for one to sixteen dots.
__host__ __device__ constexpr int dots_threads(int P, int es) {
  return (P <= 8 || (es == 4 && P <= 32)) ? kDotsThreads : kBlock;
}

// k_dots_step: dot partials of w (written by the SpMV) against the window of Vraw_0..j.
template <typename T, int P, int RING>
__global__ __launch_bounds__(dots_threads(P, sizeof(T))) void k_dots_step(LzArgs a, int j) {
  constexpr int NT = dots_threads(P, sizeof(T));
  __shared__ double red[(NT / 64) * P];
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  const RState* st = a.state + ref.task;
  if (step_skipped(a, st, j)) return;
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  const T* Vr = (const T*)a.V + tk.vec_off;
  block_dots<T, P, NT, RING>(Vr, n, window_lo(a, j), j, r0, r1, nullptr, (const T*)a.W + tk.w_off, nullptr,
                             a.part + tk.part_off + (size_t)ref.blk * kPartStride, red);
}

// Second Gram-Schmidt pass: dots of the once-orthogonalised vector (stored in the slot of j+1).
template <typename T, int P, int RING>
__global__ __launch_bounds__(kBlock) void k_dots_again(LzArgs a, int j) {
  __shared__ double red[kWaves * P];
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  const RState* st = a.state + ref.task;
  if (step_skipped(a, st, j)) return;
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  const T* Vr = (const T*)a.V + tk.vec_off;
  block_dots<T, P, kBlock, RING>(Vr, n, window_lo(a, j), j, r0, r1, nullptr, Vr + vslot(a, j + 1) * n,
                           nullptr, a.part + tk.part_off + (size_t)ref.blk * kPartStride, red);
}

// Phase B of step j: every workgroup reduces the dot partials of all workgroups of its realization
// in the canonical order (identical coefficients everywhere, no inter-workgroup synchronisation),
// then v~_{j+1} = src - sum_i c_i Vraw_i over the window (FP64 accumulation, rounded once), plus
// the partial squared norm on the final pass.
template <typename T, int P, int RING>
__device__ inline void update_body(const LzArgs& a, const Ref& ref, int j, int from_w, int final_pass, int second,
                                   double* cs, double (*csum)[kMaxChunks], double* red) {
  const Task tk = a.tasks[ref.task];
  RState* st = a.state + ref.task;
  constexpr int CH = P < 8 ? P : 8;
  const int tid = threadIdx.x, lo = window_lo(a, j), cnt = j - lo + 1;
  const double* part = a.part + tk.part_off;
  const int nblk = tk.nblk, chunk = part_chunk(nblk), nch = (nblk + chunk - 1) / chunk;
  for (int item = tid; item < nch * cnt; item += kBlock) {
    const int c = item / cnt, d = item - c * cnt;
    double s = 0.0;
    const int b1 = min(nblk, (c + 1) * chunk);
    for (int b = c * chunk; b < b1; ++b) s += part[(size_t)b * kPartStride + d];
    csum[d][c] = s;
  }
  __syncthreads();
  if (tid < P) {
    double coef = 0.0;
    if (tid < cnt) {
      double t = 0.0;
      for (int c = 0; c < nch; ++c) t += csum[tid][c];
      const double si = st->s[lo + tid];
      const double h = si * t;
      coef = h * si;
      if (lo + tid == j && ref.blk == 0) {
        const double alpha = second ? st->alpha[j] + h : h;
        st->alpha[j] = alpha;
        if (final_pass) {  // breakdown reference of step j: max(|alpha_0..j|, beta_0..j-1)
          double sc = fabs(alpha);
          if (j > 0) sc = fmax(sc, fmax(st->scal[j - 1], st->beta[j - 1]));
          st->scal[j] = isfinite(alpha) ? sc : alpha;
        }
      }
    }
    cs[tid] = coef;
  }
  __syncthreads();
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  T* Vr = (T*)a.V + tk.vec_off;
  const T* src = from_w ? (const T*)a.W + tk.w_off : Vr + vslot(a, j + 1) * n;
  T* dst = Vr + vslot(a, j + 1) * n;
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int r = r0 + q * kBlock + tid;
    if (r < r1) {
      double acc = (double)src[r];
#pragma unroll
      for (int d0 = 0; d0 < P; d0 += CH) {
        if (d0 < cnt) {
          T v[CH];
#pragma unroll
          for (int c = 0; c < CH; ++c) {
            const int i = lo + min(d0 + c, cnt - 1);
            v[c] = Vr[(size_t)(RING ? i % RING : i) * n + r];
          }
#pragma unroll
          for (int c = 0; c < CH; ++c) acc -= cs[d0 + c] * (double)v[c];
        }
      }
      const T out = (T)acc;
      dst[r] = out;
      nrm += (double)out * (double)out;
    }
  }
  if (!final_pass) return;
  nrm = block_sum<kBlock>(nrm, red);
  if (tid == 0) a.npart[tk.part_off / kPartStride + ref.blk] = nrm;
}

template <typename T, int P, int RING>
__global__ __launch_bounds__(kBlock) void k_update(LzArgs a, int j, int from_w, int final_pass, int second) {
  __shared__ double cs[P];
  __shared__ double csum[P][kMaxChunks];
  __shared__ double red[kWaves];
  const Ref ref = resolve(a);
  if (step_skipped(a, a.state + ref.task, j)) return;
  update_body<T, P, RING>(a, ref, j, from_w, final_pass, second, cs, csum, red);
}

// Dots and update of step j in one launch, for batches whose realizations each fit one row block
// (n <= kRowsPerBlock, one workgroup per realization): the workgroup's dot partials are then the
// realization's totals, so the update reads them back after a workgroup barrier instead of after a
// launch boundary. Same steps as k_dots_step followed by k_update (one Gram-Schmidt pass, full basis).
template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_dots_update_1(LzArgs a, int j) {
  __shared__ double red_d[kWaves * P];
  __shared__ double cs[P];
  __shared__ double csum[P][kMaxChunks];
  __shared__ double red[kWaves];
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  if (step_skipped(a, a.state + ref.task, j)) return;
  const int n = min(tk.n, kRowsPerBlock);
  block_dots<T, P, kBlock, 0>((const T*)a.V + tk.vec_off, tk.n, 0, j, 0, n, nullptr, (const T*)a.W + tk.w_off,
                              nullptr, a.part + tk.part_off, red_d);
  __syncthreads();  // the partials stored above (global) are read back by other threads of the workgroup
  update_body<T, P, 0>(a, ref, j, 1, 1, 0, cs, csum, red);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_start(LzArgs a) {
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

__global__ void k_blkmap(const Task* tasks, int32_t* blkmap) {
  const Task tk = tasks[blockIdx.x];
  for (int b = threadIdx.x; b < tk.nblk; b += blockDim.x) blkmap[tk.blk_begin + b] = (int32_t)blockIdx.x;
}

}  // namespace

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
// takes the two-vector instantiation; the full basis takes 32 or 64 vectors per launch.
#define EBTC_GS_LAUNCH(KERNEL, T, ...)                                                   \
  do {                                                                                   \
    if (a.window > 0) {                                                                  \
      if (a.window != 2) return hipErrorInvalidValue;                                    \
      hipLaunchKernelGGL((KERNEL<T, 2, 3>), g, b, 0, s, __VA_ARGS__);                    \
    } else if (window_count(a, j) <= 8) {                                                \
      hipLaunchKernelGGL((KERNEL<T, 8, 0>), g, b, 0, s, __VA_ARGS__);                    \
    } else if (window_count(a, j) <= 16) {                                               \
      hipLaunchKernelGGL((KERNEL<T, 16, 0>), g, b, 0, s, __VA_ARGS__);                   \
    } else if (window_count(a, j) <= 32) {                                               \
      hipLaunchKernelGGL((KERNEL<T, 32, 0>), g, b, 0, s, __VA_ARGS__);                   \
    } else {                                                                             \
      hipLaunchKernelGGL((KERNEL<T, 64, 0>), g, b, 0, s, __VA_ARGS__);                   \
    }                                                                                    \
  } while (0)

hipError_t launch_dots_step(int dtype, int j, const LzArgs& a, int64_t nb, hipStream_t s) {
  if (a.window > 0 && a.window != 2) return hipErrorInvalidValue;
  const int wc = window_count(a, j);
  const int P = a.window > 0 ? 2 : wc <= 8 ? 8 : wc <= 16 ? 16 : (wc <= 32 ? 32 : 64);
  const dim3 g((unsigned)nb), b(dots_threads(P, dtype == EBTC_F64 ? 8 : 4));
  if (dtype == EBTC_F64) EBTC_GS_LAUNCH(k_dots_step, double, a, j);
  else EBTC_GS_LAUNCH(k_dots_step, float, a, j);
  return hipGetLastError();
}

hipError_t launch_dots_again(int dtype, int j, const LzArgs& a, int64_t nb, hipStream_t s) {
  const dim3 g((unsigned)nb), b(kBlock);
  if (dtype == EBTC_F64) EBTC_GS_LAUNCH(k_dots_again, double, a, j);
  else EBTC_GS_LAUNCH(k_dots_again, float, a, j);
  return hipGetLastError();
}

hipError_t launch_update(int dtype, int j, bool from_w, bool final_pass, bool second_pass, const LzArgs& a,
                         int64_t nb, hipStream_t s) {
  const dim3 g((unsigned)nb), b(kBlock);
  const int fw = from_w ? 1 : 0, fp = final_pass ? 1 : 0, sp = second_pass ? 1 : 0;
  if (dtype == EBTC_F64) EBTC_GS_LAUNCH(k_update, double, a, j, fw, fp, sp);
  else EBTC_GS_LAUNCH(k_update, float, a, j, fw, fp, sp);
  return hipGetLastError();
}

hipError_t launch_dots_update_1(int dtype, int j, const LzArgs& a, int64_t nb, hipStream_t s) {
  if (a.window != 0) return hipErrorInvalidValue;
  const int wc = window_count(a, j);
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
