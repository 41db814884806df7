// Device helpers shared by the Lanczos and tridiagonal kernels.
#pragma once

#include "internal.h"

namespace ebtc {

constexpr int kWaves = kBlock / 64;

// Workgroups are dispatched round-robin over the eight XCDs (workgroup id mod 8). Map them so that
// each XCD walks a contiguous range of logical workgroups: the workgroups of one realization then
// share one XCD's L2, where the gathered vector v_j stays resident.
__device__ inline int logical_block() {
  const int G = gridDim.x, b = blockIdx.x;
  const int x = b & 7, q = b >> 3;
  const int base = G >> 3, rem = G & 7;
  return x * base + (x < rem ? x : rem) + q;
}

struct Ref {
  int task;
  int blk;
};

// True when a realization takes no part in step j: finished, or (second pass of the memory-bounded
// form) past the last step whose basis vector the combination needs.
__device__ inline bool step_skipped(const LzArgs& a, const RState* st, int j) {
  return st->done || (a.stop_mused && j + 1 >= st->m_used);
}

// True when every realization of the launch stopped at step j - 1's adaptive check: the launch's
// workgroups return before reading anything else (the captured sequence runs to the step cap).
__device__ inline bool all_stopped(const LzArgs& a, int j) {
  return a.live != nullptr && j > 0 && a.live[j - 1] == 0;
}

__device__ inline Ref resolve(const LzArgs& a) {
  const int lb = logical_block();
  if (a.blkmap == nullptr) return {a.single_task, lb};
  const int gb = a.sub_blocks ? a.sub_blocks[lb] : lb;
  const int t = a.blkmap[gb];
  return {t, gb - a.tasks[t].blk_begin};
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of one double over the workgroup of NT threads; every thread gets the result. red: NT/64 doubles.
template <int NT = kBlock>
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += red[i];
  return t;
}

// Butterfly reduce-scatter of P values per lane over the 64 lanes of a wave: after the call v[0]
// of lane l holds the wave-wide sum of value index (P == 64 ? l : l >> 1). Costs P - 1 (+1)
// shuffles instead of 6 P for P separate reductions.
template <int P, int M>
struct ReduceScatter {
  __device__ static inline void run(double* v, int lane) {
    if constexpr (P > 1) {
      constexpr int h = P / 2;
      const bool up = (lane & M) != 0;
#pragma unroll
      for (int k = 0; k < h; ++k) {
        const double keep = up ? v[k + h] : v[k];
        const double send = up ? v[k] : v[k + h];
        v[k] = keep + __shfl_xor(send, M, 64);
      }
    } else {
      v[0] += __shfl_xor(v[0], M, 64);
    }
    if constexpr (M > 1) ReduceScatter<(P > 1 ? P / 2 : 1), M / 2>::run(v, lane);
  }
};



// Chunking of per-workgroup partial sums: a realization with nblk workgroups sums its partials in
// chunks of kernel-independent size (left to right inside a chunk, then chunk sums left to right).
// Every kernel that needs the same total therefore gets the same bits, whatever its thread count.
__device__ inline int part_chunk(int nblk) { return (nblk + kMaxChunks - 1) / kMaxChunks; }

// Total of x[b * stride], b < count, in the canonical order. All threads of the block call it and
// all get the result. lds: >= kMaxChunks doubles of scratch.
__device__ inline double canonical_sum(const double* x, int count, int stride, double* lds) {
  const int chunk = part_chunk(count);
  const int nch = (count + chunk - 1) / chunk;
  for (int c = threadIdx.x; c < nch; c += blockDim.x) {
    double s = 0.0;
    const int b1 = min(count, (c + 1) * chunk);
    for (int b = c * chunk; b < b1; ++b) s += x[(size_t)b * stride];
    lds[c] = s;
  }
  __syncthreads();
  double t = 0.0;
  for (int c = 0; c < nch; ++c) t += lds[c];
  __syncthreads();
  return t;
}

struct StepClose {
  double beta;
  int flags;  // EBTC_FLAG_BREAKDOWN / EBTC_FLAG_NONFINITE when the realization stops here
};

// Closes Lanczos step j from its norm partials: beta_j = ||v~_{j+1}|| and the breakdown test
// beta_j <= 64 eps scal[j], scal[j] = max(|alpha_0..j|, beta_0..j-1) (recorded by the update kernel
// that finished alpha_j). Reads only values written by earlier kernels.
__device__ inline StepClose close_step(const RState* st, const double* norm_part, int nblk, int j, double eps,
                                       double* lds) {
  const double ss = canonical_sum(norm_part, nblk, 1, lds);
  StepClose c;
  c.beta = sqrt(ss);
  const double scale = st->scal[j];
  c.flags = 0;
  if (!isfinite(c.beta) || !isfinite(scale)) c.flags = EBTC_FLAG_NONFINITE;
  else if (!(c.beta > 64.0 * eps * scale)) c.flags = EBTC_FLAG_BREAKDOWN;
  return c;
}

}  // namespace ebtc
