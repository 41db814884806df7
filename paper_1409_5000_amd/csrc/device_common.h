// Device helpers shared by the Lanczos and tridiagonal kernels.
#pragma once

#include "internal.h"

namespace ebtc {

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
// beta_j <= 64 eps max(|alpha_0..j|, beta_0..j-1). Reads only values written by earlier kernels.
__device__ inline StepClose close_step(const RState* st, const double* norm_part, int nblk, int j, double eps,
                                       double* lds) {
  const double ss = canonical_sum(norm_part, nblk, 1, lds);
  StepClose c;
  c.beta = sqrt(ss);
  double scale = 0.0;
  for (int i = 0; i <= j; ++i) scale = fmax(scale, fabs(st->alpha[i]));
  for (int i = 0; i < j; ++i) scale = fmax(scale, st->beta[i]);
  c.flags = 0;
  if (!isfinite(c.beta) || !isfinite(st->alpha[j])) c.flags = EBTC_FLAG_NONFINITE;
  else if (!(c.beta > 64.0 * eps * scale)) c.flags = EBTC_FLAG_BREAKDOWN;
  return c;
}

}  // namespace ebtc
