// Adjoint of the summed scores: the gradient of L = <g, S~> with respect to every stored CSR entry.
//
// With the log-scale Sigma held fixed, dL/dA_k = e^{-Sigma} G_k,  G = int_0^1 e^{sA} g 1^T e^{(1-s)A} ds
// (the Frechet derivative of exp(A) 1 contracted with g, for the total communicability of eq. (4)
// summed as in eq. (5)). Both exponential actions are replaced by their Krylov approximations,
//   e^{sA} g ~ ||g|| W e^{sS} e1      (adjoint Lanczos started at g: basis W, tridiagonal S)
//   e^{tA} 1 ~ beta0 V e^{tT} e1      (the forward Lanczos: basis V, tridiagonal T)
// so G ~ ||g|| beta0 W X V^T with X = int_0^1 e^{sS} e1 e1^T e^{(1-s)T} ds, the upper-right block of
// exp([[S, e1 e1^T], [0, T]]) (Van Loan 1978). With a common shift theta >= both largest Ritz
// values, X_theta = e^{-theta} X is bounded, and
//   grad(i, j) = e^{theta - Sigma} ||g|| beta0 (W X_theta V^T)_ij.
// Kernels here: the start from the cotangent, the FP64 block exponential (one workgroup per
// realization), the node-major Z = c W X and V^T, and the SDDMM over the CSR pattern.
#include "device_common.h"

namespace ebtc {
namespace {

// Raw start vector Vraw_0 = g (the realization's graph block of the cotangent) and per-block partial
// squared norms; state initialised as in the forward start.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_start_vec(LzArgs a, const GraphInfo* graphs, const T* g) {
  __shared__ double red[kWaves];
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  const T* gs = g + graphs[tk.graph].score_off;
  T* v0 = (T*)a.V + tk.vec_off;
  double s = 0.0;
  for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) {
    const T x = gs[r];
    v0[r] = x;
    s += (double)x * (double)x;
  }
  s = block_sum<kBlock>(s, red);
  if (threadIdx.x == 0) a.npart[tk.part_off / kPartStride + ref.blk] = s;
  if (ref.blk == 0 && threadIdx.x == 0) {
    RState* st = a.state + ref.task;
    st->theta = 0.0;
    st->est = 0.0;
    st->m_used = 0;
    st->flags = 0;
    st->done = 0;
  }
}

// beta0 = ||g|| (canonical order) and s_0 = 1/beta0; a zero cotangent ends the realization at once.
__global__ __launch_bounds__(64) void k_start_norm(LzArgs a) {
  __shared__ double chunks[kMaxChunks];
  const Task tk = a.tasks[blockIdx.x];
  RState* st = a.state + blockIdx.x;
  const double ss = canonical_sum(a.npart + tk.part_off / kPartStride, tk.nblk, 1, chunks);
  if (threadIdx.x == 0) {
    const double b0 = sqrt(ss);
    st->beta0 = b0;
    if (b0 > 0.0 && isfinite(b0)) {
      st->s[0] = 1.0 / b0;
    } else {
      st->s[0] = 0.0;
      st->done = 1;
      st->m_used = 0;
      if (!isfinite(b0)) st->flags |= EBTC_FLAG_NONFINITE;
    }
  }
}

constexpr int kMX = 40;  // largest Krylov dimension of the adjoint block exponential (LDS resident)
static_assert(kMX <= kXLd, "adjoint output block");

// C (k1 x k2) = P (k1 x kk) * Q (kk x k2), row-major with leading dimension kMX, all in LDS.
__device__ inline void mm(double* C, const double* P, const double* Q, int k1, int kk, int k2) {
  for (int e = threadIdx.x; e < k1 * k2; e += blockDim.x) {
    const int i = e / k2, j = e - i * k2;
    double s = 0.0;
    for (int t = 0; t < kk; ++t) s += P[i * kMX + t] * Q[t * kMX + j];
    C[i * kMX + j] = s;
  }
}

// C = Tri * P / div (+ I when add_identity): Tri tridiagonal (diagonal d, off-diagonal o, size k).
__device__ inline void tri_mm(double* C, const double* d, const double* o, const double* P, int k, int cols,
                              double div, bool add_identity) {
  for (int e = threadIdx.x; e < k * cols; e += blockDim.x) {
    const int i = e / cols, j = e - i * cols;
    double s = d[i] * P[i * kMX + j];
    if (i > 0) s += o[i - 1] * P[(i - 1) * kMX + j];
    if (i + 1 < k) s += o[i] * P[(i + 1) * kMX + j];
    s /= div;
    if (add_identity && i == j) s += 1.0;
    C[i * kMX + j] = s;
  }
}

// Per realization: X' = c * diag(s'_a) X_theta with X_theta the upper-right block of
// exp([[S - theta I, e1 e1^T], [0, T - theta I]] ), c = e^{theta - Sigma_g} ||g|| beta0.
// Horner evaluation of the degree-16 Taylor polynomial of the scaled matrix (norm <= 1/2), where the
// tridiagonal factors make every Horner product O(k^2), then repeated squaring of the block-triangular
// result. Output row-major k2 x k1 in xout (leading dimension kXLd).
__global__ __launch_bounds__(kBlock) void k_block_exp(const RState* fwd, const RState* adj, const Task* tasks,
                                                      const double* log_scale, double* xout) {
  __shared__ double PA[kMX * kMX], PF[kMX * kMX], PB[kMX * kMX], TA[kMX * kMX], TF[kMX * kMX], TB[kMX * kMX];
  __shared__ double dA[kMX], oA[kMX], dB[kMX], oB[kMX];
  __shared__ double scal_s[1];
  const int r = blockIdx.x;
  const RState* f = fwd + r;
  const RState* q = adj + r;
  double* X = xout + (size_t)r * kXLd * kXLd;
  const int k1 = f->m_used, k2 = q->m_used;
  const int tid = threadIdx.x;
  if (k2 < 1 || q->beta0 == 0.0 || k1 < 1) {
    for (int e = tid; e < kXLd * kXLd; e += kBlock) X[e] = 0.0;
    return;
  }
  const double theta = fmax(f->theta, q->theta);
  if (tid < k2) {
    dA[tid] = q->alpha[tid] - theta;
    oA[tid] = tid + 1 < k2 ? q->beta[tid] : 0.0;
  }
  if (tid < k1) {
    dB[tid] = f->alpha[tid] - theta;
    oB[tid] = tid + 1 < k1 ? f->beta[tid] : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double rho = 0.0;
    for (int i = 0; i < k2; ++i) rho = fmax(rho, fabs(dA[i]) + (i ? fabs(oA[i - 1]) : 0.0) + fabs(oA[i]));
    for (int i = 0; i < k1; ++i) rho = fmax(rho, fabs(dB[i]) + (i ? fabs(oB[i - 1]) : 0.0) + fabs(oB[i]));
    rho += 1.0;  // the coupling block e1 e1^T
    int s = 0;
    while (rho > 0.5 && s < 60) {
      rho *= 0.5;
      ++s;
    }
    scal_s[0] = (double)s;
  }
  __syncthreads();
  const int sq = (int)scal_s[0];
  const double sc = ldexp(1.0, -sq);
  if (tid < k2) {
    dA[tid] *= sc;
    oA[tid] *= sc;
  }
  if (tid < k1) {
    dB[tid] *= sc;
    oB[tid] *= sc;
  }
  // Horner: P <- I + (M/k) P for k = 16..1, starting from P = I; block form
  //   PA <- I + A PA / k,  PF <- (A PF + E PB) / k,  PB <- I + B PB / k,  E = e1 e1^T (scaled by sc)
  for (int e = tid; e < kMX * kMX; e += kBlock) {
    const int i = e / kMX, j = e - i * kMX;
    PA[e] = (i == j) ? 1.0 : 0.0;
    PB[e] = (i == j) ? 1.0 : 0.0;
    PF[e] = 0.0;
  }
  __syncthreads();
  for (int k = 16; k >= 1; --k) {
    tri_mm(TA, dA, oA, PA, k2, k2, (double)k, true);
    tri_mm(TF, dA, oA, PF, k2, k1, 1.0, false);
    tri_mm(TB, dB, oB, PB, k1, k1, (double)k, true);
    __syncthreads();
    for (int e = tid; e < k2 * k1; e += kBlock) {
      const int i = e / k1, j = e - i * k1;
      double v = TF[i * kMX + j];
      if (i == 0) v += sc * PB[j];  // E PB: row 0 of PB
      PF[i * kMX + j] = v / (double)k;
    }
    for (int e = tid; e < kMX * kMX; e += kBlock) {
      PA[e] = TA[e];
      PB[e] = TB[e];
    }
    __syncthreads();
  }
  // squaring: [[PA, PF], [0, PB]]^2 = [[PA^2, PA PF + PF PB], [0, PB^2]]
  for (int t = 0; t < sq; ++t) {
    mm(TA, PA, PA, k2, k2, k2);
    mm(TF, PA, PF, k2, k2, k1);
    mm(TB, PB, PB, k1, k1, k1);
    __syncthreads();
    mm(PA, PF, PB, k2, k1, k1);  // PA (free) <- PF PB
    __syncthreads();
    for (int e = tid; e < kMX * kMX; e += kBlock) {
      PF[e] = TF[e] + PA[e];
      PA[e] = TA[e];
      PB[e] = TB[e];
    }
    __syncthreads();
  }
  const int g = tasks[r].graph;
  const double c = exp(theta - log_scale[g]) * q->beta0 * f->beta0;
  for (int e = tid; e < kXLd * kXLd; e += kBlock) {
    const int i = e / kXLd, j = e - i * kXLd;
    X[e] = (i < k2 && j < k1) ? c * q->s[i] * PF[i * kMX + j] : 0.0;
  }
}

// Node-major Z[i][b] = sum_a Wraw_a[i] X'[a][b] and Vn[i][b] = s_b Vraw_b[i] (b < k1), stride LD.
// One thread per row and all LD columns at once, so the adjoint basis is read once (eight of its
// elements in flight per thread); each sum still runs over a = 0..k2-1 in order from 0. Outputs leave
// as 16-byte stores (LD is a multiple of 8 and every realization's part starts at a multiple of LD
// elements).
template <typename T, int LD>
__global__ __launch_bounds__(kBlock) void k_build_zv(LzArgs fwd, LzArgs adj, const double* xall, T* Z, T* Vn) {
  static_assert(LD % 8 == 0 && LD <= kMX, "column chunks of eight");
  __shared__ double X[LD * LD];
  __shared__ double sb[LD];
  const Ref ref = resolve(fwd);
  const Task tk = fwd.tasks[ref.task];
  const RState* f = fwd.state + ref.task;
  const RState* q = adj.state + ref.task;
  const int k1 = f->m_used, k2 = min(q->m_used, LD);
  const double* xr = xall + (size_t)ref.task * kXLd * kXLd;
  for (int e = threadIdx.x; e < LD * LD; e += kBlock) X[e] = xr[(e / LD) * kXLd + e % LD];
  if ((int)threadIdx.x < LD) sb[threadIdx.x] = (int)threadIdx.x < k1 ? f->s[threadIdx.x] : 0.0;
  __syncthreads();
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  const T* Vr = (const T*)fwd.V + tk.vec_off;
  const T* Wr = (const T*)adj.V + tk.vec_off;
  T* Zr = Z + tk.w_off * (int64_t)LD;
  T* Vnr = Vn + tk.w_off * (int64_t)LD;
  using V4 = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
  constexpr int PER = 16 / sizeof(T);  // elements per 16-byte store
  for (int i = r0 + (int)threadIdx.x; i < r1; i += kBlock) {
    double acc[LD];
#pragma unroll
    for (int c = 0; c < LD; ++c) acc[c] = 0.0;
    for (int a0 = 0; a0 < k2; a0 += 8) {
      T wv[8];  // eight loads issued before the first use (a guarded load would be waited on at once)
#pragma unroll
      for (int u = 0; u < 8; ++u) wv[u] = Wr[(size_t)min(a0 + u, k2 - 1) * n + i];  // past k2: unused
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (a0 + u < k2) {
          const double wa = (double)wv[u];
#pragma unroll
          for (int c = 0; c < LD; ++c) acc[c] += wa * X[(a0 + u) * LD + c];
        }
      }
    }
#pragma unroll
    for (int b0 = 0; b0 < LD; b0 += PER) {
      T zo[PER], vo[PER];
#pragma unroll
      for (int c = 0; c < PER; ++c) vo[c] = Vr[(size_t)max(min(b0 + c, k1 - 1), 0) * n + i];  // past k1: unused
#pragma unroll
      for (int c = 0; c < PER; ++c) {
        const int b = b0 + c;
        zo[c] = (T)acc[b];
        vo[c] = b < k1 ? (T)(sb[b] * (double)vo[c]) : (T)0;
      }
      *(V4*)(Zr + (size_t)i * LD + b0) = *(const V4*)zo;
      *(V4*)(Vnr + (size_t)i * LD + b0) = *(const V4*)vo;
    }
  }
}

// grad[k] = <Z[i, :], Vn[col_k, :]> for every stored entry (i, col_k) of the realization; lane groups
// of 4 per row, the row's Z kept in registers, one contiguous LD-element gather per entry.
template <typename T, int LD>
__global__ __launch_bounds__(kBlock) void k_sddmm(LzArgs fwd, const T* Z, const T* Vn, T* grad) {
  constexpr int L = 4;
  const Ref ref = resolve(fwd);
  const Task tk = fwd.tasks[ref.task];
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  const int32_t* rp = fwd.row_ptr + tk.rowptr_off;
  const int32_t* ci = fwd.col_idx + tk.nnz_off;
  const T* Zr = Z + tk.w_off * (int64_t)LD;
  const T* Vnr = Vn + tk.w_off * (int64_t)LD;
  T* gr = grad + tk.nnz_off;
  const int grp = threadIdx.x / L, lane = threadIdx.x % L;
  for (int i = r0 + grp; i < r1; i += kBlock / L) {
    T z[LD];
#pragma unroll
    for (int b = 0; b < LD; ++b) z[b] = Zr[(size_t)i * LD + b];
    const int e = rp[i + 1];
    // two of the lane's entries per round (k and k + L), both gathers in flight together
    for (int k = rp[i] + lane; k < e; k += 2 * L) {
      const int k1 = k + L < e ? k + L : k;  // the round's second entry (or k again)
      const T* v0 = Vnr + (size_t)ci[k] * LD;
      const T* v1 = Vnr + (size_t)ci[k1] * LD;
      T x0[LD], x1[LD];
#pragma unroll
      for (int b = 0; b < LD; ++b) {
        x0[b] = v0[b];
        x1[b] = v1[b];
      }
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int b = 0; b < LD; ++b) {
        s0 += (double)z[b] * (double)x0[b];
        s1 += (double)z[b] * (double)x1[b];
      }
      gr[k] = (T)s0;
      if (k1 != k) gr[k1] = (T)s1;
    }
  }
}

template <typename T>
hipError_t build_zv_ld(int ld, const LzArgs& fwd, const LzArgs& adj, const double* x, void* Z, void* Vn, int64_t nb,
                       hipStream_t s) {
  const dim3 g((unsigned)nb), b(kBlock);
  switch (ld) {
    case 8: hipLaunchKernelGGL((k_build_zv<T, 8>), g, b, 0, s, fwd, adj, x, (T*)Z, (T*)Vn); break;
    case 16: hipLaunchKernelGGL((k_build_zv<T, 16>), g, b, 0, s, fwd, adj, x, (T*)Z, (T*)Vn); break;
    case 24: hipLaunchKernelGGL((k_build_zv<T, 24>), g, b, 0, s, fwd, adj, x, (T*)Z, (T*)Vn); break;
    case 32: hipLaunchKernelGGL((k_build_zv<T, 32>), g, b, 0, s, fwd, adj, x, (T*)Z, (T*)Vn); break;
    case 40: hipLaunchKernelGGL((k_build_zv<T, 40>), g, b, 0, s, fwd, adj, x, (T*)Z, (T*)Vn); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t sddmm_ld(int ld, const LzArgs& fwd, const void* Z, const void* Vn, void* grad, int64_t nb, hipStream_t s) {
  const dim3 g((unsigned)nb), b(kBlock);
  switch (ld) {
    case 8: hipLaunchKernelGGL((k_sddmm<T, 8>), g, b, 0, s, fwd, (const T*)Z, (const T*)Vn, (T*)grad); break;
    case 16: hipLaunchKernelGGL((k_sddmm<T, 16>), g, b, 0, s, fwd, (const T*)Z, (const T*)Vn, (T*)grad); break;
    case 24: hipLaunchKernelGGL((k_sddmm<T, 24>), g, b, 0, s, fwd, (const T*)Z, (const T*)Vn, (T*)grad); break;
    case 32: hipLaunchKernelGGL((k_sddmm<T, 32>), g, b, 0, s, fwd, (const T*)Z, (const T*)Vn, (T*)grad); break;
    case 40: hipLaunchKernelGGL((k_sddmm<T, 40>), g, b, 0, s, fwd, (const T*)Z, (const T*)Vn, (T*)grad); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The forward recomputation against the forward call's checkpoint, bit for bit: alpha_0..k-1,
// beta_0..k-1, theta*, beta0, the step count k and the flags of each realization (one thread each).
// Every realization that differs adds one to *mismatch, which k_zero_count clears first.
__global__ void k_zero_count(int32_t* count) { *count = 0; }

__global__ __launch_bounds__(kBlock) void k_ckpt_check(const RState* st, const double* ckpt, int64_t R,
                                                       int32_t* mismatch) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= R) return;
  const RState& s = st[r];
  const double* c = ckpt + r * kCkptDoubles;
  auto same = [](double a, double b) { return __double_as_longlong(a) == __double_as_longlong(b); };
  const int k = s.m_used;
  bool ok = (double)k == c[2 * kMLimit + 2] && (double)s.flags == c[2 * kMLimit + 3] && same(s.theta, c[2 * kMLimit]) &&
            same(s.beta0, c[2 * kMLimit + 1]) && k >= 0 && k <= kMLimit;
  for (int i = 0; ok && i < k; ++i) ok = same(s.alpha[i], c[i]) && same(s.beta[i], c[kMLimit + i]);
  if (!ok) atomicAdd(mismatch, 1);
}

}  // namespace

int adjoint_max_m() { return kMX; }

hipError_t launch_ckpt_check(const RState* st, const double* ckpt, int64_t R, int32_t* mismatch, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, mismatch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || R < 1) return e;
  hipLaunchKernelGGL(k_ckpt_check, dim3((unsigned)((R + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, st, ckpt, R,
                     mismatch);
  return hipGetLastError();
}

hipError_t launch_start_vec(int dtype, const LzArgs& a, const GraphInfo* graphs, const void* g, int64_t nb,
                            hipStream_t s) {
  if (dtype == EBTC_F64)
    hipLaunchKernelGGL(k_start_vec<double>, dim3((unsigned)nb), dim3(kBlock), 0, s, a, graphs, (const double*)g);
  else
    hipLaunchKernelGGL(k_start_vec<float>, dim3((unsigned)nb), dim3(kBlock), 0, s, a, graphs, (const float*)g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_start_norm(const LzArgs& a, int64_t R, hipStream_t s) {
  hipLaunchKernelGGL(k_start_norm, dim3((unsigned)R), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_block_exp(const RState* fwd, const RState* adj, const Task* tasks, const double* log_scale,
                            double* xout, int64_t R, hipStream_t s) {
  hipLaunchKernelGGL(k_block_exp, dim3((unsigned)R), dim3(kBlock), 0, s, fwd, adj, tasks, log_scale, xout);
  return hipGetLastError();
}

hipError_t launch_build_zv(int dtype, const LzArgs& fwd, const LzArgs& adj, const double* x, void* Z, void* Vn,
                           int ld, int64_t nb, hipStream_t s) {
  return dtype == EBTC_F64 ? build_zv_ld<double>(ld, fwd, adj, x, Z, Vn, nb, s)
                           : build_zv_ld<float>(ld, fwd, adj, x, Z, Vn, nb, s);
}

hipError_t launch_sddmm(int dtype, int ld, const LzArgs& fwd, const void* Z, const void* Vn, void* grad, int64_t nb,
                        hipStream_t s) {
  return dtype == EBTC_F64 ? sddmm_ld<double>(ld, fwd, Z, Vn, grad, nb, s)
                           : sddmm_ld<float>(ld, fwd, Z, Vn, grad, nb, s);
}

}  // namespace ebtc
