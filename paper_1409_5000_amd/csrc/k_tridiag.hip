// The small exponential of the Krylov approximation, FP64, one wave (64 lanes) per realization.
//
// After m Lanczos steps exp(A) 1 ~ beta0 V_m exp(T_m) e1 (eq. (4) through the Krylov method). With
// theta* the largest eigenvalue of T_m this is computed as e^{theta*} * beta0 V_m y with
//   y = exp(T_m - theta* I) e1,
// so no intermediate overflows (every eigenvalue of T_m - theta* I is <= 0).
//   theta*  -- Sturm-sequence multisection: each lane counts the eigenvalues below its own probe
//              point (LDL^T pivots of T - x I); the bracket of lambda_max shrinks 64-fold per round.
//   y       -- Chebyshev expansion of exp on an interval holding the spectrum of T - theta* I
//              (Gershgorin bounds), coefficients e^-d I_k(d) by Miller's backward recurrence,
//              evaluated by Clenshaw's recurrence in the same backward loop: about sqrt(84 d) + 30
//              tridiagonal products for a spectrum of half-width d (a Taylor series scaled to unit
//              norm needs 20 per unit of width). Lane l owns rows l and l + 64; the tridiagonal
//              product takes its neighbours' entries with wave shuffles.
//   est     -- Saad's a-posteriori estimate beta_{m-1} |y_{m-1}| / ||y||_2 (relative).
#include "step_device.h"

namespace ebtc {
namespace {


// mode 0: final; mode 1: adaptive check after step j (tridiag_prepare). One wave per realization.
__global__ __launch_bounds__(64) void k_tridiag_state(LzArgs args, int64_t first, int mode, int j, int m_steps,
                                                      int shift, double tol, ebtc_diag* diag, double* ckpt) {
  if (mode == 1 && all_stopped(args, j)) return;
  __shared__ double a[kMLimit];
  __shared__ double b[kMLimit];
  __shared__ double chunks[kMaxChunks];
  const int64_t r = first + blockIdx.x;
  const Task tk = args.tasks[r];
  RState* st = args.state + r;
  const TriPrep p = tridiag_prepare(args, st, args.npart + tk.part_off / kPartStride, tk.nblk, r, mode, j, m_steps,
                                    diag, chunks);
  if (p.exit) return;
  tridiag_load(st, p, a, b);
  __syncthreads();
  tridiag_finish(args, st, r, mode, j, p, a, b, shift, tol, diag, ckpt);
}

__global__ __launch_bounds__(64) void k_tridiag_arrays(int32_t k, const double* alpha, const double* beta,
                                                       double* y, double* theta, int32_t shift) {
  __shared__ double a[kMLimit];
  __shared__ double b[kMLimit];
  const int64_t c = blockIdx.x;
  const int lane = threadIdx.x;
  for (int i = lane; i < k; i += 64) {
    a[i] = alpha[c * k + i];
    b[i] = beta[c * k + i];
  }
  __syncthreads();
  const ExpvOut o = tridiag_expv_wave(a, b, k, shift != 0);
  if (lane < k) y[c * k + lane] = o.y0;
  if (lane + 64 < k) y[c * k + lane + 64] = o.y1;
  if (lane == 0) theta[c] = o.theta;
}

}  // namespace

hipError_t launch_tridiag_state(const LzArgs& a, int64_t first, int64_t count, int mode, int j, int m_steps,
                                int shift, double tol, ebtc_diag* diag, double* ckpt, hipStream_t s) {
  hipLaunchKernelGGL(k_tridiag_state, dim3((unsigned)count), dim3(64), 0, s, a, first, mode, j, m_steps, shift, tol,
                     diag, ckpt);
  return hipGetLastError();
}

hipError_t launch_tridiag_arrays(int32_t count, int32_t k, const double* alpha, const double* beta, double* y,
                                 double* theta, int32_t shift, hipStream_t s) {
  hipLaunchKernelGGL(k_tridiag_arrays, dim3((unsigned)count), dim3(64), 0, s, k, alpha, beta, y, theta, shift);
  return hipGetLastError();
}

}  // namespace ebtc
