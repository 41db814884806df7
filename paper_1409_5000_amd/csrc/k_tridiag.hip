// The small exponential of the Krylov approximation, FP64, one wave (64 lanes) per realization.
//
// After m Lanczos steps exp(A) 1 ~ beta0 V_m exp(T_m) e1 (eq. (4) through the Krylov method). With
// theta* the largest eigenvalue of T_m this is computed as e^{theta*} * beta0 V_m y with
//   y = exp(T_m - theta* I) e1,
// so no intermediate overflows (every eigenvalue of T_m - theta* I is <= 0).
//   theta*  -- Sturm-sequence multisection: each lane counts the eigenvalues below its own probe
//              point (LDL^T pivots of T - x I); the bracket of lambda_max shrinks 64-fold per round.
//   y       -- truncated Taylor series of exp((T - theta* I)/s), applied s times, with
//              s = ceil(||T - theta* I||_inf) so every series has argument norm <= 1 and 20 terms
//              reach double precision (1/20! < 1e-18). Lane i owns row i; the tridiagonal product
//              takes its neighbours' entries with wave shuffles.
//   est     -- Saad's a-posteriori estimate beta_{m-1} |y_{m-1}| / ||y||_2 (relative).
#include "device_common.h"

namespace ebtc {
namespace {

constexpr int kTaylorTerms = 20;

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Number of eigenvalues of the tridiagonal (a, b) below x.
__device__ inline int sturm_count(const double* a, const double* b, int k, double x, double pivmin) {
  double d = a[0] - x;
  if (fabs(d) < pivmin) d = -pivmin;
  int cnt = d < 0.0;
  for (int i = 1; i < k; ++i) {
    d = (a[i] - x) - b[i - 1] * b[i - 1] / d;
    if (fabs(d) < pivmin) d = -pivmin;
    cnt += d < 0.0;
  }
  return cnt;
}

struct ExpvOut {
  double theta;
  double y;      // this lane's component (0 for lanes >= k)
  double ynorm;  // ||y||_2
  bool finite;
};

// a, b: LDS arrays (k diagonal, k-1 off-diagonal entries). Called by all 64 lanes of a wave.
__device__ ExpvOut tridiag_expv_wave(const double* a, const double* b, int k, bool shift) {
  const int lane = threadIdx.x & 63;
  const double ai0 = lane < k ? a[lane] : 0.0;
  const double bl = (lane >= 1 && lane < k) ? b[lane - 1] : 0.0;
  const double br = (lane + 1 < k) ? b[lane] : 0.0;
  double theta = 0.0;
  if (shift) {
    if (k == 1) {
      theta = a[0];
    } else {
      const double rad = fabs(bl) + fabs(br);
      double lo = wave_min(lane < k ? ai0 - rad : INFINITY);
      double hi = wave_max(lane < k ? ai0 + rad : -INFINITY);
      const double bmax = wave_max(fabs(br));
      const double pivmin = 1e-290 * fmax(1.0, bmax * bmax);
      const double eps = 1.1102230246251565e-16;
      hi += 4.0 * eps * fmax(fabs(hi), fabs(lo)) + pivmin;
      lo -= 4.0 * eps * fmax(fabs(hi), fabs(lo)) + pivmin;
      for (int it = 0; it < 40; ++it) {
        if (hi - lo <= 4.0 * eps * fmax(fabs(lo), fabs(hi)) + 2.0 * pivmin) break;
        const double w = hi - lo;
        const double x = (lane == 63) ? hi : lo + w * (double)(lane + 1) * (1.0 / 64.0);
        const int c = sturm_count(a, b, k, x, pivmin);
        const unsigned long long mask = __ballot(c == k);
        const int first = mask ? (__ffsll((long long)mask) - 1) : 63;
        const double nhi = (first == 63) ? hi : lo + w * (double)(first + 1) * (1.0 / 64.0);
        const double nlo = (first == 0) ? lo : lo + w * (double)first * (1.0 / 64.0);
        lo = nlo;
        hi = nhi;
      }
      theta = 0.5 * (lo + hi);
    }
  }
  const double ai = (lane < k) ? ai0 - theta : 0.0;
  const double rho = wave_max(fabs(ai) + fabs(bl) + fabs(br));
  const double sd = fmin(fmax(1.0, ceil(rho)), 1048576.0);
  const int steps = (int)sd;
  const double inv_s = 1.0 / sd;
  double x = (lane == 0) ? 1.0 : 0.0;
  for (int st = 0; st < steps; ++st) {
    double term = x, acc = x;
#pragma unroll
    for (int p = 1; p <= kTaylorTerms; ++p) {
      const double up = __shfl_up(term, 1, 64);
      const double dn = __shfl_down(term, 1, 64);
      term = (ai * term + bl * up + br * dn) * (inv_s / (double)p);
      acc += term;
    }
    x = (lane < k) ? acc : 0.0;
  }
  ExpvOut o;
  o.theta = theta;
  o.y = x;
  o.ynorm = sqrt(wave_sum(x * x));
  o.finite = isfinite(o.ynorm) && isfinite(theta);
  return o;
}

// mode 0: final. A realization still open after its last step (fixed m) is closed here (beta of the
//         last step, breakdown test); then y, theta and the estimate are stored, with diag and
//         checkpoint when given.
// mode 1: adaptive check after step j: closes step j, stops on breakdown, when the estimate drops
//         below tol, or at m_max (CAPPED). A realization that goes on is closed again, with the
//         same bits, by the next phase A.
__global__ __launch_bounds__(64) void k_tridiag_state(LzArgs args, int64_t first, int mode, int j, int m_steps,
                                                      int shift, double tol, ebtc_diag* diag, double* ckpt) {
  __shared__ double a[kMLimit];
  __shared__ double b[kMLimit];
  __shared__ double chunks[kMaxChunks];
  const int64_t r = first + blockIdx.x;
  RState* st = args.state + r;
  const Task tk = args.tasks[r];
  const double* npart = args.npart + tk.part_off / kPartStride;
  const int lane = threadIdx.x;
  int k;
  int flags = st->flags;
  double beta_last;
  if (mode == 1) {
    if (st->done) return;
    k = j + 1;
    const StepClose c = close_step(st, npart, tk.nblk, j, args.eps, chunks);
    beta_last = c.beta;
    if (c.flags) {
      if (lane == 0) {
        st->beta[j] = c.beta;
        st->flags = flags | c.flags;
        st->done = 1;
        st->m_used = k;
      }
      return;
    }
  } else if (st->done && st->m_used < 1) {
    // nothing to expand (an adjoint started at a zero cotangent): empty result
    if (lane == 0) {
      st->theta = 0.0;
      st->est = 0.0;
      if (diag) {
        diag[r].m_used = 0;
        diag[r].flags = st->flags;
        diag[r].theta = 0.0;
        diag[r].est = 0.0;
      }
    }
    return;
  } else if (st->done) {
    k = st->m_used;
    beta_last = st->beta[k - 1];
  } else {
    k = m_steps;
    const StepClose c = close_step(st, npart, tk.nblk, k - 1, args.eps, chunks);
    beta_last = c.beta;
    flags |= c.flags;
  }
  if (lane < k) {
    a[lane] = st->alpha[lane];
    b[lane] = lane < k - 1 ? st->beta[lane] : beta_last;
  }
  __syncthreads();
  const ExpvOut o = tridiag_expv_wave(a, b, k, shift != 0);
  const double ylast = __shfl(o.y, k - 1, 64);
  const double est = (o.ynorm > 0.0) ? beta_last * fabs(ylast) / o.ynorm : 0.0;
  if (mode == 1) {
    if (lane == 0) {
      int stop = 0;
      if (!o.finite) {
        flags |= EBTC_FLAG_NONFINITE;
        stop = 1;
      } else if (est < tol) {
        stop = 1;
      } else if (k >= args.m_max) {
        flags |= EBTC_FLAG_CAPPED;
        stop = 1;
      }
      if (stop) {
        st->beta[j] = beta_last;
        st->flags = flags;
        st->done = 1;
        st->m_used = k;
      }
    }
    return;
  }
  if (lane < k) st->y[lane] = o.y;
  if (lane == 0) {
    if (!o.finite) flags |= EBTC_FLAG_NONFINITE;
    const double e = (flags & EBTC_FLAG_BREAKDOWN) ? 0.0 : est;
    st->beta[k - 1] = beta_last;
    st->m_used = k;
    st->done = 1;
    st->flags = flags;
    st->theta = o.theta;
    st->est = e;
    if (diag) {
      diag[r].m_used = k;
      diag[r].flags = flags;
      diag[r].theta = o.theta;
      diag[r].est = e;
    }
  }
  if (ckpt) {
    double* c = ckpt + r * kCkptDoubles;
    c[lane] = lane < k ? a[lane] : 0.0;
    c[kMLimit + lane] = lane < k ? b[lane] : 0.0;
    if (lane == 0) {
      c[2 * kMLimit] = o.theta;
      c[2 * kMLimit + 1] = st->beta0;
      c[2 * kMLimit + 2] = (double)k;
      c[2 * kMLimit + 3] = (double)flags;
    }
  }
}

__global__ __launch_bounds__(64) void k_tridiag_arrays(int32_t k, const double* alpha, const double* beta,
                                                       double* y, double* theta, int32_t shift) {
  __shared__ double a[kMLimit];
  __shared__ double b[kMLimit];
  const int64_t c = blockIdx.x;
  const int lane = threadIdx.x;
  if (lane < k) {
    a[lane] = alpha[c * k + lane];
    b[lane] = beta[c * k + lane];
  }
  __syncthreads();
  const ExpvOut o = tridiag_expv_wave(a, b, k, shift != 0);
  if (lane < k) y[c * k + lane] = o.y;
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
