// Device steps of the Lanczos process shared by the per-phase kernels (one launch per phase over
// every realization) and the single-kernel solve (one workgroup runs a realization's whole process):
// both call these functions, so they compute the same bits.
#pragma once

#include "device_common.h"

namespace ebtc {
namespace {

// ------------------------------------------------------------------------------- phase A: SpMV
// Opens phase A of step j: closes step j-1 from its norm partials (all workgroups of the
// realization compute the same bits; workgroup 0 records them). Returns false when the
// realization is finished; *sj = 1/beta_{j-1} (or s_0 at j = 0).
__device__ inline bool open_step(const LzArgs& a, const Task& tk, RState* st, int blk, int j, double* chunks,
                                 double* sj, const double* npart = nullptr) {
  if (step_skipped(a, st, j)) return false;
  if (j == 0) {
    *sj = st->s[0];
    return true;
  }
  const StepClose c = close_step(st, npart ? npart : a.npart + tk.part_off / kPartStride, tk.nblk, j - 1, a.eps, chunks);
  if (blk == 0 && threadIdx.x == 0) {
    st->beta[j - 1] = c.beta;
    if (c.flags) {
      st->flags |= c.flags;
      st->done = 1;
      st->m_used = j;
    } else {
      st->s[j] = 1.0 / c.beta;
    }
  }
  if (c.flags) return false;
  *sj = 1.0 / c.beta;
  return true;
}

constexpr int kStreamRows = 256;
constexpr int kStreamU = 8;
template <typename T>
struct StreamShape {
  static constexpr int CAP = sizeof(T) == 8 ? 3072 : 6144;  // product slots (24 KB)
};

// SEQ_HUB: a row beyond the capacity is summed by one thread in entry order instead (the first
// product's arithmetic, for a caller that must reproduce it).
// RP_LDS: rp_lds already holds the rows' pointers (rp unused). NT_LOADS: the entries are read with the
// non-temporal policy (they live in HBM and are read once per product); off when they sit in LDS.
// HUB_NT: a row beyond the capacity is reduced in the order of a workgroup of HUB_NT threads (the
// first HUB_NT threads form the per-thread sums; the other waves add exact zeros).
template <typename T, bool HAS_VAL, int NT = kBlock, int CAP = StreamShape<T>::CAP, bool SEQ_HUB = false,
          bool RP_LDS = false, bool NT_LOADS = true, int HUB_NT = NT>
__device__ inline void spmv_stream_rows(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                        const T* __restrict__ va, const T* __restrict__ x, int r0, int rows,
                                        double scale, int* rp_lds, T* prod, T* w_out, double* red) {
  constexpr int U = kStreamU;
  const int tid = threadIdx.x;
  if constexpr (!RP_LDS) {
    for (int i = tid; i <= rows; i += NT) rp_lds[i] = rp[r0 + i];
    __syncthreads();
  }
  int ra = 0;
  while (ra < rows) {
    const int nz0 = rp_lds[ra];
    if (SEQ_HUB && rp_lds[ra + 1] - nz0 > CAP) {
      if (tid == 0) {
        double acc = 0.0;
        for (int k = nz0; k < rp_lds[ra + 1]; ++k) {
          const T xv = x[ci[k]];
          if constexpr (HAS_VAL) acc += (double)(va[k] * xv); else acc += (double)xv;
        }
        w_out[ra] = (T)(acc * scale);
      }
      ++ra;
      continue;
    }
    if (rp_lds[ra + 1] - nz0 > CAP) {  // hub row: whole workgroup, direct gathers
      static_assert(HUB_NT <= NT && HUB_NT % 64 == 0, "hub reduction layout");
      const int e = rp_lds[ra + 1];
      T acc = 0;
      if (tid < HUB_NT)
        for (int k = nz0 + tid; k < e; k += HUB_NT) {
          const T xv = x[ci[k]];
          if constexpr (HAS_VAL) acc += va[k] * xv; else acc += xv;
        }
      const double tot = block_sum<NT>((double)acc, red);
      if (tid == 0) w_out[ra] = (T)(tot * scale);
      ++ra;
      continue;
    }
    // largest rb with rp[rb] - rp[ra] <= CAP (every thread finds the same rb)
    int lo = ra + 1, hi = rows;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rp_lds[mid] - nz0 <= CAP) lo = mid; else hi = mid - 1;
    }
    const int rb = lo;
    const int cnt = rp_lds[rb] - nz0;
    for (int k0 = tid; k0 < cnt; k0 += NT * U) {
      int c[U];
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * NT;
        // the matrix is read once per product: non-temporal loads leave the cache lines of the
        // gathered vector resident
        if constexpr (NT_LOADS) {
          c[u] = k < cnt ? __builtin_nontemporal_load(ci + nz0 + k) : -1;
          if constexpr (HAS_VAL) v[u] = k < cnt ? __builtin_nontemporal_load(va + nz0 + k) : (T)0;
        } else {
          c[u] = k < cnt ? ci[nz0 + k] : -1;
          if constexpr (HAS_VAL) v[u] = k < cnt ? va[nz0 + k] : (T)0;
        }
      }
      T xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = c[u] >= 0 ? x[c[u]] : (T)0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * NT;
        if (k < cnt) {
          if constexpr (HAS_VAL) prod[k] = v[u] * xv[u]; else prod[k] = xv[u];
        }
      }
    }
    __syncthreads();
    for (int r = ra + tid; r < rb; r += NT) {
      double acc = 0.0;  // FP64: sequential sums over long (BA hub) rows stay accurate
      const int e = rp_lds[r + 1] - nz0;
      for (int k = rp_lds[r] - nz0; k < e; ++k) acc += (double)prod[k];
      w_out[r] = (T)(acc * scale);
    }
    __syncthreads();
    ra = rb;
  }
}

// ------------------------------------------------------------------------------- phase B: Gram-Schmidt
// Partial dots p_d = sum_rows Vraw_{lo+d}[r] * w[r] (d < cnt = j - lo + 1 <= P) of this workgroup's
// rows, reduced over the workgroup and stored to part_blk[d]. NT fixes the arithmetic: thread t of NT
// sums rows r0 + t, r0 + t + NT, ... and the per-thread sums are reduced wave by wave, then wave by
// wave in order. The workgroup runs it with NREAL threads (NT a multiple of NREAL), each taking the
// NT / NREAL threads t = tid, tid + NREAL, ... in turn, so a smaller workgroup computes the same
// bits. Basis loads are issued min(P, 8) vectors at a time (clamped to the last one, whose extra
// contributions are masked) so that many loads are in flight per thread. RING > 0: vector i lives in
// slot i % RING (the ring of the memory-bounded form). red: (NT / 64) * P doubles of LDS.
template <typename T, int P, int NT, int RING, int NREAL = NT>
__device__ inline void block_dots(const T* __restrict__ Vr, int n, int lo, int j, int r0, int r1,
                                  const T* wsrc_lds, const T* wsrc_glob, T* wstore, double* part_blk, double* red) {
  static_assert(P == 2 || P == 8 || P == 16 || P == 32 || P == 64, "lane layout of ReduceScatter");
  static_assert(NT % NREAL == 0 && NREAL % 64 == 0, "virtual thread layout");
  constexpr int RPT = kRowsPerBlock / NT;
  constexpr int CH = P < 8 ? P : 8;
  const int tid = threadIdx.x, cnt = j - lo + 1;
  // one pass of NREAL threads, forming the sums of threads t0 + tid of NT
  auto pass = [&](int t0) {
    const int vt = t0 + tid;  // the thread of NT whose sums this pass forms
    constexpr int LP0 = 64 / P;
    if (NREAL < NT && t0 >= r1 - r0) {  // no rows in this pass: its partials are zeros
      if ((tid & 63) % LP0 == 0) red[(vt >> 6) * P + (tid & 63) / LP0] = 0.0;
      return;
    }
    T p[P];
#pragma unroll
    for (int i = 0; i < P; ++i) p[i] = 0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = r0 + q * NT + vt;
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
    const int lane = tid & 63, wave = vt >> 6;
    ReduceScatter<P, 32>::run(pd, lane);
    constexpr int LP = 64 / P;  // lanes per value after the reduce-scatter: lane l holds value l / LP
    if (lane % LP == 0) red[wave * P + lane / LP] = pd[0];
  };
  if constexpr (NREAL == NT) {
    pass(0);  // straight-line code for the usual case: a loop, even of one trip, costs the scheduling
  } else {
#pragma unroll 1
    for (int t0 = 0; t0 < NT; t0 += NREAL) pass(t0);
  }
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

// Phase B of step j: every workgroup reduces the dot partials of all workgroups of its realization
// in the canonical order (identical coefficients everywhere, no inter-workgroup synchronisation),
// then v~_{j+1} = src - sum_i c_i Vraw_i over the window (FP64 accumulation, rounded once), plus
// the partial squared norm on the final pass.
// Where one realization's step data lives: its workspace blocks, or LDS in the single-kernel solve.
template <typename T>
struct StepMem {
  RState* st;    // Lanczos state
  T* V;          // raw basis, vector-major (n elements per vector)
  double* part;  // dot partials, kPartStride per row block
  double* npart; // norm partials, one per row block
};

template <typename T>
__device__ inline StepMem<T> step_mem(const LzArgs& a, const Task& tk, int task) {
  return {a.state + task, (T*)a.V + tk.vec_off, a.part + tk.part_off, a.npart + tk.part_off / kPartStride};
}

// wsrc (nullable): where the product w of this step is read instead of the W arena (the single-kernel
// solve keeps it in LDS); xcopy (nullable): also receives v~_{j+1}[r - r0], the next step's gather
// source in LDS. The arithmetic of a row is the same for every P >= the window.
template <typename T, int P, int RING>
__device__ inline void update_body(const LzArgs& a, const Task& tk, const StepMem<T>& mem, int blk, int j, int from_w,
                                   int final_pass, int second, double* cs, double (*csum)[kMaxChunks], double* red,
                                   const T* wsrc = nullptr, T* xcopy = nullptr) {
  RState* st = mem.st;
  constexpr int CH = P < 8 ? P : 8;
  const int tid = threadIdx.x, lo = window_lo(a, j), cnt = j - lo + 1;
  const double* part = mem.part;
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
      if (lo + tid == j && blk == 0) {
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
  const int n = tk.n, r0 = blk * kRowsPerBlock, r1 = min(n, r0 + kRowsPerBlock);
  T* Vr = mem.V;
  const T* src = from_w ? (wsrc ? wsrc - r0 : (const T*)a.W + tk.w_off) : Vr + vslot(a, j + 1) * n;
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
      if (xcopy) xcopy[r - r0] = out;
      nrm += (double)out * (double)out;
    }
  }
  if (!final_pass) return;
  nrm = block_sum<kBlock>(nrm, red);
  if (tid == 0) mem.npart[blk] = nrm;
}

// ------------------------------------------------------------------------------- small exponential
constexpr int kChebMax = 1 << 16;  // Chebyshev terms of the small exponential (d up to 5e7)

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
  double y0, y1;  // this lane's components: rows lane and lane + 64 (0 beyond k)
  double ynorm;   // ||y||_2
  bool finite;
};

// a, b: LDS arrays (k diagonal, k-1 off-diagonal entries), k <= 128. Called by all 64 lanes of a
// wave; lane l owns rows l and l + 64 of T.
__device__ ExpvOut tridiag_expv_wave(const double* a, const double* b, int k, bool shift) {
  const int lane = threadIdx.x & 63;
  const int q0 = lane, q1 = lane + 64;
  const double ai0_0 = q0 < k ? a[q0] : 0.0, ai0_1 = q1 < k ? a[q1] : 0.0;
  const double bl_0 = (q0 >= 1 && q0 < k) ? b[q0 - 1] : 0.0, bl_1 = q1 < k ? b[q1 - 1] : 0.0;
  const double br_0 = (q0 + 1 < k) ? b[q0] : 0.0, br_1 = (q1 + 1 < k) ? b[q1] : 0.0;
  double theta = 0.0;
  if (shift) {
    if (k == 1) {
      theta = a[0];
    } else {
      const double rad0 = fabs(bl_0) + fabs(br_0), rad1 = fabs(bl_1) + fabs(br_1);
      double lo = wave_min(fmin(q0 < k ? ai0_0 - rad0 : INFINITY, q1 < k ? ai0_1 - rad1 : INFINITY));
      double hi = wave_max(fmax(q0 < k ? ai0_0 + rad0 : -INFINITY, q1 < k ? ai0_1 + rad1 : -INFINITY));
      const double bmax = wave_max(fmax(fabs(br_0), fabs(br_1)));
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
  // y = exp(M) e1, M = T - theta I, by the Chebyshev expansion of exp on [bot, top], an interval that
  // holds the spectrum of M (Gershgorin; top = 0 when theta = lambda_max): with x = c + d t,
  //   exp(x) = e^top (i_0 + 2 sum_{k>=1} i_k T_k(t)),  i_k = e^-d I_k(d)  (I_k modified Bessel),
  // and i_k falls like e^{-k^2 / 2d}, so sqrt(84 d) + 20 terms reach double precision. The i_k come
  // from Miller's backward recurrence I_{k-1} = I_{k+1} + (2k/d) I_k, unnormalised and in the order
  // Clenshaw's recurrence b_k = c_k e1 + 2 t b_{k+1} - b_{k+2} consumes them, so one backward loop does
  // both and the sum divides by the normalisation sum_k c_k T_k(1) = 1 at the end.
  const double ai_0 = q0 < k ? ai0_0 - theta : 0.0, ai_1 = q1 < k ? ai0_1 - theta : 0.0;
  const double lo = wave_min(fmin(q0 < k ? ai_0 - fabs(bl_0) - fabs(br_0) : INFINITY,
                                  q1 < k ? ai_1 - fabs(bl_1) - fabs(br_1) : INFINITY));
  const double hi = wave_max(fmax(q0 < k ? ai_0 + fabs(bl_0) + fabs(br_0) : -INFINITY,
                                  q1 < k ? ai_1 + fabs(bl_1) + fabs(br_1) : -INFINITY));
  const double top = shift ? 0.0 : hi;
  const double bot = fmin(lo, top);
  const double c = 0.5 * (bot + top), d = 0.5 * (top - bot);
  // t = (M - c I) / d, row by row (rows beyond k stay zero: no coupling, no diagonal)
  const double sc = d > 1e-10 ? 1.0 / d : 1.0;
  const double ta_0 = q0 < k ? (ai_0 - c) * sc : 0.0, ta_1 = q1 < k ? (ai_1 - c) * sc : 0.0;
  const double tl_0 = bl_0 * sc, tl_1 = bl_1 * sc, tr_0 = br_0 * sc, tr_1 = br_1 * sc;
  // (t v) for the two rows of this lane; rows 63 and 64 are neighbours across the lane's two halves
  auto tmul = [&](double v0, double v1, double& o0, double& o1) {
    const double up0 = __shfl_up(v0, 1, 64);
    const double dn0r = __shfl_down(v0, 1, 64);
    const double row64 = __shfl(v1, 0, 64);
    const double up1r = __shfl_up(v1, 1, 64);
    const double row63 = __shfl(v0, 63, 64);
    const double dn1 = __shfl_down(v1, 1, 64);
    const double dn0 = lane == 63 ? row64 : dn0r;
    const double up1 = lane == 0 ? row63 : up1r;
    o0 = ta_0 * v0 + tl_0 * up0 + tr_0 * dn0;
    o1 = ta_1 * v1 + tl_1 * up1 + tr_1 * dn1;
  };
  const double e = exp(top);
  double x0, x1;
  if (!(d > 1e-10)) {  // M within 1e-10 of c I: second-order Taylor (error below d^3 / 6)
    const double u0 = lane == 0 ? 1.0 : 0.0;
    double p0, p1, r0, r1;
    tmul(u0, 0.0, p0, p1);
    tmul(p0, p1, r0, r1);
    const double ec = exp(c);
    x0 = ec * (u0 + p0 + 0.5 * r0);
    x1 = ec * (p1 + 0.5 * r1);
  } else {
    const int K = min((int)ceil(sqrt(84.0 * d)) + 20, kChebMax);
    double m1 = 0.0, m0 = 1e-200, S = 0.0;
    double b1_0 = 0.0, b1_1 = 0.0, b2_0 = 0.0, b2_1 = 0.0;  // b_{k+1}, b_{k+2}
    for (int kk = K + 10; kk >= 0; --kk) {
      const double ck = kk == 0 ? m0 : 2.0 * m0;
      S += ck;
      double t0, t1;
      tmul(b1_0, b1_1, t0, t1);
      const double n0 = (lane == 0 ? ck : 0.0) + 2.0 * t0 - b2_0;
      const double n1 = 2.0 * t1 - b2_1;
      b2_0 = b1_0;
      b2_1 = b1_1;
      b1_0 = n0;
      b1_1 = n1;
      if (kk > 0) {
        const double mn = m1 + (2.0 * kk * sc) * m0;
        m1 = m0;
        m0 = mn;
        if (m0 > 1e200) {  // keep the unnormalised recurrence in range
          m0 *= 1e-200;
          m1 *= 1e-200;
          S *= 1e-200;
          b1_0 *= 1e-200;
          b1_1 *= 1e-200;
          b2_0 *= 1e-200;
          b2_1 *= 1e-200;
        }
      }
    }
    double t0, t1;
    tmul(b2_0, b2_1, t0, t1);  // f = b_0 - t b_1
    x0 = e * (b1_0 - t0) / S;
    x1 = e * (b1_1 - t1) / S;
  }
  x0 = q0 < k ? x0 : 0.0;
  x1 = q1 < k ? x1 : 0.0;
  ExpvOut o;
  o.theta = theta;
  o.y0 = x0;
  o.y1 = x1;
  o.ynorm = sqrt(wave_sum(x0 * x0 + x1 * x1));
  o.finite = isfinite(o.ynorm) && isfinite(theta);
  return o;
}

// The small exponential of one realization after its last step (mode 0) or after step j of an
// adaptive run (mode 1), in three parts so that a workgroup of any size can run it:
//   tridiag_prepare  every thread of the workgroup (close_step reduces with all of them): the order k
//                    of T, the last beta and the flags. mode 1 closes step j and stops the
//                    realization on breakdown; mode 0 closes the last step of a realization still
//                    open after m_steps (fixed m). exit: nothing more to do here (thread 0 has
//                    recorded any stop);
//   tridiag_load     the lanes of the first wave copy T to LDS (then a workgroup barrier);
//   tridiag_finish   the first wave: theta*, y = exp(T - theta* I) e1, Saad's estimate. mode 1 stops
//                    the realization when the estimate is below tol or k reached m_max (CAPPED); a
//                    realization that goes on is closed again, with the same bits, by the next phase
//                    A. mode 0 records y, theta, the estimate, diag and the checkpoint when given.
struct TriPrep {
  int k;
  double beta_last;
  int flags;
  bool exit;
};

__device__ inline TriPrep tridiag_prepare(const LzArgs& args, RState* st, const double* npart, int nblk, int64_t r,
                                          int mode, int j, int m_steps, ebtc_diag* diag, double* chunks) {
  TriPrep p{0, 0.0, st->flags, false};
  if (mode == 1) {
    if (st->done) {
      p.exit = true;
      return p;
    }
    p.k = j + 1;
    const StepClose c = close_step(st, npart, nblk, j, args.eps, chunks);
    p.beta_last = c.beta;
    if (c.flags) {
      if (threadIdx.x == 0) {
        st->beta[j] = c.beta;
        st->flags = p.flags | c.flags;
        st->done = 1;
        st->m_used = p.k;
      }
      p.exit = true;
    }
    return p;
  }
  if (st->done && st->m_used < 1) {
    // nothing to expand (an adjoint started at a zero cotangent): empty result
    if (threadIdx.x == 0) {
      st->theta = 0.0;
      st->est = 0.0;
      if (diag) {
        diag[r].m_used = 0;
        diag[r].flags = st->flags;
        diag[r].theta = 0.0;
        diag[r].est = 0.0;
      }
    }
    p.exit = true;
  } else if (st->done) {
    p.k = st->m_used;
    p.beta_last = st->beta[p.k - 1];
  } else {
    p.k = m_steps;
    const StepClose c = close_step(st, npart, nblk, p.k - 1, args.eps, chunks);
    p.beta_last = c.beta;
    p.flags |= c.flags;
  }
  return p;
}

__device__ inline void tridiag_load(const RState* st, const TriPrep& p, double* a, double* b) {
  for (int i = threadIdx.x; i < p.k; i += 64) {
    a[i] = st->alpha[i];
    b[i] = i < p.k - 1 ? st->beta[i] : p.beta_last;
  }
}

__device__ inline void tridiag_finish(const LzArgs& args, RState* st, int64_t r, int mode, int j, const TriPrep& p,
                                      const double* a, const double* b, int shift, double tol, ebtc_diag* diag,
                                      double* ckpt) {
  const int lane = threadIdx.x, k = p.k;
  const double beta_last = p.beta_last;
  int flags = p.flags;
  const ExpvOut o = tridiag_expv_wave(a, b, k, shift != 0);
  const double ylast = k <= 64 ? __shfl(o.y0, k - 1, 64) : __shfl(o.y1, k - 65, 64);
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
      } else if (args.live != nullptr) {
        // the count of realizations still running after step j (an integer, so its value does not
        // depend on the order of the adds); the next step's kernels read it after the launch boundary
        atomicAdd(&args.live[j], 1);
      }
    }
    return;
  }
  if (lane < k) st->y[lane] = o.y0;
  if (lane + 64 < k) st->y[lane + 64] = o.y1;
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
    for (int i = lane; i < kMLimit; i += 64) {
      c[i] = i < k ? a[i] : 0.0;
      c[kMLimit + i] = i < k ? b[i] : 0.0;
    }
    if (lane == 0) {
      c[2 * kMLimit] = o.theta;
      c[2 * kMLimit + 1] = st->beta0;
      c[2 * kMLimit + 2] = (double)k;
      c[2 * kMLimit + 3] = (double)flags;
    }
  }
}

}  // namespace
}  // namespace ebtc
