// CSR SpMV kernels of the Lanczos step, w = s_j A v_j (the Krylov approximation's product, eq. (4)).
//
// Two forms, chosen per batch on the host:
//   direct  (k_spmv_step)   gathers v_j[col] from HBM / L2. 256 threads, the workgroup's row_ptr
//                           slice staged in LDS, L lanes per row, two rows per lane group in flight
//                           and four entries per lane loaded before any is used. Rows with more than
//                           `hub` entries are reduced by the whole workgroup.
//   staged  (k_spmv_staged) the random gathers are what limits the direct form (each divergent
//                           4-byte gather costs an L1 miss); here v_j streams through LDS in column
//                           segments that fill the 160 KB of a gfx950 workgroup, and the gathers
//                           become LDS reads. Every lane first loads its rows' entries (U per row,
//                           L = 4 lanes per row, Q rows per lane group) into registers -- 2QU
//                           independent loads in flight per lane -- then, for each segment, adds
//                           the products of its entries whose column falls in the segment. Entries
//                           beyond L*U per row are gathered directly, by the lane group for short
//                           overflows and by the whole workgroup for hub rows.
// Both write w for their kRowsPerBlock rows with coalesced stores; the dot products run in a
// separate streaming kernel.
#include "device_common.h"

namespace ebtc {
namespace {

// Opens phase A of step j: closes step j-1 from its norm partials (all workgroups of the
// realization compute the same bits; workgroup 0 records them). Returns false when the
// realization is finished; *sj = 1/beta_{j-1} (or s_0 at j = 0).
__device__ inline bool open_step(const LzArgs& a, const Task& tk, RState* st, int blk, int j, double* chunks,
                                 double* sj) {
  if (st->done) return false;
  if (j == 0) {
    *sj = st->s[0];
    return true;
  }
  const StepClose c = close_step(st, a.npart + tk.part_off / kPartStride, tk.nblk, j - 1, a.eps, chunks);
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

// ------------------------------------------------------------------------------- direct gathers
template <typename T, bool HAS_VAL, int L>
__device__ inline void spmv_direct_block(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                         const T* __restrict__ va, const T* __restrict__ x, int r0, int rows, int hub,
                                         double scale, int* rp_lds, T* w_lds, short* hubs, int* hub_count,
                                         double* red) {
  constexpr int U = 4;
  const int tid = threadIdx.x;
  if (tid == 0) *hub_count = 0;
  for (int i = tid; i <= rows; i += kBlock) rp_lds[i] = rp[r0 + i];
  __syncthreads();
  constexpr int G = kBlock / L;
  const int grp = tid / L, lane = tid % L;
  for (int r = grp; r < rows; r += 2 * G) {
    const int rb = r + G;
    int b0 = rp_lds[r], e0 = rp_lds[r + 1];
    int b1 = rb < rows ? rp_lds[rb] : 0, e1 = rb < rows ? rp_lds[rb + 1] : 0;
    const bool h0 = e0 - b0 > hub, h1 = e1 - b1 > hub;
    if (lane == 0) {
      if (h0) hubs[atomicAdd(hub_count, 1)] = (short)r;
      if (h1) hubs[atomicAdd(hub_count, 1)] = (short)rb;
    }
    if (h0) e0 = b0;
    if (h1) e1 = b1;
    T acc0 = 0, acc1 = 0;
    for (int k0 = b0 + lane, k1 = b1 + lane; k0 < e0 || k1 < e1; k0 += U * L, k1 += U * L) {
      int c0[U], c1[U];
      T v0[U], v1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int ka = k0 + u * L, kb = k1 + u * L;
        c0[u] = ka < e0 ? ci[ka] : -1;
        c1[u] = kb < e1 ? ci[kb] : -1;
        if constexpr (HAS_VAL) {
          v0[u] = ka < e0 ? va[ka] : (T)0;
          v1[u] = kb < e1 ? va[kb] : (T)0;
        }
      }
      T x0[U], x1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        x0[u] = c0[u] >= 0 ? x[c0[u]] : (T)0;
        x1[u] = c1[u] >= 0 ? x[c1[u]] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (HAS_VAL) {
          acc0 += v0[u] * x0[u];
          acc1 += v1[u] * x1[u];
        } else {
          acc0 += x0[u];
          acc1 += x1[u];
        }
      }
    }
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) {
      acc0 += __shfl_xor(acc0, o, 64);
      acc1 += __shfl_xor(acc1, o, 64);
    }
    if (lane == 0) {
      if (!h0) w_lds[r] = (T)((double)acc0 * scale);
      if (rb < rows && !h1) w_lds[rb] = (T)((double)acc1 * scale);
    }
  }
  __syncthreads();
  const int nh = *hub_count;
  for (int h = 0; h < nh; ++h) {
    const int r = hubs[h];
    const int b = rp_lds[r], e = rp_lds[r + 1];
    T acc = 0;
    for (int k = b + tid; k < e; k += kBlock) {
      const T xv = x[ci[k]];
      if constexpr (HAS_VAL) acc += va[k] * xv; else acc += xv;
    }
    const double tot = block_sum<kBlock>((double)acc, red);
    if (tid == 0) w_lds[r] = (T)(tot * scale);
  }
  __syncthreads();
}

template <typename T, bool HAS_VAL, int L>
__global__ __launch_bounds__(kBlock) void k_spmv_step(LzArgs a, int j) {
  __shared__ int rp_lds[kRowsPerBlock + 1];
  __shared__ T w_lds[kRowsPerBlock];
  __shared__ short hubs[kRowsPerBlock];
  __shared__ int hub_count;
  __shared__ double chunks[kMaxChunks];
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  RState* st = a.state + ref.task;
  double sj;
  if (!open_step(a, tk, st, ref.blk, j, chunks, &sj)) return;
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, rows = min(n - r0, kRowsPerBlock);
  const T* va = HAS_VAL ? (const T*)a.values + tk.nnz_off : nullptr;
  spmv_direct_block<T, HAS_VAL, L>(a.row_ptr + tk.rowptr_off, a.col_idx + tk.nnz_off, va,
                                   (const T*)a.V + tk.vec_off + (size_t)j * n, r0, rows, a.hub_threshold, sj, rp_lds,
                                   w_lds, hubs, &hub_count, chunks);
  T* W = (T*)a.W + tk.w_off + r0;
  for (int i = threadIdx.x; i < rows; i += kBlock) W[i] = w_lds[i];
}

// ------------------------------------------------------------------------------- CSR stream
// k_spmv_stream: each workgroup (256 threads) owns kStreamRows rows, i.e. an eighth of a Lanczos
// row block. Its entries are one contiguous range of col_idx / values: the workgroup loads them with
// independent coalesced loads (kStreamU per thread in flight), gathers v_j[col], and writes the
// products to LDS; then thread t sums row t's products in order, in FP64 (deterministic, and
// accurate on rows of thousands of entries). A
// range longer than the LDS capacity is cut into row chunks; a single row beyond the capacity (a
// hub) is reduced by the whole workgroup. The whole row block costs two memory round trips per
// chunk instead of one per row per lane group.
constexpr int kStreamRows = 256;
constexpr int kStreamU = 8;
template <typename T>
struct StreamShape {
  static constexpr int CAP = sizeof(T) == 8 ? 3072 : 6144;  // product slots (24 KB)
};

template <typename T, bool HAS_VAL>
__device__ inline void spmv_stream_rows(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                        const T* __restrict__ va, const T* __restrict__ x, int r0, int rows,
                                        double scale, int* rp_lds, T* prod, T* w_out, double* red) {
  constexpr int CAP = StreamShape<T>::CAP, U = kStreamU;
  const int tid = threadIdx.x;
  for (int i = tid; i <= rows; i += kBlock) rp_lds[i] = rp[r0 + i];
  __syncthreads();
  int ra = 0;
  while (ra < rows) {
    const int nz0 = rp_lds[ra];
    if (rp_lds[ra + 1] - nz0 > CAP) {  // hub row: whole workgroup, direct gathers
      const int e = rp_lds[ra + 1];
      T acc = 0;
      for (int k = nz0 + tid; k < e; k += kBlock) {
        const T xv = x[ci[k]];
        if constexpr (HAS_VAL) acc += va[k] * xv; else acc += xv;
      }
      const double tot = block_sum<kBlock>((double)acc, red);
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
    for (int k0 = tid; k0 < cnt; k0 += kBlock * U) {
      int c[U];
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * kBlock;
        c[u] = k < cnt ? ci[nz0 + k] : -1;
        if constexpr (HAS_VAL) v[u] = k < cnt ? va[nz0 + k] : (T)0;
      }
      T xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = c[u] >= 0 ? x[c[u]] : (T)0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * kBlock;
        if (k < cnt) {
          if constexpr (HAS_VAL) prod[k] = v[u] * xv[u]; else prod[k] = xv[u];
        }
      }
    }
    __syncthreads();
    for (int r = ra + tid; r < rb; r += kBlock) {
      double acc = 0.0;  // FP64: sequential sums over long (BA hub) rows stay accurate
      const int e = rp_lds[r + 1] - nz0;
      for (int k = rp_lds[r] - nz0; k < e; ++k) acc += (double)prod[k];
      w_out[r] = (T)(acc * scale);
    }
    __syncthreads();
    ra = rb;
  }
}

// Workgroup w of the launch handles rows [q * kStreamRows, (q+1) * kStreamRows) of Lanczos row block
// w / 8 (q = w % 8); the realization of that block comes from the usual workgroup map.
template <typename T, bool HAS_VAL>
__global__ __launch_bounds__(kBlock) void k_spmv_stream(LzArgs a, int j) {
  constexpr int SUB = kRowsPerBlock / kStreamRows;
  __shared__ int rp_lds[kStreamRows + 1];
  __shared__ T prod[StreamShape<T>::CAP];
  __shared__ double chunks[kMaxChunks];
  const int lb = logical_block();
  const int blk_flat = lb / SUB, q = lb - blk_flat * SUB;
  Ref ref;
  if (a.blkmap == nullptr) {
    ref.task = a.single_task;
    ref.blk = blk_flat;
  } else {
    ref.task = a.blkmap[blk_flat];
    ref.blk = blk_flat - a.tasks[ref.task].blk_begin;
  }
  const Task tk = a.tasks[ref.task];
  RState* st = a.state + ref.task;
  double sj;
  // only the first sub-block of block 0 records the closed step (all compute it)
  if (!open_step(a, tk, st, q == 0 ? ref.blk : 1, j, chunks, &sj)) return;
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock + q * kStreamRows;
  if (r0 >= n) return;
  const int rows = min(n - r0, kStreamRows);
  const T* va = HAS_VAL ? (const T*)a.values + tk.nnz_off : nullptr;
  spmv_stream_rows<T, HAS_VAL>(a.row_ptr + tk.rowptr_off, a.col_idx + tk.nnz_off, va,
                               (const T*)a.V + tk.vec_off + (size_t)j * n, r0, rows, sj, rp_lds, prod,
                               (T*)a.W + tk.w_off + r0, chunks);
}

template <typename T, bool HAS_VAL>
__global__ __launch_bounds__(kBlock) void k_spmv_stream_1(int32_t n, const int32_t* rp, const int32_t* ci,
                                                          const T* va, const T* x, T* y) {
  __shared__ int rp_lds[kStreamRows + 1];
  __shared__ T prod[StreamShape<T>::CAP];
  __shared__ double red[kWaves];
  const int r0 = logical_block() * kStreamRows;
  if (r0 >= n) return;
  spmv_stream_rows<T, HAS_VAL>(rp, ci, va, x, r0, min(n - r0, kStreamRows), 1.0, rp_lds, prod, y + r0, red);
}

// ------------------------------------------------------------------------------- LDS-staged gathers
constexpr int kSL = 4;  // lanes per row
// Register budget at 1024 threads is 128 VGPRs without spills: FP32 keeps 3 rows x 6 entries per
// lane (4 rows for pattern-only graphs, whose values need no registers), 24 entries per row; FP64
// keeps 2 rows x 8 entries (32 per row).
template <typename T, bool HAS_VAL>
struct StagedShape {
  static constexpr int Q = sizeof(T) == 8 ? 2 : (HAS_VAL ? 3 : 4);  // rows per lane group at once
  static constexpr int U = sizeof(T) == 8 ? 8 : 6;           // entries per lane per row in registers
  static constexpr int G = kStagedThreads / kSL;              // lane groups
  static constexpr int HROWS = Q * G;                         // rows per register pass
  static constexpr int HUB = 4 * kSL * U;                     // above: whole-workgroup tail
};

template <typename T, bool HAS_VAL>
__device__ inline void spmv_staged_block(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                         const T* __restrict__ va, const T* __restrict__ x, int n, int seglen, int r0,
                                         int rows, double scale, T* xs, int* rp_lds, T* w_lds, short* hubs,
                                         int* hub_count, double* red) {
  using S = StagedShape<T, HAS_VAL>;
  constexpr int Q = S::Q, U = S::U, L = kSL, G = S::G, NT = kStagedThreads;
  const int tid = threadIdx.x, grp = tid / L, lane = tid % L;
  if (tid == 0) *hub_count = 0;
  for (int i = tid; i <= rows; i += NT) rp_lds[i] = rp[r0 + i];
  __syncthreads();
  for (int h0 = 0; h0 < rows; h0 += S::HROWS) {
    int c[Q][U];
    T v[Q][U];
    T acc[Q];
    int bq[Q], eq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int r = h0 + grp + q * G;
      bq[q] = r < rows ? rp_lds[r] : 0;
      eq[q] = r < rows ? rp_lds[r + 1] : 0;
      acc[q] = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = bq[q] + lane + u * L;
        c[q][u] = k < eq[q] ? ci[k] : -1;
        if constexpr (HAS_VAL) v[q][u] = k < eq[q] ? va[k] : (T)0;
      }
    }
    for (int base = 0; base < n; base += seglen) {
      const int len = min(seglen, n - base);
      __syncthreads();  // the previous segment is no longer read
      for (int i0 = tid; i0 < len; i0 += 8 * NT) {
        T t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = i0 + u * NT < len ? x[base + i0 + u * NT] : (T)0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (i0 + u * NT < len) xs[i0 + u * NT] = t[u];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const unsigned off = (unsigned)(c[q][u] - base);
          if (off < (unsigned)len) {
            const T xv = xs[off];
            if constexpr (HAS_VAL) acc[q] += v[q][u] * xv; else acc[q] += xv;
          }
        }
      }
    }
    // entries beyond L*U: the lane group gathers directly (short overflow), hubs go to the workgroup
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int r = h0 + grp + q * G;
      const int deg = eq[q] - bq[q];
      if (deg > S::HUB) {
        if (lane == 0) hubs[atomicAdd(hub_count, 1)] = (short)r;
      } else {
        for (int k = bq[q] + L * U + lane; k < eq[q]; k += L) {
          const T xv = x[ci[k]];
          if constexpr (HAS_VAL) acc[q] += va[k] * xv; else acc[q] += xv;
        }
      }
#pragma unroll
      for (int o = L / 2; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
      if (lane == 0 && r < rows) w_lds[r] = acc[q];
    }
  }
  __syncthreads();
  const int nh = *hub_count;
  for (int h = 0; h < nh; ++h) {
    const int r = hubs[h];
    const int b = rp_lds[r] + L * U, e = rp_lds[r + 1];
    T acc = 0;
    for (int k = b + tid; k < e; k += NT) {
      const T xv = x[ci[k]];
      if constexpr (HAS_VAL) acc += va[k] * xv; else acc += xv;
    }
    const double tot = block_sum<NT>((double)acc, red);
    if (tid == 0) w_lds[r] += (T)tot;
    __syncthreads();
  }
  for (int r = tid; r < rows; r += NT) w_lds[r] = (T)((double)w_lds[r] * scale);
  __syncthreads();
}

template <typename T, bool HAS_VAL>
__global__ __launch_bounds__(kStagedThreads) void k_spmv_staged(LzArgs a, int j) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int rp_lds[kRowsPerBlock + 1];
  __shared__ T w_lds[kRowsPerBlock];
  __shared__ short hubs[kRowsPerBlock];
  __shared__ int hub_count;
  __shared__ double chunks[kMaxChunks];
  __shared__ double red[kStagedThreads / 64];
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  RState* st = a.state + ref.task;
  double sj;
  if (!open_step(a, tk, st, ref.blk, j, chunks, &sj)) return;
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, rows = min(n - r0, kRowsPerBlock);
  const T* va = HAS_VAL ? (const T*)a.values + tk.nnz_off : nullptr;
  spmv_staged_block<T, HAS_VAL>(a.row_ptr + tk.rowptr_off, a.col_idx + tk.nnz_off, va,
                                (const T*)a.V + tk.vec_off + (size_t)j * n, n, a.seglen, r0, rows, sj, (T*)smem,
                                rp_lds, w_lds, hubs, &hub_count, red);
  T* W = (T*)a.W + tk.w_off + r0;
  for (int i = threadIdx.x; i < rows; i += kStagedThreads) W[i] = w_lds[i];
}

// ------------------------------------------------------------------------------- standalone y = A x
template <typename T, bool HAS_VAL, int L>
__global__ __launch_bounds__(kBlock) void k_spmv_direct_1(int32_t n, const int32_t* rp, const int32_t* ci,
                                                          const T* va, const T* x, T* y, int hub) {
  __shared__ int rp_lds[kRowsPerBlock + 1];
  __shared__ T w_lds[kRowsPerBlock];
  __shared__ short hubs[kRowsPerBlock];
  __shared__ int hub_count;
  __shared__ double red[kWaves];
  const int r0 = logical_block() * kRowsPerBlock, rows = min(n - r0, kRowsPerBlock);
  spmv_direct_block<T, HAS_VAL, L>(rp, ci, va, x, r0, rows, hub, 1.0, rp_lds, w_lds, hubs, &hub_count, red);
  for (int i = threadIdx.x; i < rows; i += kBlock) y[r0 + i] = w_lds[i];
}

template <typename T, bool HAS_VAL>
__global__ __launch_bounds__(kStagedThreads) void k_spmv_staged_1(int32_t n, const int32_t* rp, const int32_t* ci,
                                                                  const T* va, const T* x, T* y, int seglen) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int rp_lds[kRowsPerBlock + 1];
  __shared__ T w_lds[kRowsPerBlock];
  __shared__ short hubs[kRowsPerBlock];
  __shared__ int hub_count;
  __shared__ double red[kStagedThreads / 64];
  const int r0 = logical_block() * kRowsPerBlock, rows = min(n - r0, kRowsPerBlock);
  spmv_staged_block<T, HAS_VAL>(rp, ci, va, x, n, seglen, r0, rows, 1.0, (T*)smem, rp_lds, w_lds, hubs, &hub_count,
                                red);
  for (int i = threadIdx.x; i < rows; i += kStagedThreads) y[r0 + i] = w_lds[i];
}

// Static LDS of the staged kernels: row_ptr slice, w, hub list, counters and reduction scratch.
template <typename T>
constexpr size_t staged_static_bytes() {
  return (size_t)(kRowsPerBlock + 1) * 4 + (size_t)kRowsPerBlock * (sizeof(T) + 2) + 1024;
}

template <typename K>
hipError_t allow_lds(K kernel, size_t dyn) {
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
}

template <typename T>
hipError_t prepare_t() {
  const size_t dyn = kLdsBytes - staged_static_bytes<T>();
  hipError_t e = allow_lds(k_spmv_staged<T, true>, dyn);
  if (e == hipSuccess) e = allow_lds(k_spmv_staged<T, false>, dyn);
  if (e == hipSuccess) e = allow_lds(k_spmv_staged_1<T, true>, dyn);
  if (e == hipSuccess) e = allow_lds(k_spmv_staged_1<T, false>, dyn);
  return e;
}

template <typename T, bool HAS_VAL>
hipError_t step_direct(int lanes, int j, const LzArgs& a, int64_t nb, hipStream_t s) {
  const dim3 g((unsigned)nb), b(kBlock);
  switch (lanes) {
    case 4: hipLaunchKernelGGL((k_spmv_step<T, HAS_VAL, 4>), g, b, 0, s, a, j); break;
    case 8: hipLaunchKernelGGL((k_spmv_step<T, HAS_VAL, 8>), g, b, 0, s, a, j); break;
    case 16: hipLaunchKernelGGL((k_spmv_step<T, HAS_VAL, 16>), g, b, 0, s, a, j); break;
    case 32: hipLaunchKernelGGL((k_spmv_step<T, HAS_VAL, 32>), g, b, 0, s, a, j); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, bool HAS_VAL>
hipError_t step_any(int lanes, int j, const LzArgs& a, int64_t nb, hipStream_t s) {
  if (a.seglen > 0) {
    hipLaunchKernelGGL((k_spmv_staged<T, HAS_VAL>), dim3((unsigned)nb), dim3(kStagedThreads),
                       (size_t)a.seglen * sizeof(T), s, a, j);
    return hipGetLastError();
  }
  if (lanes == 0) {
    hipLaunchKernelGGL((k_spmv_stream<T, HAS_VAL>), dim3((unsigned)(nb * (kRowsPerBlock / kStreamRows))),
                       dim3(kBlock), 0, s, a, j);
    return hipGetLastError();
  }
  return step_direct<T, HAS_VAL>(lanes, j, a, nb, s);
}

template <typename T, bool HAS_VAL>
hipError_t one_any(int lanes, int hub, int seglen, int32_t n, const int32_t* rp, const int32_t* ci, const void* va,
                   const void* x, void* y, hipStream_t s) {
  const int nb = (n + kRowsPerBlock - 1) / kRowsPerBlock;
  if (seglen > 0) {
    hipLaunchKernelGGL((k_spmv_staged_1<T, HAS_VAL>), dim3(nb), dim3(kStagedThreads), (size_t)seglen * sizeof(T), s, n,
                       rp, ci, (const T*)va, (const T*)x, (T*)y, seglen);
    return hipGetLastError();
  }
  if (lanes == 0) {
    hipLaunchKernelGGL((k_spmv_stream_1<T, HAS_VAL>), dim3((n + kStreamRows - 1) / kStreamRows), dim3(kBlock), 0, s, n,
                       rp, ci, (const T*)va, (const T*)x, (T*)y);
    return hipGetLastError();
  }
  const dim3 g(nb), b(kBlock);
  switch (lanes) {
    case 4: hipLaunchKernelGGL((k_spmv_direct_1<T, HAS_VAL, 4>), g, b, 0, s, n, rp, ci, (const T*)va, (const T*)x, (T*)y, hub); break;
    case 8: hipLaunchKernelGGL((k_spmv_direct_1<T, HAS_VAL, 8>), g, b, 0, s, n, rp, ci, (const T*)va, (const T*)x, (T*)y, hub); break;
    case 16: hipLaunchKernelGGL((k_spmv_direct_1<T, HAS_VAL, 16>), g, b, 0, s, n, rp, ci, (const T*)va, (const T*)x, (T*)y, hub); break;
    case 32: hipLaunchKernelGGL((k_spmv_direct_1<T, HAS_VAL, 32>), g, b, 0, s, n, rp, ci, (const T*)va, (const T*)x, (T*)y, hub); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t prepare_staged_kernels() {
  static hipError_t e = [] {
    hipError_t r = prepare_t<float>();
    if (r == hipSuccess) r = prepare_t<double>();
    return r;
  }();
  return e;
}

int staged_max_seglen(int dtype) {
  return dtype == EBTC_F64 ? (int)((kLdsBytes - staged_static_bytes<double>()) / 8)
                           : (int)((kLdsBytes - staged_static_bytes<float>()) / 4);
}

hipError_t launch_spmv_step(int dtype, bool has_val, int lanes, int j, const LzArgs& a, int64_t nb, hipStream_t s) {
  if (dtype == EBTC_F64)
    return has_val ? step_any<double, true>(lanes, j, a, nb, s) : step_any<double, false>(lanes, j, a, nb, s);
  return has_val ? step_any<float, true>(lanes, j, a, nb, s) : step_any<float, false>(lanes, j, a, nb, s);
}

hipError_t launch_spmv(int dtype, bool has_val, int lanes, int hub, int seglen, int32_t n, const int32_t* rp,
                       const int32_t* ci, const void* va, const void* x, void* y, hipStream_t s) {
  if (dtype == EBTC_F64)
    return has_val ? one_any<double, true>(lanes, hub, seglen, n, rp, ci, va, x, y, s)
                   : one_any<double, false>(lanes, hub, seglen, n, rp, ci, va, x, y, s);
  return has_val ? one_any<float, true>(lanes, hub, seglen, n, rp, ci, va, x, y, s)
                 : one_any<float, false>(lanes, hub, seglen, n, rp, ci, va, x, y, s);
}

}  // namespace ebtc
