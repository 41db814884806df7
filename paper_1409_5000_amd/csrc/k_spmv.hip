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
#include <algorithm>
#include <type_traits>

#include "step_device.h"

namespace ebtc {
namespace {


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
  if (all_stopped(a, j)) return;
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
                                   (const T*)a.V + tk.vec_off + vslot(a, j) * n, r0, rows, a.hub_threshold, sj, rp_lds,
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

// Workgroup w of the launch handles rows [q * kStreamRows, (q+1) * kStreamRows) of Lanczos row block
// w / 8 (q = w % 8); the realization of that block comes from the usual workgroup map.
template <typename T, bool HAS_VAL>
__global__ __launch_bounds__(kBlock) void k_spmv_stream(LzArgs a, int j) {
  if (all_stopped(a, j)) return;
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
    const int gb = a.sub_blocks ? a.sub_blocks[blk_flat] : blk_flat;
    ref.task = a.blkmap[gb];
    ref.blk = gb - a.tasks[ref.task].blk_begin;
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
                               (const T*)a.V + tk.vec_off + vslot(a, j) * n, r0, rows, sj, rp_lds, prod,
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

// ------------------------------------------------------------------------------- entry-balanced
// Power-law graphs keep most of their entries in a few rows, numbered first (a Barabasi-Albert
// graph of 1e6 nodes holds 22 times the mean in its first 2048 rows), so one row block's workgroup
// sets the time of a launch. Here each workgroup takes an equal share of a realization's entries:
// the rows whose first entry falls in its share of entries, whole (a row is never split, so its
// sum is the CSR-stream form's, bit for bit), walked 256 rows at a time by the stream arithmetic.

// Row bounds of every share, once per call: one workgroup per realization, one thread per share.
__global__ __launch_bounds__(kBlock) void k_bal_rows(LzArgs a, int t0) {
  const int t = t0 + blockIdx.x;
  const Task tk = a.tasks[t];
  const int32_t* rp = a.row_ptr + tk.rowptr_off;
  const int n = tk.n, base = rp[0];
  const int64_t p0 = a.bal_begin[t], np = a.bal_begin[t + 1] - p0;
  auto first_at_or_after = [&](int64_t e) {  // first row r with rp[r] >= base + e, in [0, n]
    int lo = 0, hi = n;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((int64_t)rp[mid] - base < e) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  for (int64_t q = threadIdx.x; q < np; q += kBlock) {
    BalPart bp;
    bp.task = t;
    bp.q = (int32_t)q;
    bp.r_begin = first_at_or_after(q * a.bal_entries);
    bp.r_end = q + 1 == np ? n : first_at_or_after((q + 1) * a.bal_entries);
    a.bal[p0 + q] = bp;
  }
}

// FIRST: the first product from the all-ones start, whose rows beyond the LDS capacity are summed in
// entry order as the row-sum kernel does (the other forms' first product), so that every step
// matches the CSR-stream form bit for bit.
template <typename T, bool HAS_VAL, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_spmv_bal(LzArgs a, int j) {
  if (all_stopped(a, j)) return;
  __shared__ int rp_lds[kStreamRows + 1];
  __shared__ T prod[StreamShape<T>::CAP];
  __shared__ double chunks[kMaxChunks];
  const int lb = logical_block();
  const BalPart bp = a.bal[a.blkmap != nullptr ? (int64_t)lb : a.bal_begin[a.single_task] + lb];
  const Task tk = a.tasks[bp.task];
  RState* st = a.state + bp.task;
  double sj;
  // only the first share of a realization records the closed step (all compute it)
  if (!open_step(a, tk, st, bp.q == 0 ? 0 : 1, j, chunks, &sj)) return;
  const int n = tk.n;
  const T* va = HAS_VAL ? (const T*)a.values + tk.nnz_off : nullptr;
  const T* x = (const T*)a.V + tk.vec_off + vslot(a, j) * n;
  T* W = (T*)a.W + tk.w_off;
  for (int r0 = bp.r_begin; r0 < bp.r_end; r0 += kStreamRows) {
    if (r0 > bp.r_begin) __syncthreads();  // the previous rows' LDS readers are done
    spmv_stream_rows<T, HAS_VAL, kBlock, StreamShape<T>::CAP, FIRST>(a.row_ptr + tk.rowptr_off, a.col_idx + tk.nnz_off,
                                                                    va, x, r0, min(bp.r_end - r0, kStreamRows), sj,
                                                                    rp_lds, prod, W + r0, chunks);
  }
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
  if (all_stopped(a, j)) return;
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
                                (const T*)a.V + tk.vec_off + vslot(a, j) * n, n, a.seglen, r0, rows, sj, (T*)smem,
                                rp_lds, w_lds, hubs, &hub_count, red);
  T* W = (T*)a.W + tk.w_off + r0;
  for (int i = threadIdx.x; i < rows; i += kStagedThreads) W[i] = w_lds[i];
}

// Step 0 of a process started at the all-ones vector: A v_0 = s_0 A 1, each row's sum of its values
// (its entry count for a pattern-only graph), summed in FP64 in entry order like every SpMV form, so
// the result is theirs bit for bit without reading a column index or gathering the vector. The row
// block's values are staged through LDS in chunks with coalesced loads; a row longer than a chunk is
// summed straight from memory.
// With values: 1024 threads and 32 KB chunks of values, a chunk at most one round of eight
// coalesced loads per thread. Pattern-only: 256 threads (row pointers only; fewer waves to launch).
__host__ __device__ constexpr int first_threads(bool has_val) { return has_val ? 1024 : kBlock; }
template <typename T, bool HAS_VAL>
__global__ __launch_bounds__(first_threads(HAS_VAL)) void k_spmv_first(LzArgs a) {
  constexpr int NT = first_threads(HAS_VAL), CAP = 32768 / (int)sizeof(T), U = kStreamU;
  __shared__ double chunks[kMaxChunks];
  __shared__ int rp_lds[kRowsPerBlock + 1];
  __shared__ T lv[HAS_VAL ? CAP : 1];
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  RState* st = a.state + ref.task;
  double sj;
  if (!open_step(a, tk, st, ref.blk, 0, chunks, &sj)) return;
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, rows = min(n - r0, kRowsPerBlock), tid = threadIdx.x;
  const int32_t* rp = a.row_ptr + tk.rowptr_off + r0;
  T* w = (T*)a.W + tk.w_off + r0;
  if constexpr (!HAS_VAL) {
    for (int r = tid; r < rows; r += NT) w[r] = (T)((double)(rp[r + 1] - rp[r]) * sj);
  } else {
    const T* va = (const T*)a.values + tk.nnz_off;
    for (int i = tid; i <= rows; i += NT) rp_lds[i] = rp[i];
    __syncthreads();
    int ra = 0;
    while (ra < rows) {
      const int k0 = rp_lds[ra];
      if (rp_lds[ra + 1] - k0 > CAP) {  // one long row: thread 0 sums it in order
        if (tid == 0) {
          double acc = 0.0;
          for (int k = k0; k < rp_lds[ra + 1]; ++k) acc += (double)va[k];
          w[ra] = (T)(acc * sj);
        }
        ++ra;
        continue;
      }
      int lo = ra + 1, hi = rows;  // largest rb with rp[rb] - rp[ra] <= CAP (same for every thread)
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rp_lds[mid] - k0 <= CAP) lo = mid; else hi = mid - 1;
      }
      const int rb = lo, ce = rp_lds[rb] - k0;
      for (int q0 = tid; q0 < ce; q0 += NT * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = q0 + u * NT < ce ? va[k0 + q0 + u * NT] : (T)0;
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (q0 + u * NT < ce) lv[q0 + u * NT] = v[u];
      }
      __syncthreads();
      for (int r = ra + tid; r < rb; r += NT) {
        double acc = 0.0;
        for (int k = rp_lds[r] - k0; k < rp_lds[r + 1] - k0; ++k) acc += (double)lv[k];
        w[r] = (T)(acc * sj);
      }
      __syncthreads();
      ra = rb;
    }
  }
}

// ------------------------------------------------------------------------------- column-segmented
// The random gathers of the CSR-stream form each cost an L1 miss: a row block's entries touch the
// whole vector. Here every call first sorts each row block's entries by column segment
// (k_seg_prepare, once per call: stable, so a row keeps its order inside a segment); each step then
// walks the segments in order: it stages v_j[segment] in LDS, streams the segment's entries (16-bit
// in-segment column, value) with coalesced loads, serves every gather from LDS into a product
// buffer, and adds each row's products to that row's FP64 sum in a register. Every wave owns a band
// of 128 consecutive rows (two per lane) and a private region of the product buffer: the band's
// entries of a segment are contiguous (offsets recorded by k_seg_prepare), so a wave forms and sums
// its products with no workgroup barrier. The vector slices are double-buffered, which leaves one
// workgroup barrier per segment. The loads of segment s + 1 (vector slice, per-row counts, entries)
// are issued into registers before the gathers of segment s, so one segment's memory latency hides
// behind the previous segment's LDS work.
// A row's products are added segment by segment and in entry order within a segment, so for rows
// stored with ascending columns the sums are those of the CSR-stream form, bit for bit.
constexpr int kSegThreads = 1024;
constexpr int kSegWaves = kSegThreads / 64;
constexpr int kBandRows = kRowsPerBlock / kSegWaves;  // rows per wave: 128, two per lane
template <typename T>
struct SegShape {
  static constexpr int WCAP = sizeof(T) == 8 ? 384 : 768;  // product slots per wave (3 KB)
  static constexpr int UE = WCAP / 64;                      // prefetched entries per lane
  static constexpr int XP = sizeof(T) == 8 ? 6 : 12;         // prefetched vector elements per thread
  static constexpr int MAXCOLS = XP * kSegThreads;           // largest segment (48 KB per LDS buffer)
};
static_assert(kBandRows == 128, "two rows per lane");

// Exclusive prefix sum of one int per thread over the workgroup; *total = the sum of all. wtot:
// NT/64 ints. Ends with a barrier, so wtot may be reused by the next call.
template <int NT>
__device__ inline int block_excl_scan(int v, int* wtot, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wtot[w] = inc;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const int t = wtot[i];
    before += i < w ? t : 0;
    all += t;
  }
  *total = all;
  __syncthreads();
  return before + inc - v;
}

// Visits the rows [0, rows) of a row block in chunks whose entries fit `cap` LDS slots: loads each
// chunk's columns (and values when HAS_VAL) with coalesced loads, then calls row_fn(r, cols, vals,
// first, last) with the row's entries at [first, last) of the staged arrays, each row on one
// thread. A row longer than cap is passed straight from global memory (cols = ci, vals = va).
template <typename T, bool HAS_VAL, int NT, typename F>
__device__ inline void for_rows_staged(const int32_t* __restrict__ ci, const T* __restrict__ va, const int* rp_lds,
                                       int rows, int cap, int* lci, T* lva, F row_fn) {
  const int tid = threadIdx.x;
  int ra = 0;
  while (ra < rows) {
    const int k0 = rp_lds[ra];
    if (rp_lds[ra + 1] - k0 > cap) {
      if (tid == 0) row_fn(ra, ci, va, k0, rp_lds[ra + 1]);
      __syncthreads();
      ++ra;
      continue;
    }
    int lo = ra + 1, hi = rows;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rp_lds[mid] - k0 <= cap) lo = mid; else hi = mid - 1;
    }
    const int rb = lo, ce = rp_lds[rb] - k0;
    for (int q0 = tid; q0 < ce; q0 += NT * 8) {
      int c[8];
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = q0 + u * NT;
        c[u] = k < ce ? ci[k0 + k] : 0;
        if constexpr (HAS_VAL) v[u] = k < ce ? va[k0 + k] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = q0 + u * NT;
        if (k < ce) {
          lci[k] = c[u];
          if constexpr (HAS_VAL) lva[k] = v[u];
        }
      }
    }
    __syncthreads();
    for (int r = ra + tid; r < rb; r += NT) row_fn(r, lci, lva, rp_lds[r] - k0, rp_lds[r + 1] - k0);
    __syncthreads();
    ra = rb;
  }
}

// for_rows_staged with each entry staged as one byte, f(column), instead of its column, so a chunk
// holds four times the entries: row_fn(r, s, first, last) sees the row's bytes at s[first, last). A
// row longer than cap is passed with s = nullptr and [first, last) its entries' positions in ci.
template <int NT, typename G, typename F>
__device__ inline void for_rows_staged_u8(const int32_t* __restrict__ ci, const int* rp_lds, int rows, int cap,
                                          uint8_t* ls, G f, F row_fn) {
  const int tid = threadIdx.x;
  int ra = 0;
  while (ra < rows) {
    const int k0 = rp_lds[ra];
    if (rp_lds[ra + 1] - k0 > cap) {
      if (tid == 0) row_fn(ra, (const uint8_t*)nullptr, k0, rp_lds[ra + 1]);
      __syncthreads();
      ++ra;
      continue;
    }
    int lo = ra + 1, hi = rows;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rp_lds[mid] - k0 <= cap) lo = mid; else hi = mid - 1;
    }
    const int rb = lo, ce = rp_lds[rb] - k0;
    for (int q0 = tid; q0 < ce; q0 += NT * 8) {
      int c[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = q0 + u * NT;
        c[u] = k < ce ? ci[k0 + k] : 0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = q0 + u * NT;
        if (k < ce) ls[k] = f(c[u]);
      }
    }
    __syncthreads();
    for (int r = ra + tid; r < rb; r += NT) row_fn(r, (const uint8_t*)ls, rp_lds[r] - k0, rp_lds[r + 1] - k0);
    __syncthreads();
    ra = rb;
  }
}

// One workgroup per row block. Dynamic LDS: the per-(segment, row) counters (16-bit, smax x 2048),
// then a staging area for `cap` entries (columns, and values for weighted graphs).
template <typename T, bool HAS_VAL>
__global__ __launch_bounds__(kSegThreads) void k_seg_prepare(LzArgs a, int cap) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NT = kSegThreads;
  __shared__ int rp_lds[kRowsPerBlock + 1];
  __shared__ int wtot[NT / 64];
  __shared__ int bad;
  __shared__ int maxband;  // slots of the block's largest padded band
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  const int n = tk.n, r0 = ref.blk * kRowsPerBlock, rows = min(n - r0, kRowsPerBlock);
  const int blk = tk.aux_blk + ref.blk, tid = threadIdx.x;  // the block in the form's arenas
  const int SEG = a.seg_cols, S = (n + SEG - 1) / SEG, tot = S * rows;
  // a column's segment c / SEG without an integer division per entry: the FP32 quotient, then one
  // step of correction (c < 2^24, so the estimate is off by at most one)
  const float inv_seg = 1.0f / (float)SEG;
  auto seg_of = [&](int c) {
    int q = (int)((float)c * inv_seg);
    q -= q * SEG > c ? 1 : 0;
    q += (q + 1) * SEG <= c ? 1 : 0;
    return q;
  };
  uint16_t* cnt = (uint16_t*)smem;  // [S * rows]: counts, then insertion cursors
  const size_t cnt_bytes = ((size_t)(a.seg_stride) * 2 + 15) / 16 * 16;
  int* lci = (int*)(smem + cnt_bytes);
  T* lva = (T*)(smem + cnt_bytes + (size_t)cap * 4);
  const int32_t* rp = a.row_ptr + tk.rowptr_off;
  for (int i = tid; i <= rows; i += NT) rp_lds[i] = rp[r0 + i];
  for (int i = tid; i < tot; i += NT) cnt[i] = 0;
  if (tid == 0) {
    bad = 0;
    maxband = 0;
  }
  __syncthreads();
  const int e0 = rp_lds[0];
  const int nz = rp_lds[rows] - e0;
  SegBlock* desc = a.seg_blk + blk;
  // Step 0's product from the all-ones start, when the caller has it computed here rather than in a
  // launch of its own (the values pass through this kernel anyway): each row's values added in entry
  // order in FP64 and scaled by s_0 = 1/sqrt(n), as the row-sum kernel does.
  const bool first = HAS_VAL && a.first_in_prepare;
  T* w0 = (T*)a.W + tk.w_off + r0;
  const double s0 = 1.0 / sqrt((double)n);
  auto direct_sums = [&](const T* v) {  // a block the sort does not take: rows from memory (v[rp_lds[r]])
    if (!first) return;
    for (int r = tid; r < rows; r += NT) {
      double acc = 0.0;
      for (int k = rp_lds[r]; k < rp_lds[r + 1]; ++k) acc += (double)v[k];
      w0[r] = (T)(acc * s0);
    }
  };
  // the block's first slot: its first entry's index in the form's arenas, moved past the padding
  // slots of the blocks before it and rounded up to a multiple of four (8- and 16-byte accesses)
  const int64_t base = (tk.aux_off + e0 + (int64_t)blk * kSegSlack + 3) & ~(int64_t)3;
  auto finish = [&](int f, int slots) {  // the block's flag and descriptor (band starts written by the caller)
    if (tid == 0) {
      a.seg_flag[blk] = f;
      desc->entries = base;
      desc->vec_off = tk.vec_off;
      desc->n = n;
      desc->nnz = slots;
      desc->rows = (int16_t)rows;
      desc->flag = (int16_t)f;
      desc->quads = (uint16_t)min(3, max(1, (maxband + 255) / 256));
    }
  };
  // offsets must fit 16 bits, the padding included (at most three slots per wave band)
  if (nz + 3 * kSegWaves * S > 65535 || S > kSegMax) {
    direct_sums(HAS_VAL ? (const T*)a.values + tk.nnz_off : nullptr);
    finish(0, 0);
    return;
  }
  const int32_t* ci = a.col_idx + tk.nnz_off + e0;
  const T* va = HAS_VAL ? (const T*)a.values + tk.nnz_off + e0 : nullptr;
  __syncthreads();  // every thread has read rp_lds[0] and rp_lds[rows]
  for (int i = tid; i <= rows; i += NT) rp_lds[i] -= e0;
  __syncthreads();
  // counts per (segment, row): a row is visited by one thread, so no counter has two writers. Only
  // each entry's segment is needed to count, so the entries are staged as their segment numbers, one
  // byte each (255: a column out of range), across the whole staging area: a chunk holds
  // 4 + sizeof(T) times the entries of a placement chunk (one chunk for a row block of the n=1e5,
  // degree-20 graph).
  const int cap8 = cap * (4 + (HAS_VAL ? (int)sizeof(T) : 0));
  const int32_t* ci_count = ci;
  for_rows_staged_u8<NT>(
      ci, rp_lds, rows, cap8, (uint8_t*)lci,
      [&](int c) { return (unsigned)c < (unsigned)n ? (uint8_t)seg_of(c) : (uint8_t)255; },
      [&](int r, const uint8_t* sg, int k, int e) {
        for (; k < e; ++k) {
          int q;
          if (sg != nullptr) {
            q = sg[k];
          } else {  // a row longer than the staging area: its columns from memory
            const int c = ci_count[k];
            q = (unsigned)c < (unsigned)n ? seg_of(c) : 255;
          }
          if (q == 255) {
            bad = 1;
            return;
          }
          const int idx = q * rows + r;
          if (cnt[idx] == 255) {  // the step kernel reads 8-bit counts
            bad = 1;
            return;
          }
          cnt[idx] = (uint16_t)(cnt[idx] + 1);
        }
      });
  if (bad) {
    direct_sums(va);
    finish(0, 0);
    return;
  }
  // counts with the rows of a segment at an even stride (one 2-byte load reads a lane's two rows;
  // the pad row of an odd block counts 0)
  const int rows2 = (rows + 1) & ~1;
  uint8_t* cnt_out = a.seg_cnt + (size_t)blk * a.seg_stride;
  for (int sg = 0; sg < S; ++sg)
    for (int r = tid; r < rows2; r += NT) cnt_out[sg * rows2 + r] = r < rows ? (uint8_t)cnt[sg * rows + r] : (uint8_t)0;
  // exclusive scan in (segment, row) order: thread t owns counters [b, e)
  const int per = (tot + NT - 1) / NT;
  const int b = min(tid * per, tot), e = min(b + per, tot);
  int sum = 0;
  for (int i = b; i < e; ++i) sum += cnt[i];
  int total;
  int run = block_excl_scan<NT>(sum, wtot, &total);
  for (int i = b; i < e; ++i) {
    const int c = cnt[i];
    cnt[i] = (uint16_t)run;
    run += c;
  }
  __syncthreads();
  // wave bands: the entries of rows [128 w, 128 w + 128) in segment s, in (segment, band) order. Each
  // band's run is padded with zeros to a multiple of four entries, so that every band starts at a
  // multiple of four slots; band t's entries move by the padding of the bands before it.
  const int nbw = (rows + kBandRows - 1) / kBandRows, NB = S * nbw;  // NB <= 32 x 16 <= NT
  __shared__ int bpad[kSegMax * kSegWaves];
  int ustart = 0, ulen = 0;
  if (tid < NB) {
    const int sg = tid / nbw, w = tid - sg * nbw;
    ustart = cnt[sg * rows + w * kBandRows];
    const int uend = w + 1 < nbw ? cnt[sg * rows + (w + 1) * kBandRows] : (sg + 1 < S ? cnt[(sg + 1) * rows] : total);
    ulen = uend - ustart;
  }
  int padtot;
  const int pex = block_excl_scan<NT>(tid < NB ? ((ulen + 3) & ~3) - ulen : 0, wtot, &padtot);
  if (tid < NB) bpad[tid] = pex;
  __syncthreads();
  const int slots = total + padtot;
  if (b < e) {  // this thread's counters move by their bands' padding (one division, then steps)
    int sg = b / rows, r = b - sg * rows;
    for (int i = b; i < e; ++i) {
      cnt[i] = (uint16_t)(cnt[i] + bpad[sg * nbw + (r >> 7)]);
      if (++r == rows) {
        r = 0;
        ++sg;
      }
    }
  }
  __syncthreads();
  // band table: wo[s][w] = start of band w of segment s; wo[s][w] for w >= the block's bands (and
  // wo[s][16]) = the end of segment s. A band beyond the per-wave product capacity sends the block to
  // the stream form.
  uint16_t* wo = a.seg_woff + (size_t)blk * a.seg_wstride;
  auto band_start = [&](int sg, int w) {
    return w < nbw ? (int)cnt[sg * rows + w * kBandRows] : (sg + 1 < S ? (int)cnt[(sg + 1) * rows] : slots);
  };
  for (int i = tid; i < S * (kSegWaves + 1); i += NT) {
    const int sg = i / (kSegWaves + 1), w = i - sg * (kSegWaves + 1);
    const int v = band_start(sg, w);
    wo[i] = (uint16_t)v;
    if (i <= kSegWaves) desc->wo0[i] = (uint16_t)v;  // segment 0 (i = w)
    if (w < kSegWaves) {
      const int len = band_start(sg, w + 1) - v;
      if (len > SegShape<T>::WCAP) bad = 1;
      atomicMax(&maxband, len);
    }
  }
  __syncthreads();
  if (bad) {
    direct_sums(va);
    finish(0, 0);
    return;
  }
  uint16_t* pc = a.seg_col + base;
  T* pv = HAS_VAL ? (T*)a.seg_val + base : nullptr;
  if (tid < NB) {  // the band's padding slots
    const int p0 = ustart + pex + ulen, p1 = ustart + pex + ((ulen + 3) & ~3);
    for (int p = p0; p < p1; ++p) {
      pc[p] = 0;
      if constexpr (HAS_VAL) pv[p] = (T)0;
    }
  }
  for_rows_staged<T, HAS_VAL, NT>(ci, va, rp_lds, rows, cap, lci, lva,
                                  [&](int r, const int* cs, const T* vs, int k, int e) {
                                    double acc = 0.0;
                                    for (; k < e; ++k) {
                                      const int c = cs[k];
                                      const int sg = seg_of(c);
                                      const int pos = cnt[sg * rows + r];
                                      cnt[sg * rows + r] = (uint16_t)(pos + 1);
                                      pc[pos] = (uint16_t)(c - sg * SEG);
                                      if constexpr (HAS_VAL) {
                                        pv[pos] = vs[k];
                                        acc += (double)vs[k];
                                      }
                                    }
                                    if (first) w0[r] = (T)(acc * s0);
                                  });
  finish(1, slots);
}

// Raw buffer resource over [p, p + bytes): loads through it take 32-bit byte offsets and return 0
// past the end.
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}

// A row block's descriptor with its fields in scalar registers. The buffer resources built from them
// must be wave-uniform; a field read with a vector load (the compiler's choice) would put them in
// vector registers, and every load through them would then loop over the wave's distinct values.
struct SegDesc {
  int64_t entries, vec_off;
  int n, nnz, rows, flag;
};
__device__ inline int64_t wave_uniform(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline SegDesc seg_desc(const SegBlock* d) {
  SegDesc r;
  r.entries = wave_uniform(d->entries);
  r.vec_off = wave_uniform(d->vec_off);
  r.n = __builtin_amdgcn_readfirstlane(d->n);
  r.nnz = __builtin_amdgcn_readfirstlane(d->nnz);
  r.rows = __builtin_amdgcn_readfirstlane((int)d->rows);
  r.flag = __builtin_amdgcn_readfirstlane((int)d->flag);
  return r;
}

// Cache-policy operand of a buffer load that streams the matrix (read once per product): the
// non-temporal bit, so that the L2 keeps the lines of the vector slices instead (measured: 4% off the
// segmented product, and the dot kernel that reads its output gains as well).
constexpr int kStreamPolicy = 2;

template <typename T, int AUX = 0>
__device__ inline T load_elem(__amdgpu_buffer_rsrc_t r, int i) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8, 0, AUX));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, AUX));
}

// Wave-exclusive prefix sum of v (lanes below this one), in registers with DPP: inclusive scans of
// the four rows of 16 lanes by row shifts 1, 2, 4, 8, then lane 15's total broadcast into rows 1
// and 3 and lane 31's into rows 2 and 3. Disabled rows and lanes whose source is outside the row
// read 0.
__device__ inline int wave_excl_scan(int v) {
  int x = v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
  return x - v;
}

// LDS writes of this wave visible to all of its lanes.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One workgroup barrier per segment: after it, the slice of segment s + 1 is staged in the other
// buffer. The loads of segment s + 1 are issued at the top of segment s; the first segment's loads
// are issued before the step is opened.
template <typename T, bool HAS_VAL, bool VEC>
__global__ __launch_bounds__(kSegThreads) void k_spmv_seg(LzArgs a, int j) {
  if (all_stopped(a, j)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  using SS = SegShape<T>;
  constexpr int NT = kSegThreads, UE = SS::UE, XP = SS::XP, WCAP = SS::WCAP;
  __shared__ T prod[kSegWaves * WCAP];
  __shared__ int p_lds[kRowsPerBlock + 1];  // stream fallback only
  __shared__ uint16_t wo_lds[kSegMax * (kSegWaves + 1)];
  __shared__ double chunks[kMaxChunks];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  // The first segment's loads wait on the block's descriptor alone: in a batched launch the logical
  // workgroup is the block's index in the form's arenas (the launch covers the form's blocks in order).
  const int lb = logical_block();
  const int blk = a.blkmap != nullptr ? lb : a.tasks[a.single_task].aux_blk + lb;
  const SegBlock* d = a.seg_blk + blk;
  const int n = d->n, rows = d->rows, flag = d->flag, E = d->nnz;
  const int SEG = a.seg_cols, S = (n + SEG - 1) / SEG;
  T* pw = prod + wv * WCAP;
  const T* x = (const T*)a.V + d->vec_off + vslot(a, j) * n;
  const uint8_t* cnt = a.seg_cnt + (size_t)blk * a.seg_stride;
  const uint16_t* wo = a.seg_woff + (size_t)blk * a.seg_wstride;
  const uint16_t* pc = a.seg_col + d->entries;
  const T* pv = HAS_VAL ? (const T*)a.seg_val + d->entries : nullptr;
  const int rr = 2 * tid;  // this lane's two rows: 128 wv + 2 lane and the next
  const int rows2 = (rows + 1) & ~1;  // the counts' stride per segment
  // Buffer resources (scalar registers) over the block's entries, its counts and the vector: loads
  // take 32-bit byte offsets, and an offset past the end reads 0, which is what every guard wants.
  const __amdgpu_buffer_rsrc_t r_pc = make_rsrc(pc, 2 * E);
  const __amdgpu_buffer_rsrc_t r_pv = make_rsrc(pv, HAS_VAL ? (int)sizeof(T) * E : 0);
  const __amdgpu_buffer_rsrc_t r_cnt = make_rsrc(cnt, S * rows2);
  const __amdgpu_buffer_rsrc_t r_x = make_rsrc(x, (int)sizeof(T) * n);
  // registers holding the next segment: vector slice, two counts, the band's entries
  // VEC: 16-byte slice loads and LDS stores (the host selects it when every realization's n and the
  // segment length are multiples of the vector width, so that every segment start and length is one
  // too and no store passes the end of its slice)
  constexpr int VW = 16 / sizeof(T);
  using VT = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
  T xr[VEC ? 1 : XP];
  VT xq[VEC ? XP / VW : 1];
  int nb0 = 0, nb1 = 0;
  uint32_t craw = 0;
  int ec[UE] = {};
  T ev[UE] = {};
  auto prefetch = [&](int s, int b0, int b1) {  // b0, b1: the band's entry range in segment s
    const int base = s * SEG, len = min(SEG, n - base);
    if constexpr (VEC) {
#pragma unroll
      for (int u = 0; u < XP / VW; ++u) {
        const int i = (tid + u * NT) * VW;  // past the segment: the next one's or zeros, never stored
        xq[u] = __builtin_bit_cast(VT, __builtin_amdgcn_raw_buffer_load_b128(r_x, (base + i) * (int)sizeof(T), 0, 0));
      }
    } else {
#pragma unroll
      for (int u = 0; u < XP; ++u) {
        const int i = tid + u * NT;
        xr[u] = i < len ? load_elem<T>(r_x, base + i) : (T)0;
      }
    }
    // the two counts as one 16-bit word (the even stride keeps it 2-byte aligned), unpacked when
    // staged: an unpack here would wait for this load and every load before it
    craw = rr < rows ? __builtin_amdgcn_raw_buffer_load_b16(r_cnt, s * rows2 + rr, 0, kStreamPolicy) : 0u;
    nb0 = b0;
    nb1 = b1;
    const int nbw = __builtin_amdgcn_readfirstlane(b1 - b0);  // the band's entries (wave-uniform)
#pragma unroll
    for (int u = 0; u < UE; ++u) {
      if (u * 64 < nbw) {  // slots wholly past the band issue no load
        const int k = b0 + lane + u * 64;
        const int kk = k < b1 ? k : E;  // past the band: read as zero (never used)
        ec[u] = __builtin_amdgcn_raw_buffer_load_b16(r_pc, 2 * kk, 0, kStreamPolicy);
        if constexpr (HAS_VAL) ev[u] = load_elem<T, kStreamPolicy>(r_pv, kk);
      }
    }
  };
  if (flag) prefetch(0, d->wo0[wv], d->wo0[wv + 1]);  // consumed only if the step runs
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  RState* st = a.state + ref.task;
  const int r0 = ref.blk * kRowsPerBlock;
  T* w_out = (T*)a.W + tk.w_off + r0;
  const int32_t* rp = a.row_ptr + tk.rowptr_off;
  double sj;
  if (!open_step(a, tk, st, ref.blk, j, chunks, &sj)) return;
  if (!flag) {
    const T* va = HAS_VAL ? (const T*)a.values + tk.nnz_off : nullptr;
    spmv_stream_rows<T, HAS_VAL, NT, kSegWaves * WCAP>(rp, a.col_idx + tk.nnz_off, va, x, r0, rows, sj, p_lds, prod,
                                                      w_out, red);
    return;
  }
  for (int i = tid; i < S * (kSegWaves + 1); i += NT) wo_lds[i] = wo[i];
  // the current segment: its entries, this lane's counts and offsets in the wave's product region
  int cc[UE];
  T cv[UE];
  int c0 = 0, c1 = 0, ex = 0, bn = 0;
  auto stage = [&](int s, int buf) {
    const int len = min(SEG, n - s * SEG);
    T* xb = (T*)smem + buf * SEG;
    if constexpr (VEC) {
#pragma unroll
      for (int u = 0; u < XP / VW; ++u) {
        const int i = (tid + u * NT) * VW;
        if (i < len) *(VT*)(xb + i) = xq[u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < XP; ++u) {
        const int i = tid + u * NT;
        if (i < len) xb[i] = xr[u];
      }
    }
    c0 = (int)(craw & 0xFF);
    c1 = (int)(craw >> 8);
    ex = wave_excl_scan(c0 + c1);
    bn = __builtin_amdgcn_readfirstlane(nb1 - nb0);
#pragma unroll
    for (int u = 0; u < UE; ++u) {
      cc[u] = ec[u];
      if constexpr (HAS_VAL) cv[u] = ev[u];
    }
  };
  stage(0, 0);
  __syncthreads();  // slice 0 and the band table published
  double acc0 = 0.0, acc1 = 0.0;  // rows rr and rr + 1
  constexpr int WO = kSegWaves + 1;
  for (int s = 0; s < S; ++s) {
    const int buf = s & 1;
    if (s + 1 < S) prefetch(s + 1, wo_lds[(s + 1) * WO + wv], wo_lds[(s + 1) * WO + wv + 1]);
    const T* xb = (const T*)smem + buf * SEG;
#pragma unroll
    for (int u = 0; u < UE; ++u) {
      if (u * 64 < bn) {  // wave-uniform
        const int k = lane + u * 64;
        if (k < bn) {
          const T xv = xb[cc[u]];
          if constexpr (HAS_VAL) pw[k] = cv[u] * xv; else pw[k] = xv;
        }
      }
    }
    wave_lds_sync();
    for (int k = ex; k < ex + c0; ++k) acc0 += (double)pw[k];
    for (int k = ex + c0; k < ex + c0 + c1; ++k) acc1 += (double)pw[k];
    wave_lds_sync();  // the band's next products overwrite pw
    if (s + 1 < S) {
      stage(s + 1, buf ^ 1);  // the other buffer's last readers were segment s - 1's products
      __syncthreads();
    }
  }
  if (rr < rows) w_out[rr] = (T)(acc0 * sj);
  if (rr + 1 < rows) w_out[rr + 1] = (T)(acc1 * sj);
}

// FP32 form of the same product with its loads reorganised. Every band starts at a multiple of four
// slots (the sort pads the runs with zeros), so a lane loads four columns with one 8-byte load and
// four values with one 16-byte load, and stores its four products with one 16-byte LDS store. Every
// lane issues the same loads for every segment: its band's quad slots, its share of the slice and its
// counts. Slots past the band, past the block, and segments past the last are pointed past the end of
// their buffer resource and read zeros without touching memory (the range check). So where a
// segment's registers are read, the compiler knows how many later loads may stay in flight. The
// loads of segment s + 2 are issued as soon as segment s's products are formed and stay in flight
// while segment s + 1 is staged, about two segments before they are used; two register sets take the
// segments of even and odd index. The sums are those of the form above, bit for bit: the same
// products added to the same FP64 row sums in the same order.
// One row block with UQ quad slots per lane and segment (its largest band holds at most 256 UQ
// slots). smem: the two slice buffers; prod: the waves' product slots; p_lds, chunks, red: scratch of
// the stream arithmetic and the step's opening.
template <bool HAS_VAL, bool VEC, int UQ>
__device__ inline void seg4_block(const LzArgs& a, int j, int blk, const SegBlock* d, unsigned char* smem,
                                  float* prod, int* p_lds, uint16_t* wo_lds, double* chunks, double* red) {
  using T = float;
  using SS = SegShape<T>;
  constexpr int NT = kSegThreads, XP = SS::XP, WCAP = SS::WCAP, WO = kSegWaves + 1;
  static_assert(UQ >= 1 && 256 * UQ <= WCAP && XP % 4 == 0, "quad slots within the product slots");
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const SegDesc dd = seg_desc(d);
  const int n = dd.n, rows = dd.rows, flag = dd.flag, E = dd.nnz;
  const int SEG = a.seg_cols, S = (n + SEG - 1) / SEG, rows2 = (rows + 1) & ~1, QEND = (E + 3) >> 2;
  T* pw = prod + wv * WCAP;
  const T* x = (const T*)a.V + dd.vec_off + vslot(a, j) * n;
  const uint8_t* cnt = a.seg_cnt + (size_t)blk * a.seg_stride;
  const uint16_t* wo = a.seg_woff + (size_t)blk * a.seg_wstride;
  const int rr = 2 * tid;  // this lane's two rows
  const __amdgpu_buffer_rsrc_t r_pc = make_rsrc(a.seg_col + dd.entries, 2 * E);
  const __amdgpu_buffer_rsrc_t r_pv =
      make_rsrc(HAS_VAL ? (const T*)a.seg_val + dd.entries : nullptr, HAS_VAL ? 4 * E : 0);
  const __amdgpu_buffer_rsrc_t r_cnt = make_rsrc(cnt, S * rows2);
  const __amdgpu_buffer_rsrc_t r_x = make_rsrc(x, 4 * n);
  struct Set {
    float4 xq[VEC ? XP / 4 : 1];  // the slice, 16 bytes per load
    T xr[VEC ? 1 : XP];           // the slice, one element per load
    uint32_t craw;                // the lane's two 8-bit counts
    uint64_t cq[UQ];              // four 16-bit columns per quad slot
    float4 vq[HAS_VAL ? UQ : 1];  // four values per quad slot
  };
  // the loads of segment s into p (zeros for s >= S); [q0, q1) = the wave's band in quads
  auto load = [&](Set& p, int s, int q0, int q1) {
    const int base = s * SEG;
    if constexpr (VEC) {
#pragma unroll
      for (int u = 0; u < XP / 4; ++u)
        p.xq[u] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r_x, (base + (tid + u * NT) * 4) * 4, 0, 0));
    } else {
#pragma unroll
      for (int u = 0; u < XP; ++u) p.xr[u] = load_elem<T>(r_x, base + tid + u * NT);
    }
    p.craw = __builtin_amdgcn_raw_buffer_load_b16(r_cnt, s * rows2 + rr, 0, kStreamPolicy);
#pragma unroll
    for (int u = 0; u < UQ; ++u) {
      const int q = q0 + lane + 64 * u < q1 ? q0 + lane + 64 * u : QEND;  // past the band: out of range
      p.cq[u] = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r_pc, 8 * q, 0, kStreamPolicy));
      if constexpr (HAS_VAL)
        p.vq[u] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r_pv, 16 * q, 0, kStreamPolicy));
    }
  };
  Set A, B;
  if (flag) load(A, 0, d->wo0[wv] >> 2, d->wo0[wv + 1] >> 2);  // consumed only if the step runs
  const Ref ref = resolve(a);
  const Task tk = a.tasks[ref.task];
  RState* st = a.state + ref.task;
  const int r0 = ref.blk * kRowsPerBlock;
  T* w_out = (T*)a.W + tk.w_off + r0;
  const int32_t* rp = a.row_ptr + tk.rowptr_off;
  double sj;
  if (!open_step(a, tk, st, ref.blk, j, chunks, &sj)) return;
  if (!flag) {
    const T* va = HAS_VAL ? (const T*)a.values + tk.nnz_off : nullptr;
    spmv_stream_rows<T, HAS_VAL, NT, kSegWaves * WCAP>(rp, a.col_idx + tk.nnz_off, va, x, r0, rows, sj, p_lds, prod,
                                                      w_out, red);
    return;
  }
  for (int i = tid; i < S * WO; i += NT) wo_lds[i] = wo[i];
  load(B, 1, S > 1 ? (int)wo[WO + wv] >> 2 : QEND, S > 1 ? (int)wo[WO + wv + 1] >> 2 : QEND);
  int c0 = 0, c1 = 0, ex = 0;  // the current segment's counts of the lane's two rows, their offset in pw
  auto stage = [&](const Set& p, int s) {
    const int len = min(SEG, n - s * SEG);
    T* xb = (T*)smem + (s & 1) * SEG;
    if constexpr (VEC) {
#pragma unroll
      for (int u = 0; u < XP / 4; ++u) {
        const int i = (tid + u * NT) * 4;
        if (i < len) *(float4*)(xb + i) = p.xq[u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < XP; ++u) {
        const int i = tid + u * NT;
        if (i < len) xb[i] = p.xr[u];
      }
    }
    const uint32_t cr = rr < rows ? p.craw : 0u;
    c0 = (int)(cr & 0xFF);
    c1 = (int)((cr >> 8) & 0xFF);
    ex = wave_excl_scan(c0 + c1);
  };
  stage(A, 0);
  __syncthreads();  // slice 0 and the band table published
  double acc0 = 0.0, acc1 = 0.0;  // rows rr and rr + 1
  // segment s: its products from set p, then p takes the loads of segment s + 2, the row sums, and
  // segment s + 1 staged from set q
  auto segment = [&](int s, Set& p, const Set& q) {
    const T* xb = (const T*)smem + (s & 1) * SEG;
    const int bn = __builtin_amdgcn_readfirstlane((int)wo_lds[s * WO + wv + 1] - (int)wo_lds[s * WO + wv]);
#pragma unroll
    for (int u = 0; u < UQ; ++u) {
      if (u * 256 < bn) {  // wave-uniform: quad slots wholly past the band form no products
        const uint64_t c4 = p.cq[u];
        const T x0 = xb[(int)(c4 & 0xFFFF)], x1 = xb[(int)((c4 >> 16) & 0xFFFF)];
        const T x2 = xb[(int)((c4 >> 32) & 0xFFFF)], x3 = xb[(int)(c4 >> 48)];
        float4 pr;
        if constexpr (HAS_VAL) {
          pr.x = p.vq[u].x * x0;
          pr.y = p.vq[u].y * x1;
          pr.z = p.vq[u].z * x2;
          pr.w = p.vq[u].w * x3;
        } else {
          pr = make_float4(x0, x1, x2, x3);
        }
        *(float4*)(pw + 4 * (lane + 64 * u)) = pr;
      }
    }
    load(p, s + 2, s + 2 < S ? (int)wo_lds[(s + 2) * WO + wv] >> 2 : QEND,
         s + 2 < S ? (int)wo_lds[(s + 2) * WO + wv + 1] >> 2 : QEND);
    wave_lds_sync();
    for (int k = ex; k < ex + c0; ++k) acc0 += (double)pw[k];
    for (int k = ex + c0; k < ex + c0 + c1; ++k) acc1 += (double)pw[k];
    wave_lds_sync();  // the band's next products overwrite pw
    if (s + 1 < S) {
      stage(q, s + 1);  // the other buffer's last readers were segment s - 1's products
      __syncthreads();
    }
  };
  // pairs of segments, then an odd last one: the loop's back edge always follows a segment of set B,
  // so the count of loads in flight where set A is read is the same on every path into the loop head
  int s = 0;
  for (; s + 1 < S; s += 2) {
    segment(s, A, B);
    segment(s + 1, B, A);
  }
  if (s < S) segment(s, A, B);
  if (rr < rows) w_out[rr] = (T)(acc0 * sj);
  if (rr + 1 < rows) w_out[rr + 1] = (T)(acc1 * sj);
}

template <bool HAS_VAL, bool VEC>
__global__ __launch_bounds__(kSegThreads) void k_spmv_seg4(LzArgs a, int j) {
  if (all_stopped(a, j)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ __align__(16) float prod[kSegWaves * SegShape<float>::WCAP];
  __shared__ int p_lds[kRowsPerBlock + 1];  // stream fallback only
  __shared__ uint16_t wo_lds[kSegMax * (kSegWaves + 1)];
  __shared__ double chunks[kMaxChunks];
  __shared__ double red[kSegThreads / 64];
  // the first segments' loads wait on the block's descriptor alone: in a batched launch the logical
  // workgroup is the block's index in the form's arenas (the launch covers the form's blocks in order)
  const int lb = logical_block();
  const int blk = a.blkmap != nullptr ? lb : a.tasks[a.single_task].aux_blk + lb;
  const SegBlock* d = a.seg_blk + blk;
  // the block's quad slots per segment (one branch per workgroup: each count is its own loop, so the
  // number of loads in flight stays fixed inside it)
  switch (d->quads) {
    case 1: seg4_block<HAS_VAL, VEC, 1>(a, j, blk, d, smem, prod, p_lds, wo_lds, chunks, red); break;
    case 2: seg4_block<HAS_VAL, VEC, 2>(a, j, blk, d, smem, prod, p_lds, wo_lds, chunks, red); break;
    default: seg4_block<HAS_VAL, VEC, 3>(a, j, blk, d, smem, prod, p_lds, wo_lds, chunks, red); break;
  }
}

template <typename T>
constexpr size_t seg_static_bytes() {
  return (size_t)kSegWaves * SegShape<T>::WCAP * sizeof(T) + (size_t)(kRowsPerBlock + 1) * 4 +
         (size_t)kSegMax * (kSegWaves + 1) * 2 + kMaxChunks * 8 + (kSegThreads / 64) * 8 + 512;
}

// Static LDS of k_seg_prepare (row pointers, band padding, scan scratch) with a margin.
constexpr size_t kSegPrepStatic = (size_t)(kRowsPerBlock + 1) * 4 + (size_t)kSegMax * kSegWaves * 4 + 1024;
// Staging capacity (entries) of k_seg_prepare next to smax x kRowsPerBlock 16-bit counters.
template <typename T, bool HAS_VAL>
int seg_prepare_cap(int smax) {
  const size_t fixed = kSegPrepStatic;
  const size_t cnt = ((size_t)smax * kRowsPerBlock * 2 + 15) / 16 * 16;
  const size_t per = 4 + (HAS_VAL ? sizeof(T) : 0);
  const size_t cap = (kLdsBytes - fixed - cnt) / per;
  return (int)std::min<size_t>(16384, cap / 256 * 256);
}

// ------------------------------------------------------------------------------- paneled
// For vectors of megabytes (n = 1e6: 82 column panels of 12288 FP32 elements) the column-segmented
// form would stage every segment once per row block, so its slice traffic grows with n; the gathers of
// the stream form miss L2. Here the two are decoupled. Rows are cut into units of pan_unit rows (64,
// 128 or 256, dividing the 2048-row block), units into groups. Once per call the entries of each group
// are put in (panel, unit) order: k_pan_count counts each unit's entries per panel, k_pan_scan turns
// the counts into run offsets in that order, k_pan_place writes each entry's 16-bit in-panel column,
// its 16-bit position in the unit's CSR range and its value at the next free slot of its run (the order
// inside a run does not matter: the row-sum pass puts every product back at its CSR position). Each
// step then runs two passes:
//   products  one workgroup per (realization, panel, group): the panel's slice of v_j is staged in LDS
//             once and serves the group's entries of that panel, one contiguous range read and written
//             with coalesced loads and stores (prod = value * slice[column], in the working precision,
//             as the stream form forms them). Items are ordered by panel, and each XCD takes a
//             contiguous range of them, so the slices an XCD reads stay in its L2;
//   row sums  one workgroup per unit: the unit's per-panel runs, scattered into LDS by CSR position,
//             then each row's products added in entry order in FP64 (the stream form's sums, bit for
//             bit), times s_j. The step's opening (beta_{j-1}, s_j, breakdown) is taken by the products
//             pass, whose items are fewer, and read here from the realization's state.
// A unit with more entries than the row-sum pass holds in LDS (pan_lds), or with a row beyond the
// stream form's capacity (whose sum that form forms another way), is left out of the sort and summed
// with the stream arithmetic in the row-sum pass.
constexpr int kPanPrepThreads = 256;
constexpr int kPanScanThreads = 1024;
constexpr int kPanProdThreads = 512;
constexpr int kPanRowThreads = 256;

template <typename T>
struct PanShape {
  static constexpr int MAXCOLS = sizeof(T) == 8 ? 6144 : 12288;  // slice of the products pass (48 KB)
};

// Dynamic LDS of the row-sum pass: the unit's products (at least the stream arithmetic's buffer, which
// the pass falls back to), then the runs' prefix sums and offsets.
template <typename T>
__host__ __device__ inline size_t pan_rows_lds(int pan_lds, int pmax) {
  const size_t prod = (size_t)(pan_lds > StreamShape<T>::CAP ? pan_lds : StreamShape<T>::CAP) * sizeof(T);
  return (prod + 15) / 16 * 16 + (size_t)(2 * pmax + 2) * sizeof(int);
}

struct PanRef {
  int task;
  int u;       // unit index in the realization
  int64_t gu;  // unit index in the launch's unit arrays
};

// Units of the launch: kRowsPerBlock / pan_unit per row block, in block order.
__device__ inline PanRef pan_ref(const LzArgs& a) {
  const int k = kRowsPerBlock / a.pan_unit;
  const int lb = logical_block(), lblk = lb / k, sub = lb - lblk * k;
  int t, blk;
  if (a.blkmap == nullptr) {
    t = a.single_task;
    blk = lblk;
  } else {
    const int gb = a.sub_blocks ? a.sub_blocks[lblk] : lblk;
    t = a.blkmap[gb];
    blk = gb - a.tasks[t].blk_begin;
  }
  return {t, blk * k + sub, ((int64_t)a.tasks[t].aux_blk + blk) * k + sub};
}

template <typename T>
__global__ __launch_bounds__(kPanPrepThreads) void k_pan_count(LzArgs a) {
  constexpr int NT = kPanPrepThreads;
  __shared__ int rp_lds[kPanMaxUnit + 1];
  __shared__ int cnt[kPanMaxPanels];
  __shared__ int bad;
  const PanRef ref = pan_ref(a);
  const Task tk = a.tasks[ref.task];
  const int n = tk.n, U = a.pan_unit, r0 = ref.u * U, rows = min(n - r0, U), tid = threadIdx.x;
  const int S = a.pan_cols, P = (n + S - 1) / S;
  if (rows <= 0) {  // the trailing units of a realization's last block
    if (tid == 0) a.pan_flag[ref.gu] = 0;
    return;
  }
  int2* run = a.pan_run + ref.gu * a.pan_pmax;
  const int32_t* rp = a.row_ptr + tk.rowptr_off;
  for (int i = tid; i <= rows; i += NT) rp_lds[i] = rp[r0 + i];
  for (int p = tid; p < P; p += NT) cnt[p] = 0;
  if (tid == 0) bad = P > a.pan_pmax ? 1 : 0;
  __syncthreads();
  const int e0 = rp_lds[0], nz = rp_lds[rows] - e0;
  for (int r = tid; r < rows; r += NT)
    if (rp_lds[r + 1] - rp_lds[r] > StreamShape<T>::CAP) bad = 1;
  __syncthreads();
  const bool ok = !bad && nz <= a.pan_lds;
  if (ok) {
    const int32_t* ci = a.col_idx + tk.nnz_off + e0;
    for (int e = tid; e < nz; e += NT) atomicAdd(&cnt[min(max(ci[e] / S, 0), P - 1)], 1);
    __syncthreads();
  }
  for (int p = tid; p < min(P, a.pan_pmax); p += NT) run[p] = make_int2(0, ok ? cnt[p] : 0);
  if (tid == 0) a.pan_flag[ref.gu] = ok ? 1 : 0;
}

// Run offsets of one group (units [b0, b1) of a realization), in (panel, unit) order, from the entry
// offset of the group's first row on.
__global__ __launch_bounds__(kPanScanThreads) void k_pan_scan(LzArgs a, const PanItem* groups) {
  constexpr int NT = kPanScanThreads;
  __shared__ int wtot[NT / 64];
  const PanItem g = groups[blockIdx.x];
  const Task tk = a.tasks[g.task];
  const int n = tk.n, U = a.pan_unit, S = a.pan_cols, P = (n + S - 1) / S, tid = threadIdx.x;
  const int gsz = g.b1 - g.b0, E = P * gsz;
  const int64_t gu0 = (int64_t)tk.aux_blk * (kRowsPerBlock / U) + g.b0;
  int carry = a.row_ptr[tk.rowptr_off + min(n, g.b0 * U)];
  for (int i0 = 0; i0 < E; i0 += NT) {
    const int i = i0 + tid, p = i / gsz, uu = i - p * gsz;
    int2* cell = a.pan_run + (gu0 + uu) * a.pan_pmax + p;
    const int v = i < E ? cell->y : 0;
    int total = 0;
    const int ex = block_excl_scan<NT>(v, wtot, &total);
    if (i < E) cell->x = carry + ex;
    carry += total;
  }
}

template <typename T, bool HAS_VAL>
__global__ __launch_bounds__(kPanPrepThreads) void k_pan_place(LzArgs a) {
  constexpr int NT = kPanPrepThreads;
  __shared__ int rp_lds[2];
  __shared__ int cursor[kPanMaxPanels];
  const PanRef ref = pan_ref(a);
  if (!a.pan_flag[ref.gu]) return;
  const Task tk = a.tasks[ref.task];
  const int n = tk.n, U = a.pan_unit, r0 = ref.u * U, rows = min(n - r0, U), tid = threadIdx.x;
  const int S = a.pan_cols, P = (n + S - 1) / S;
  const int2* run = a.pan_run + ref.gu * a.pan_pmax;
  const int32_t* rp = a.row_ptr + tk.rowptr_off;
  if (tid == 0) {
    rp_lds[0] = rp[r0];
    rp_lds[1] = rp[r0 + rows];
  }
  for (int p = tid; p < P; p += NT) cursor[p] = run[p].x;
  __syncthreads();
  const int e0 = rp_lds[0], nz = rp_lds[1] - e0;
  const int32_t* ci = a.col_idx + tk.nnz_off + e0;
  const T* va = HAS_VAL ? (const T*)a.values + tk.nnz_off + e0 : nullptr;
  uint16_t* oc = a.pan_col + tk.aux_off;
  uint16_t* op = a.pan_perm + tk.aux_off;
  T* ov = HAS_VAL ? (T*)a.pan_val + tk.aux_off : nullptr;
  for (int e = tid; e < nz; e += NT) {
    const int c = ci[e], p = min(max(c / S, 0), P - 1);
    const int pos = atomicAdd(&cursor[p], 1);
    oc[pos] = (uint16_t)min(max(c - p * S, 0), S - 1);
    op[pos] = (uint16_t)e;
    if constexpr (HAS_VAL) ov[pos] = va[e];
  }
}

// Products of one work item: panel `panel` of units [b0, b1), one contiguous range of entries.
template <typename T, bool HAS_VAL>
__global__ __launch_bounds__(kPanProdThreads) void k_pan_products(LzArgs a, int j) {
  if (all_stopped(a, j)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NT = kPanProdThreads, U = 8;
  T* slice = (T*)smem;
  __shared__ double chunks[kMaxChunks];
  const PanItem it = a.pan_items[logical_block()];
  const Task tk = a.tasks[it.task];
  // the step's opening (beta_{j-1} from the partials, breakdown) is taken here, once per item instead
  // of once per row unit; the realization's first item records it for the row-sum pass
  double sj;
  if (!open_step(a, tk, a.state + it.task, it.panel == 0 && it.b0 == 0 ? 0 : 1, j, chunks, &sj)) return;
  const int n = tk.n, S = a.pan_cols, c0 = it.panel * S, len = min(S, n - c0), tid = threadIdx.x;
  const int64_t gu0 = (int64_t)tk.aux_blk * (kRowsPerBlock / a.pan_unit);
  const int2 first = a.pan_run[(gu0 + it.b0) * a.pan_pmax + it.panel];
  const int2 last = a.pan_run[(gu0 + it.b1 - 1) * a.pan_pmax + it.panel];
  const int vb = first.x, ve = last.x + last.y;
  const T* x = (const T*)a.V + tk.vec_off + vslot(a, j) * n + c0;
  for (int i = tid; i < len; i += NT) slice[i] = x[i];
  __syncthreads();
  const uint16_t* col = a.pan_col + tk.aux_off;
  const T* val = HAS_VAL ? (const T*)a.pan_val + tk.aux_off : nullptr;
  T* prod = (T*)a.pan_prod + tk.aux_off;
  // four entries per thread and load: groups of four from the 4-aligned entry at or below vb (the
  // realization's arrays are 8- and 16-byte aligned only when its arena offset is a multiple of 4, so
  // the vector accesses are used only then)
  if ((tk.aux_off & 3) == 0) {
    const int g0 = vb >> 2, g1 = (ve + 3) >> 2;
    const uint64_t* col4 = (const uint64_t*)col;
    for (int q0 = g0 + tid; q0 < g1; q0 += NT * U) {
      uint64_t c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * NT;
        c[u] = q < g1 ? __builtin_nontemporal_load(col4 + q) : (uint64_t)0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * NT;
        if (q >= g1) continue;
        const uint16_t cc[4] = {(uint16_t)c[u], (uint16_t)(c[u] >> 16), (uint16_t)(c[u] >> 32),
                                (uint16_t)(c[u] >> 48)};
        if (4 * q >= vb && 4 * q + 4 <= ve) {  // a whole group: one vector store per lane
          typedef T T4 __attribute__((ext_vector_type(4)));
          T4 pr;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const T xv = slice[cc[i]];
            if constexpr (HAS_VAL) pr[i] = val[4 * q + i] * xv; else pr[i] = xv;
          }
          __builtin_nontemporal_store(pr, (T4*)(prod + 4 * q));
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int v = 4 * q + i;
            if (v < vb || v >= ve) continue;
            const T xv = slice[cc[i]];
            T pr;
            if constexpr (HAS_VAL) pr = val[v] * xv; else pr = xv;
            __builtin_nontemporal_store(pr, prod + v);
          }
        }
      }
    }
    return;
  }
  for (int v0 = vb + tid; v0 < ve; v0 += NT * U) {
    uint16_t c[U];
    T w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int v = v0 + u * NT;
      c[u] = v < ve ? __builtin_nontemporal_load(col + v) : (uint16_t)0;
      if constexpr (HAS_VAL) w[u] = v < ve ? __builtin_nontemporal_load(val + v) : (T)0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int v = v0 + u * NT;
      if (v < ve) {
        const T xv = slice[c[u]];
        T pr;
        if constexpr (HAS_VAL) pr = w[u] * xv; else pr = xv;
        __builtin_nontemporal_store(pr, prod + v);
      }
    }
  }
}

template <typename T, bool HAS_VAL>
__global__ __launch_bounds__(kPanRowThreads) void k_pan_rows(LzArgs a, int j) {
  if (all_stopped(a, j)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NT = kPanRowThreads, U = 16;
  T* pl = (T*)smem;  // the unit's products in CSR order
  const size_t prod_bytes = (pan_rows_lds<T>(a.pan_lds, a.pan_pmax) - (size_t)(2 * a.pan_pmax + 2) * sizeof(int));
  int* pre = (int*)(smem + prod_bytes);  // [P + 1] first flattened entry of each run
  int* rx = pre + a.pan_pmax + 1;        // [P] each run's first entry
  __shared__ int rp_lds[kPanMaxUnit + 1];
  __shared__ double red[NT / 64];
  __shared__ int wtot[NT / 64];
  const PanRef ref = pan_ref(a);
  const Task tk = a.tasks[ref.task];
  RState* st = a.state + ref.task;
  const int n = tk.n, Ur = a.pan_unit, r0 = ref.u * Ur, rows = min(n - r0, Ur), tid = threadIdx.x;
  if (rows <= 0 || step_skipped(a, st, j)) return;
  const double sj = st->s[j];  // recorded by the products pass (st->s[0] at step 0)
  const int32_t* rp = a.row_ptr + tk.rowptr_off;
  T* w = (T*)a.W + tk.w_off + r0;
  if (!a.pan_flag[ref.gu]) {  // the CSR-stream arithmetic, gathering from the vector in memory
    const T* va = HAS_VAL ? (const T*)a.values + tk.nnz_off : nullptr;
    spmv_stream_rows<T, HAS_VAL, NT, StreamShape<T>::CAP, false, false, true, kBlock>(
        rp, a.col_idx + tk.nnz_off, va, (const T*)a.V + tk.vec_off + vslot(a, j) * n, r0, rows, sj, rp_lds, pl, w,
        red);
    return;
  }
  const int S = a.pan_cols, P = (n + S - 1) / S;
  const int2* run = a.pan_run + ref.gu * a.pan_pmax;
  for (int i = tid; i <= rows; i += NT) rp_lds[i] = rp[r0 + i];
  int carry = 0;
  for (int p0 = 0; p0 < P; p0 += NT) {
    const int p = p0 + tid;
    const int2 rv = p < P ? run[p] : make_int2(0, 0);
    int total = 0;
    const int ex = block_excl_scan<NT>(rv.y, wtot, &total);
    if (p < P) {
      pre[p] = carry + ex;
      rx[p] = rv.x;
    }
    carry += total;
  }
  if (tid == 0) pre[P] = carry;
  __syncthreads();
  const int e0 = rp_lds[0], total = carry;
  const uint16_t* perm = a.pan_perm + tk.aux_off;
  const T* prod = (const T*)a.pan_prod + tk.aux_off;
  int top = 1;  // the largest power of two below P: the search's first stride
  while (top * 2 < P) top *= 2;
  for (int v0 = tid; v0 < total; v0 += NT * U) {
    // the last run starting at or before each entry, by a search of fixed length (the U searches
    // interleave their LDS reads)
    int lo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) lo[u] = 0;
    for (int stride = P > 1 ? top : 0; stride > 0; stride >>= 1) {
      // unconditional reads (index clamped) and a select: the U reads issue back to back
      int pv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) pv[u] = pre[min(lo[u] + stride, P - 1)];
#pragma unroll
      for (int u = 0; u < U; ++u) lo[u] = (lo[u] + stride < P && pv[u] <= v0 + u * NT) ? lo[u] + stride : lo[u];
    }
    uint16_t q[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int f = v0 + u * NT;
      const int pos = rx[lo[u]] + (f - pre[lo[u]]);
      q[u] = f < total ? __builtin_nontemporal_load(perm + pos) : (uint16_t)0;
      v[u] = f < total ? __builtin_nontemporal_load(prod + pos) : (T)0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (v0 + u * NT < total) pl[q[u]] = v[u];
  }
  __syncthreads();
  for (int r = tid; r < rows; r += NT) {
    double acc = 0.0;
    int k = rp_lds[r] - e0;
    const int k1 = rp_lds[r + 1] - e0;
    for (; k + U <= k1; k += U) {
      T t[U];
#pragma unroll
      for (int u = 0; u < U; ++u) t[u] = pl[k + u];
#pragma unroll
      for (int u = 0; u < U; ++u) acc += (double)t[u];
    }
    for (; k < k1; ++k) acc += (double)pl[k];
    w[r] = (T)(acc * sj);
  }
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
  if (a.pan_cols > 0) {
    hipLaunchKernelGGL((k_pan_products<T, HAS_VAL>), dim3((unsigned)a.pan_nitems), dim3(kPanProdThreads),
                       (size_t)a.pan_cols * sizeof(T), s, a, j);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_pan_rows<T, HAS_VAL>), dim3((unsigned)(nb * (kRowsPerBlock / a.pan_unit))),
                       dim3(kPanRowThreads), pan_rows_lds<T>(a.pan_lds, a.pan_pmax), s, a, j);
    return hipGetLastError();
  }
  if (a.bal != nullptr) {
    if (j == 0 && a.unit_start)
      hipLaunchKernelGGL((k_spmv_bal<T, HAS_VAL, true>), dim3((unsigned)a.nbal), dim3(kBlock), 0, s, a, j);
    else
      hipLaunchKernelGGL((k_spmv_bal<T, HAS_VAL, false>), dim3((unsigned)a.nbal), dim3(kBlock), 0, s, a, j);
    return hipGetLastError();
  }
  if (a.seg_cols > 0) {
    const size_t dyn = 2 * (size_t)a.seg_cols * sizeof(T);
    if constexpr (sizeof(T) == 4) {
      if (a.seg_vec)
        hipLaunchKernelGGL((k_spmv_seg4<HAS_VAL, true>), dim3((unsigned)nb), dim3(kSegThreads), dyn, s, a, j);
      else
        hipLaunchKernelGGL((k_spmv_seg4<HAS_VAL, false>), dim3((unsigned)nb), dim3(kSegThreads), dyn, s, a, j);
    } else {
      if (a.seg_vec)
        hipLaunchKernelGGL((k_spmv_seg<T, HAS_VAL, true>), dim3((unsigned)nb), dim3(kSegThreads), dyn, s, a, j);
      else
        hipLaunchKernelGGL((k_spmv_seg<T, HAS_VAL, false>), dim3((unsigned)nb), dim3(kSegThreads), dyn, s, a, j);
    }
    return hipGetLastError();
  }
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

namespace {

template <typename T>
hipError_t prepare_seg_t() {
  const size_t dyn = kLdsBytes - seg_static_bytes<T>();
  const size_t dyn_prep = kLdsBytes - kSegPrepStatic;
  hipError_t e = hipSuccess;
  if constexpr (sizeof(T) == 4) {
    e = allow_lds(k_spmv_seg4<true, true>, dyn);
    if (e == hipSuccess) e = allow_lds(k_spmv_seg4<false, true>, dyn);
    if (e == hipSuccess) e = allow_lds(k_spmv_seg4<true, false>, dyn);
    if (e == hipSuccess) e = allow_lds(k_spmv_seg4<false, false>, dyn);
  } else {
    e = allow_lds(k_spmv_seg<T, true, true>, dyn);
    if (e == hipSuccess) e = allow_lds(k_spmv_seg<T, false, true>, dyn);
    if (e == hipSuccess) e = allow_lds(k_spmv_seg<T, true, false>, dyn);
    if (e == hipSuccess) e = allow_lds(k_spmv_seg<T, false, false>, dyn);
  }
  if (e == hipSuccess) e = allow_lds(k_seg_prepare<T, true>, dyn_prep);
  if (e == hipSuccess) e = allow_lds(k_seg_prepare<T, false>, dyn_prep);
  return e;
}

template <typename T, bool HAS_VAL>
hipError_t seg_prepare_t(const LzArgs& a, int64_t nb, int smax, hipStream_t s) {
  if (a.seg_stride != smax * kRowsPerBlock) return hipErrorInvalidValue;
  const int cap = seg_prepare_cap<T, HAS_VAL>(smax);
  if (cap < 256) return hipErrorInvalidValue;
  const size_t dyn = ((size_t)smax * kRowsPerBlock * 2 + 15) / 16 * 16 + (size_t)cap * (4 + (HAS_VAL ? sizeof(T) : 0));
  hipLaunchKernelGGL((k_seg_prepare<T, HAS_VAL>), dim3((unsigned)nb), dim3(kSegThreads), dyn, s, a, cap);
  return hipGetLastError();
}

}  // namespace

hipError_t prepare_seg_kernels() {
  static hipError_t e = [] {
    hipError_t r = prepare_seg_t<float>();
    if (r == hipSuccess) r = prepare_seg_t<double>();
    return r;
  }();
  return e;
}

int seg_max_cols(int dtype) {
  return dtype == EBTC_F64 ? SegShape<double>::MAXCOLS : SegShape<float>::MAXCOLS;
}

namespace {

template <typename T>
hipError_t prepare_pan_t() {
  hipError_t e = allow_lds(k_pan_products<T, true>, PanShape<T>::MAXCOLS * sizeof(T));
  if (e == hipSuccess) e = allow_lds(k_pan_products<T, false>, PanShape<T>::MAXCOLS * sizeof(T));
  const size_t rows_max = pan_rows_lds<T>(pan_max_lds(sizeof(T) == 8 ? EBTC_F64 : EBTC_F32), kPanMaxPanels);
  if (e == hipSuccess) e = allow_lds(k_pan_rows<T, true>, rows_max);
  if (e == hipSuccess) e = allow_lds(k_pan_rows<T, false>, rows_max);
  return e;
}

}  // namespace

hipError_t prepare_pan_kernels() {
  static hipError_t e = [] {
    hipError_t r = prepare_pan_t<float>();
    if (r == hipSuccess) r = prepare_pan_t<double>();
    return r;
  }();
  return e;
}

int pan_max_cols(int dtype) { return dtype == EBTC_F64 ? PanShape<double>::MAXCOLS : PanShape<float>::MAXCOLS; }

int pan_max_lds(int dtype) { return (int)(kPanCapBytes / (dtype == EBTC_F64 ? 8 : 4)); }

int stream_cap(int dtype) { return dtype == EBTC_F64 ? StreamShape<double>::CAP : StreamShape<float>::CAP; }

hipError_t launch_pan_prepare(int dtype, bool has_val, const LzArgs& a, int64_t nb, const PanItem* groups,
                              int ngroups, hipStream_t s) {
  if (a.pan_cols <= 0 || a.pan_cols > pan_max_cols(dtype) || a.pan_pmax < 1 || a.pan_pmax > kPanMaxPanels ||
      (a.pan_unit != 64 && a.pan_unit != 128 && a.pan_unit != 256) || a.pan_lds < 1 || a.pan_lds > pan_max_lds(dtype) ||
      a.pan_lds > 65536)
    return hipErrorInvalidValue;
  const dim3 g((unsigned)(nb * (kRowsPerBlock / a.pan_unit))), b(kPanPrepThreads);
  if (dtype == EBTC_F64) hipLaunchKernelGGL((k_pan_count<double>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_pan_count<float>), g, b, 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ngroups > 0) {
    hipLaunchKernelGGL(k_pan_scan, dim3((unsigned)ngroups), dim3(kPanScanThreads), 0, s, a, groups);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (dtype == EBTC_F64) {
    if (has_val) hipLaunchKernelGGL((k_pan_place<double, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_pan_place<double, false>), g, b, 0, s, a);
  } else {
    if (has_val) hipLaunchKernelGGL((k_pan_place<float, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_pan_place<float, false>), g, b, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_bal_rows(const LzArgs& a, int t0, int count, hipStream_t s) {
  if (a.bal == nullptr || count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bal_rows, dim3((unsigned)count), dim3(kBlock), 0, s, a, t0);
  return hipGetLastError();
}

hipError_t launch_seg_prepare(int dtype, bool has_val, const LzArgs& a, int64_t nb, int smax, hipStream_t s) {
  if (smax < 1 || smax > kSegMax || a.seg_cols <= 0) return hipErrorInvalidValue;
  if (dtype == EBTC_F64)
    return has_val ? seg_prepare_t<double, true>(a, nb, smax, s) : seg_prepare_t<double, false>(a, nb, smax, s);
  return has_val ? seg_prepare_t<float, true>(a, nb, smax, s) : seg_prepare_t<float, false>(a, nb, smax, s);
}

int staged_max_seglen(int dtype) {
  return dtype == EBTC_F64 ? (int)((kLdsBytes - staged_static_bytes<double>()) / 8)
                           : (int)((kLdsBytes - staged_static_bytes<float>()) / 4);
}

hipError_t launch_spmv_step(int dtype, bool has_val, int lanes, int j, const LzArgs& a, int64_t nb, hipStream_t s) {
  // the first product: row sums (degrees for a pattern-only graph, from the row pointers alone); the
  // balanced form sums weighted rows itself, in equal shares of entries
  if (j == 0 && a.unit_start && (a.bal == nullptr || !has_val)) {
    const dim3 g((unsigned)nb), b(first_threads(has_val));
    if (dtype == EBTC_F64) {
      if (has_val) hipLaunchKernelGGL((k_spmv_first<double, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_spmv_first<double, false>), g, b, 0, s, a);
    } else {
      if (has_val) hipLaunchKernelGGL((k_spmv_first<float, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_spmv_first<float, false>), g, b, 0, s, a);
    }
    return hipGetLastError();
  }
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
