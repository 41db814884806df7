// Realization generator for gfx950: background graphs drawn on the device (G(n, p), Watts-Strogatz,
// Barabasi-Albert), the target pattern embedded, written as the batch's symmetric CSR.
//
// One ebtc_generate_count call (count realizations of one spec):
//   1. candidates: a thread per row (G(n, p): geometric skips, run twice -- count, scan, write) or per
//      lattice / attachment edge (WS, BA) writes the 64-bit key (r, min, max) of every drawn edge;
//      an edge with both ends among the target nodes becomes the invalid key; the pattern's edges
//      are appended;
//   2. radix sort over the bits the keys use, unique compaction (repeats and invalid keys dropped),
//      per-row degrees (integer atomics: the counts do not depend on their order), exclusive scan
//      into the row pointers (the scan and the sort are this file's own kernels, below);
//   3. both directions of every edge, radix-sorted: the CSR entries in order (rows ascending,
//      columns ascending within a row).
// ebtc_generate_fill scatters the sorted entries' columns to the caller's col_idx. Every random
// draw is a Philox4x32-10 block of its own counter, so the result is a function of the spec alone.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace ebtc {
namespace {

constexpr uint32_t kTagER = 1, kTagWS = 2, kTagBA = 3;
constexpr uint64_t kInvalidKey = ~0ull;
constexpr int kGenBlock = 256;
// workspace header (int64 words)
constexpr int kHdrCandidates = 0, kHdrOverflow = 1, kHdrUnique = 2, kHdrWords = 32;

struct GenArgs {
  int32_t n, k, count, pe;
  double p;
  uint64_t thr;          // WS: rewired iff w0 < thr = floor(beta 2^32)
  uint32_t k0, k1;       // Philox key
  int64_t first;         // realization index of the call's first realization
  int64_t per;           // WS / BA: candidate edges per realization
  const uint8_t* inside; // [n] target membership, or nullptr
};

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds, each two 32 x 32 -> 64-bit
// products mixed into the other two words with the round key; the key gains the Weyl increments
// between rounds.
__device__ inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                     uint32_t out[4]) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t x0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t x2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = x0;
    c1 = (uint32_t)p1;
    c2 = x2;
    c3 = (uint32_t)p0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// Natural logarithm from correctly rounded operations only, in a fixed order, no fused multiply-add:
// x = m 2^e with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s), s = (m - 1) / (m + 1), the atanh
// series in s^2 (terms up to s^21 / 21) by Horner, then e ln 2 + (2 s) q. Any IEEE double evaluation
// of these operations gives these bits, which makes the geometric skips reproducible off the device.
__device__ inline double exact_log(double x) {
#pragma clang fp contract(off)
  constexpr double kSqrtHalf = 0.70710678118654752440;
  constexpr double kLn2 = 0.69314718055994530942;
  constexpr double c[11] = {1.0,      1.0 / 3,  1.0 / 5,  1.0 / 7,  1.0 / 9, 1.0 / 11,
                            1.0 / 13, 1.0 / 15, 1.0 / 17, 1.0 / 19, 1.0 / 21};
  int e = 0;
  double m = frexp(x, &e);
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double q = c[10];
#pragma unroll
  for (int k = 9; k >= 0; --k) {
    q = q * z;
    q = q + c[k];
  }
  const double el = (double)e * kLn2;
  const double s2 = 2.0 * s;
  return el + s2 * q;
}

__device__ inline int64_t gtid() { return (int64_t)blockIdx.x * kGenBlock + threadIdx.x; }

__device__ inline uint64_t edge_key(const GenArgs& a, int rl, int x, int y) {
  if (a.inside && a.inside[x] && a.inside[y]) return kInvalidKey;
  const int lo = min(x, y), hi = max(x, y);
  return ((uint64_t)rl * (uint64_t)a.n + (uint64_t)lo) * (uint64_t)a.n + (uint64_t)hi;
}

// G(n, p), row i of realization rl: columns j > i by geometric skips. WRITE = false counts the row's
// edges into cnt; WRITE = true writes their keys from off[row] on (positions >= cap are dropped: the
// call reports the overflow).
template <bool WRITE>
__global__ __launch_bounds__(kGenBlock) void k_er_rows(GenArgs a, int32_t* cnt, const int64_t* off, uint64_t* keys,
                                                       int64_t cap) {
  const int64_t t = gtid();
  if (t >= (int64_t)a.count * a.n) return;
  const int n = a.n;
  const int rl = (int)(t / n);
  const int i = (int)(t - (int64_t)rl * n);
  const int64_t base = WRITE ? off[t] : 0;
  int32_t c = 0;
  auto emit = [&](int j) {
    if (WRITE && base + c < cap) keys[base + c] = edge_key(a, rl, i, j);
    ++c;
  };
  if (a.p >= 1.0) {
    for (int j = i + 1; j < n; ++j) emit(j);
  } else if (a.p > 0.0 && 1.0 - a.p != 1.0 && i < n - 1) {
    const double q = exact_log(1.0 - a.p);
    const uint32_t ridx = (uint32_t)(a.first + rl);
    int64_t j = i;
    bool more = true;
    for (uint32_t call = 0; more; ++call) {
      uint32_t w[4];
      philox4x32_10((uint32_t)i, call, ridx, kTagER, a.k0, a.k1, w);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        if (more) {
          const double u = ((double)w[h] + 0.5) * 0x1p-32;
          const double g = floor(exact_log(u) / q);
          if (g < (double)(n - 1 - j)) {
            j += 1 + (int64_t)g;
            emit((int)j);
          } else {
            more = false;
          }
        }
      }
    }
  }
  if (!WRITE) cnt[t] = c;
}

// Total G(n, p) candidates and the overflow flag (one thread).
__global__ void k_er_total(const int32_t* cnt, const int64_t* off, int64_t rows, int64_t cap, int64_t* hdr) {
  const int64_t total = rows > 0 ? off[rows - 1] + cnt[rows - 1] : 0;
  hdr[kHdrCandidates] = total;
  hdr[kHdrOverflow] = total > cap ? 1 : 0;
}

// Invalid keys in the unused tail [total, cap) of the G(n, p) candidate region.
__global__ __launch_bounds__(kGenBlock) void k_er_tail(const int64_t* hdr, uint64_t* keys, int64_t cap) {
  const int64_t t = gtid();
  if (t < cap && t >= hdr[kHdrCandidates]) keys[t] = kInvalidKey;
}

// Watts-Strogatz: lattice edge e of realization rl, rewired or kept.
__global__ __launch_bounds__(kGenBlock) void k_ws_edges(GenArgs a, uint64_t* keys) {
  const int64_t t = gtid();
  if (t >= (int64_t)a.count * a.per) return;
  const int rl = (int)(t / a.per);
  const int64_t e = t - (int64_t)rl * a.per;
  const int h = a.k / 2, n = a.n;
  const int i = (int)(e / h);
  const int far = (int)((i + 1 + e % h) % n);
  uint32_t w[4];
  philox4x32_10((uint32_t)e, 0u, (uint32_t)(a.first + rl), kTagWS, a.k0, a.k1, w);
  const int nv = (int)((i + 1 + (int64_t)(((uint64_t)w[1] * (uint64_t)(n - 1)) >> 32)) % n);
  keys[t] = edge_key(a, rl, i, (uint64_t)w[0] < a.thr ? nv : far);
}

// Barabasi-Albert: the node that brings edge e (seed star: leaf e + 1).
__device__ inline int ba_new_node(int m, int64_t e) { return e < m ? (int)(e + 1) : (int)(m + 1 + (e - m) / m); }

// Endpoint slot drawn by edge e >= m: floor(X * 2E_u / 2^64), X = w0 2^32 + w1, E_u edges before it.
__device__ inline int64_t ba_slot(const GenArgs& a, uint32_t ridx, int64_t e) {
  const int m = a.k;
  const int64_t eb = m + (int64_t)(ba_new_node(m, e) - m - 1) * m;
  uint32_t w[4];
  philox4x32_10((uint32_t)e, 0u, ridx, kTagBA, a.k0, a.k1, w);
  const uint64_t R = 2 * (uint64_t)eb;
  const uint64_t lo = ((uint64_t)w[1] * R) >> 32;
  return (int64_t)(((uint64_t)w[0] * R + lo) >> 32);
}

// Barabasi-Albert edge e of realization rl: its node and the endpoint found by following odd slots
// (the attached end of an earlier edge) back to an even slot (a new node) or the seed's centre. Each
// hop moves to a strictly earlier edge, so the walk ends.
__global__ __launch_bounds__(kGenBlock) void k_ba_edges(GenArgs a, uint64_t* keys) {
  const int64_t t = gtid();
  if (t >= (int64_t)a.count * a.per) return;
  const int rl = (int)(t / a.per);
  const int64_t e = t - (int64_t)rl * a.per;
  const int m = a.k;
  const uint32_t ridx = (uint32_t)(a.first + rl);
  int end = 0;
  if (e >= m) {
    int64_t s = ba_slot(a, ridx, e);
    for (;;) {
      const int64_t f = s >> 1;
      if ((s & 1) == 0) {
        end = ba_new_node(m, f);
        break;
      }
      if (f < m) {
        end = 0;
        break;
      }
      s = ba_slot(a, ridx, f);
    }
  }
  keys[t] = edge_key(a, rl, ba_new_node(m, e), end);
}

// Target membership flags.
__global__ __launch_bounds__(kGenBlock) void k_zero_u8(uint8_t* x, int64_t len) {
  const int64_t t = gtid();
  if (t < len) x[t] = 0;
}
__global__ void k_mark(const int32_t* targets, int t, uint8_t* inside) {
  for (int q = threadIdx.x; q < t; q += blockDim.x) inside[targets[q]] = 1;
}
__global__ __launch_bounds__(kGenBlock) void k_zero_i64(int64_t* x, int64_t len) {
  const int64_t t = gtid();
  if (t < len) x[t] = 0;
}
__global__ __launch_bounds__(kGenBlock) void k_zero_i32(int32_t* x, int64_t len) {
  const int64_t t = gtid();
  if (t < len) x[t] = 0;
}

// The pattern's edges in every realization of the call (never filtered).
__global__ __launch_bounds__(kGenBlock) void k_pattern(int n, int count, int pe, const int32_t* targets,
                                                       const int32_t* pattern, uint64_t* keys) {
  const int64_t t = gtid();
  if (t >= (int64_t)count * pe) return;
  const int rl = (int)(t / pe), q = (int)(t - (int64_t)rl * pe);
  const int x = targets[pattern[2 * q]], y = targets[pattern[2 * q + 1]];
  keys[t] = ((uint64_t)rl * (uint64_t)n + (uint64_t)min(x, y)) * (uint64_t)n + (uint64_t)max(x, y);
}

__global__ __launch_bounds__(kGenBlock) void k_unique_flags(const uint64_t* sorted, int64_t size, uint64_t limit,
                                                            int32_t* flags) {
  const int64_t t = gtid();
  if (t >= size) return;
  const uint64_t k = sorted[t];
  flags[t] = (k < limit && (t == 0 || sorted[t - 1] != k)) ? 1 : 0;
}

__global__ __launch_bounds__(kGenBlock) void k_unique_scatter(const uint64_t* sorted, const int32_t* flags,
                                                              const int64_t* pos, int64_t size, uint64_t* uniq,
                                                              int64_t* hdr) {
  const int64_t t = gtid();
  if (t >= size) return;
  if (flags[t]) uniq[pos[t]] = sorted[t];
  if (t == size - 1) hdr[kHdrUnique] = pos[t] + flags[t];
}

__global__ __launch_bounds__(kGenBlock) void k_degrees(const uint64_t* uniq, const int64_t* hdr, int64_t cap, int n,
                                                       int32_t* deg) {
  const int64_t t = gtid();
  if (t >= cap || t >= hdr[kHdrUnique]) return;
  const uint64_t nn = (uint64_t)n * (uint64_t)n, key = uniq[t];
  const int64_t rl = (int64_t)(key / nn);
  const uint64_t rem = key - (uint64_t)rl * nn;
  const int x = (int)(rem / (uint64_t)n), y = (int)(rem % (uint64_t)n);
  atomicAdd(&deg[rl * n + x], 1);
  atomicAdd(&deg[rl * n + y], 1);
}

// Local row pointers of every realization from the exclusive scan S of the concatenated degrees,
// its entry count (or -1), and whether the fill may write it.
__global__ __launch_bounds__(kGenBlock) void k_row_ptr(const int32_t* deg, const int64_t* S, int n, int count,
                                                       const int64_t* hdr, int32_t* row_ptr, int64_t* nnz,
                                                       int32_t* ok) {
  const int64_t t = gtid();
  if (t >= (int64_t)count * (n + 1)) return;
  const int rl = (int)(t / (n + 1)), i = (int)(t - (int64_t)rl * (n + 1));
  const int64_t r0 = (int64_t)rl * n;
  const int64_t v = i < n ? S[r0 + i] - S[r0] : S[r0 + n - 1] + deg[r0 + n - 1] - S[r0];
  row_ptr[t] = v < 2147483648LL ? (int32_t)v : 0;
  if (i == n) {
    const bool good = hdr[kHdrOverflow] == 0 && v < 2147483648LL;
    nnz[rl] = good ? v : -1;
    ok[rl] = good ? 1 : 0;
  }
}

// Both directions of every unique edge; invalid keys beyond 2U.
__global__ __launch_bounds__(kGenBlock) void k_directed(const uint64_t* uniq, const int64_t* hdr, int64_t cap, int n,
                                                        uint64_t* dir) {
  const int64_t t = gtid();
  if (t >= cap) return;
  if (t >= hdr[kHdrUnique]) {
    dir[2 * t] = kInvalidKey;
    dir[2 * t + 1] = kInvalidKey;
    return;
  }
  const uint64_t nn = (uint64_t)n * (uint64_t)n, key = uniq[t];
  const uint64_t rl = key / nn;
  const uint64_t rem = key - rl * nn;
  const uint64_t x = rem / (uint64_t)n, y = rem % (uint64_t)n;
  dir[2 * t] = key;
  dir[2 * t + 1] = rl * nn + y * (uint64_t)n + x;
}

__global__ __launch_bounds__(kGenBlock) void k_scatter_cols(const uint64_t* dir_sorted, const int64_t* hdr,
                                                            int64_t size, int n, const int64_t* S, const int64_t* dest,
                                                            const int32_t* ok, int32_t* col_idx) {
  const int64_t t = gtid();
  if (t >= size || t >= 2 * hdr[kHdrUnique]) return;
  const uint64_t nn = (uint64_t)n * (uint64_t)n, key = dir_sorted[t];
  const int64_t rl = (int64_t)(key / nn);
  if (!ok[rl]) return;
  col_idx[dest[rl] + (t - S[rl * n])] = (int32_t)(key % (uint64_t)n);
}

// ------------------------------------------------------------------------- scan and radix sort
// A device-wide exclusive scan of 32-bit counts into 64-bit offsets (tile sums, their scan in one
// workgroup, each tile scanned from its offset), and an LSD radix sort of 64-bit keys: one pass per
// 8-bit digit of the bits the keys use, each a per-tile digit histogram, a scan of the counts in
// (digit, tile) order and a scatter. Every pass is stable, as an LSD sort needs: a tile's keys are
// ranked in index order, within a wave by ballots over the digit's bits, then wave after wave and
// round after round, so keys of one digit leave a tile in the order they came.
constexpr int kScanThreads = 1024, kScanItems = 8, kScanTile = kScanThreads * kScanItems;
constexpr int kSortThreads = 1024, kSortRounds = 4, kSortTile = kSortThreads * kSortRounds, kRadix = 256;

// Exclusive prefix sum of one int64 per thread over a workgroup of NT threads; *total = the sum of
// all. wtot: NT / 64 words. Ends with a barrier, so wtot may be reused.
template <int NT>
__device__ inline int64_t block_excl_scan64(int64_t v, int64_t* wtot, int64_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wtot[w] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int i = 0; i < NT / 64; ++i) {
    const int64_t t = wtot[i];
    before += i < w ? t : 0;
    all += t;
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

// tsum[b] = the sum of tile b (kScanTile values)
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int32_t* in, int64_t n, int64_t* tsum) {
  __shared__ int64_t wtot[kScanThreads / 64];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
  int64_t v = 0;
  for (int u = 0; u < kScanItems; ++u) {
    const int64_t i = t0 + (int64_t)u * kScanThreads + threadIdx.x;
    if (i < n) v += in[i];
  }
  int64_t total;
  block_excl_scan64<kScanThreads>(v, wtot, &total);
  if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

// the tile sums' exclusive scan in place: one workgroup, kScanThreads sums at a time with a carry
__global__ __launch_bounds__(kScanThreads) void k_scan_carry(int64_t* tsum, int64_t nt) {
  __shared__ int64_t wtot[kScanThreads / 64];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nt; c0 += kScanThreads) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < nt ? tsum[i] : 0;
    int64_t total;
    const int64_t ex = block_excl_scan64<kScanThreads>(v, wtot, &total);
    if (i < nt) tsum[i] = carry + ex;
    carry += total;
  }
}

// out[i] = tile offset + the sum of the tile's values before i; thread t takes kScanItems adjacent
// values of its tile
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t* in, int64_t* out, int64_t n,
                                                             const int64_t* tsum) {
  __shared__ int64_t wtot[kScanThreads / 64];
  const int64_t b = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int64_t sum = 0;
#pragma unroll
  for (int u = 0; u < kScanItems; ++u) {
    v[u] = b + u < n ? in[b + u] : 0;
    sum += v[u];
  }
  int64_t total;
  int64_t run = tsum[blockIdx.x] + block_excl_scan64<kScanThreads>(sum, wtot, &total);
#pragma unroll
  for (int u = 0; u < kScanItems; ++u) {
    if (b + u < n) out[b + u] = run;
    run += v[u];
  }
}

// cnt[d * nt + b] = keys of tile b whose digit at `shift` is d
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* keys, int64_t n, int shift, int32_t* cnt,
                                                             int64_t nt) {
  __shared__ int h[kRadix];
  for (int d = threadIdx.x; d < kRadix; d += kSortThreads) h[d] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
  for (int u = 0; u < kSortRounds; ++u) {
    const int64_t i = t0 + (int64_t)u * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(int)((keys[i] >> shift) & (kRadix - 1))], 1);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kSortThreads) cnt[(int64_t)d * nt + blockIdx.x] = h[d];
}

// Stable scatter of tile b by the digit at `shift`: off[d * nt + b] = where tile b's first key of
// digit d goes (the scanned histogram). Each round takes kSortThreads consecutive keys.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t* in, uint64_t* out, int64_t n, int shift,
                                                                const int64_t* off, int64_t nt) {
  constexpr int NW = kSortThreads / 64;
  __shared__ int64_t base[kRadix];  // where the tile's next key of each digit goes
  __shared__ int wc[NW][kRadix];    // the round's counts per wave and digit, then their offsets
  __shared__ int tot[kRadix];       // the round's counts per digit
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int d = tid; d < kRadix; d += kSortThreads) base[d] = off[(int64_t)d * nt + blockIdx.x];
  const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
  const uint64_t below = (1ull << lane) - 1ull;  // the lanes before this one
  for (int u = 0; u < kSortRounds; ++u) {
    const int64_t i = t0 + (int64_t)u * kSortThreads + tid;
    const bool valid = i < n;
    const uint64_t key = valid ? in[i] : 0ull;
    const int d = (int)((key >> shift) & (kRadix - 1));
    uint64_t peers = __ballot(valid);  // the wave's lanes holding a key of the same digit
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1;
      const uint64_t m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    for (int x = lane; x < kRadix; x += 64) wc[w][x] = 0;
    __syncthreads();
    if (valid && rank == 0) wc[w][d] = __popcll(peers);
    __syncthreads();
    if (tid < kRadix) {
      int run = 0;
      for (int v = 0; v < NW; ++v) {
        const int c = wc[v][tid];
        wc[v][tid] = run;
        run += c;
      }
      tot[tid] = run;
    }
    __syncthreads();
    if (valid) out[base[d] + wc[w][d] + rank] = key;
    __syncthreads();
    if (tid < kRadix) base[tid] += tot[tid];
  }
}

// ------------------------------------------------------------------------------------ host side
size_t align_up(size_t x) { return (x + 255) / 256 * 256; }
unsigned grid(int64_t threads) { return (unsigned)((threads + kGenBlock - 1) / kGenBlock); }

int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }
int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }
size_t scan_tmp_bytes(int64_t n) { return align_up(sizeof(int64_t) * (size_t)std::max<int64_t>(1, scan_tiles(n))); }
// the alternate key buffer, the digit counts and their offsets, the offsets' scan
size_t sort_tmp_bytes(int64_t n) {
  const size_t nt = (size_t)std::max<int64_t>(1, sort_tiles(n));
  return align_up(sizeof(uint64_t) * (size_t)std::max<int64_t>(1, n)) + align_up(sizeof(int32_t) * kRadix * nt) +
         align_up(sizeof(int64_t) * kRadix * nt) + scan_tmp_bytes((int64_t)(kRadix * nt));
}

// out[i] = in[0] + ... + in[i - 1] for i < n (tmp: scan_tmp_bytes(n))
hipError_t scan_i32_i64(void* tmp, const int32_t* in, int64_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nt = scan_tiles(n);
  int64_t* tsum = (int64_t*)tmp;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kScanThreads), 0, s, in, n, tsum);
  hipLaunchKernelGGL(k_scan_carry, dim3(1), dim3(kScanThreads), 0, s, tsum, nt);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(kScanThreads), 0, s, in, out, n, (const int64_t*)tsum);
  return hipGetLastError();
}

// out = in sorted by bits [0, end_bit) of the keys, whole keys moved (tmp: sort_tmp_bytes(n)); in is
// not written
hipError_t radix_sort_u64(void* tmp, const uint64_t* in, uint64_t* out, int64_t n, int end_bit, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nt = sort_tiles(n);
  char* t = (char*)tmp;
  uint64_t* buf = (uint64_t*)t;
  t += align_up(sizeof(uint64_t) * (size_t)n);
  int32_t* cnt = (int32_t*)t;
  t += align_up(sizeof(int32_t) * kRadix * (size_t)nt);
  int64_t* off = (int64_t*)t;
  t += align_up(sizeof(int64_t) * kRadix * (size_t)nt);
  const int passes = std::max(1, (end_bit + 7) / 8);
  const uint64_t* src = in;
  for (int p = 0; p < passes; ++p) {
    uint64_t* dst = (passes - 1 - p) % 2 == 0 ? out : buf;  // the last pass writes out
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nt), dim3(kSortThreads), 0, s, src, n, 8 * p, cnt, nt);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = scan_i32_i64(t, cnt, off, kRadix * nt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nt), dim3(kSortThreads), 0, s, src, dst, n, 8 * p,
                       (const int64_t*)off, nt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    src = dst;
  }
  return hipSuccess;
}

struct GenPlan {
  int64_t rows = 0;        // count * n
  int64_t cap_bg = 0;      // background candidate slots
  int64_t cap = 0;         // + pattern edges of every realization
  uint64_t limit = 0;      // count n^2: every valid key is below it
  int end_bit = 1;
  size_t off_hdr = 0, off_inside = 0, off_host = 0, off_ok = 0, off_dest = 0, off_cnt = 0, off_S = 0, off_flags = 0,
         off_pos = 0, off_A = 0, off_Aout = 0, off_C = 0, off_Cout = 0, off_tmp = 0, tmp_bytes = 0, total = 0;
};

int check_spec(const ebtc_gen_spec* s) {
  if (!s) return report_error(EBTC_EINVAL, "spec is NULL");
  if (s->family < EBTC_GEN_ER || s->family > EBTC_GEN_BA) return report_error(EBTC_EINVAL, "unknown family");
  if (s->count < 1) return report_error(EBTC_EINVAL, "count must be >= 1");
  if (s->first < 0 || s->first + s->count > (int64_t(1) << 32))
    return report_error(EBTC_EINVAL, "realization indices must lie in [0, 2^32)");
  if (s->family == EBTC_GEN_ER) {
    if (s->n < 1) return report_error(EBTC_EINVAL, "G(n, p) needs n >= 1");
    if (!(s->p >= 0.0 && s->p <= 1.0)) return report_error(EBTC_EINVAL, "p must be in [0, 1]");
  } else if (s->family == EBTC_GEN_WS) {
    if (s->k < 2 || s->k % 2) return report_error(EBTC_EINVAL, "Watts-Strogatz needs an even k >= 2");
    if (s->n < s->k + 2) return report_error(EBTC_EINVAL, "Watts-Strogatz needs n >= k + 2");
    if (!(s->beta >= 0.0 && s->beta <= 1.0)) return report_error(EBTC_EINVAL, "beta must be in [0, 1]");
    if ((int64_t)s->n * (s->k / 2) >= (int64_t(1) << 32))
      return report_error(EBTC_ENOTSUPPORTED, "Watts-Strogatz needs n k / 2 < 2^32 lattice edges");
  } else {
    if (s->k < 1) return report_error(EBTC_EINVAL, "Barabasi-Albert needs k >= 1");
    if (s->n < s->k + 2) return report_error(EBTC_EINVAL, "Barabasi-Albert needs n >= k + 2");
    if (2 * ((int64_t)s->k + (int64_t)(s->n - s->k - 1) * s->k) >= (int64_t(1) << 32))
      return report_error(EBTC_ENOTSUPPORTED, "Barabasi-Albert needs fewer than 2^31 edges");
  }
  if (s->t < 0 || s->t > s->n) return report_error(EBTC_EINVAL, "t must be in [0, n]");
  if (s->pattern_edges < 0) return report_error(EBTC_EINVAL, "pattern_edges must be >= 0");
  if (s->t > 0 && !s->targets) return report_error(EBTC_EINVAL, "targets is NULL");
  if (s->pattern_edges > 0 && (!s->pattern || s->t < 2)) return report_error(EBTC_EINVAL, "pattern without targets");
  std::vector<char> seen((size_t)s->n, 0);
  for (int q = 0; q < s->t; ++q) {
    const int v = s->targets[q];
    if (v < 0 || v >= s->n) return report_error(EBTC_EINVAL, "target node out of range");
    if (seen[(size_t)v]) return report_error(EBTC_EINVAL, "repeated target node");
    seen[(size_t)v] = 1;
  }
  for (int q = 0; q < s->pattern_edges; ++q) {
    const int x = s->pattern[2 * q], y = s->pattern[2 * q + 1];
    if (x < 0 || y < 0 || x >= s->t || y >= s->t || x == y)
      return report_error(EBTC_EINVAL, "pattern edge ends must be distinct local ids in [0, t)");
  }
  const long double keys = (long double)s->count * (long double)s->n * (long double)s->n;
  if (keys >= 9.2e18L) return report_error(EBTC_ENOTSUPPORTED, "count n^2 must stay below 2^63: draw fewer realizations per call");
  return EBTC_OK;
}

int64_t background_slots(const ebtc_gen_spec* s) {
  const int64_t n = s->n;
  if (s->family == EBTC_GEN_WS) return n * (s->k / 2);
  if (s->family == EBTC_GEN_BA) return s->k + (n - s->k - 1) * (int64_t)s->k;
  const double pairs = 0.5 * (double)n * (double)(n - 1);
  if (s->p >= 1.0) return (int64_t)pairs;
  if (s->p <= 0.0 || 1.0 - s->p == 1.0) return 0;
  const double mu = s->p * pairs;
  return (int64_t)std::min(pairs, std::ceil(mu + 8.0 * std::sqrt(mu * (1.0 - s->p)) + 64.0));
}

int make_plan(const ebtc_gen_spec* s, GenPlan* P) {
  int rc = check_spec(s);
  if (rc) return rc;
  P->rows = (int64_t)s->count * s->n;
  P->cap_bg = background_slots(s) * s->count;
  P->cap = P->cap_bg + (int64_t)s->count * s->pattern_edges;
  P->limit = (uint64_t)s->count * (uint64_t)s->n * (uint64_t)s->n;
  P->end_bit = 64 - __builtin_clzll(P->limit | 1);
  const size_t cap = (size_t)std::max<int64_t>(P->cap, 1), rows = (size_t)std::max<int64_t>(P->rows, 1);
  const size_t need = std::max({sort_tmp_bytes((int64_t)cap), sort_tmp_bytes(2 * (int64_t)cap),
                                scan_tmp_bytes((int64_t)std::max(cap, rows))});
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  P->off_hdr = take(kHdrWords * sizeof(int64_t));
  P->off_inside = take((size_t)s->n);
  P->off_host = take(sizeof(int32_t) * ((size_t)s->t + 2 * (size_t)s->pattern_edges));
  P->off_ok = take(sizeof(int32_t) * (size_t)s->count);
  P->off_dest = take(sizeof(int64_t) * (size_t)s->count);
  P->off_cnt = take(sizeof(int32_t) * rows);
  P->off_S = take(sizeof(int64_t) * rows);
  P->off_flags = take(sizeof(int32_t) * cap);
  P->off_pos = take(sizeof(int64_t) * cap);
  P->off_A = take(sizeof(uint64_t) * cap);
  P->off_Aout = take(sizeof(uint64_t) * cap);
  P->off_C = take(sizeof(uint64_t) * 2 * cap);
  P->off_Cout = take(sizeof(uint64_t) * 2 * cap);
  P->tmp_bytes = need;
  P->off_tmp = take(need);
  P->total = off;
  return EBTC_OK;
}

GenArgs make_gen_args(const ebtc_gen_spec* s, const GenPlan& P, char* ws) {
  GenArgs a{};
  a.n = s->n;
  a.k = s->k;
  a.count = s->count;
  a.pe = s->pattern_edges;
  a.p = s->p;
  a.thr = (uint64_t)std::floor(s->beta * 4294967296.0);
  a.k0 = (uint32_t)(s->seed & 0xFFFFFFFFu);
  a.k1 = (uint32_t)(s->seed >> 32);
  a.first = s->first;
  a.per = s->count > 0 ? P.cap_bg / s->count : 0;
  a.inside = s->t > 0 ? (const uint8_t*)(ws + P.off_inside) : nullptr;
  return a;
}

#define GEN_HIP(call)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return report_error(EBTC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define GEN_LAUNCH(...)                                                                            \
  do {                                                                                             \
    hipLaunchKernelGGL(__VA_ARGS__);                                                               \
    GEN_HIP(hipGetLastError());                                                                    \
  } while (0)

}  // namespace
}  // namespace ebtc

using namespace ebtc;

extern "C" int ebtc_generate_plan(const ebtc_gen_spec* spec, size_t* ws_bytes) {
  if (!ws_bytes) return report_error(EBTC_EINVAL, "ws_bytes is NULL");
  GenPlan P;
  const int rc = make_plan(spec, &P);
  if (rc) return rc;
  *ws_bytes = P.total;
  return EBTC_OK;
}

extern "C" int ebtc_generate_count(const ebtc_gen_spec* spec, void* ws, size_t ws_bytes, int32_t* row_ptr,
                                   int64_t* nnz, void* stream) {
  GenPlan P;
  int rc = make_plan(spec, &P);
  if (rc) return rc;
  if (!ws || !row_ptr || !nnz) return report_error(EBTC_EINVAL, "NULL device pointer");
  if (ws_bytes < P.total) return report_error(EBTC_EWORKSPACE, "workspace smaller than ebtc_generate_plan reported");
  const hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  int64_t* hdr = (int64_t*)(w + P.off_hdr);
  int32_t* cnt = (int32_t*)(w + P.off_cnt);
  int64_t* S = (int64_t*)(w + P.off_S);
  int32_t* flags = (int32_t*)(w + P.off_flags);
  int64_t* pos = (int64_t*)(w + P.off_pos);
  uint64_t* A = (uint64_t*)(w + P.off_A);
  uint64_t* Aout = (uint64_t*)(w + P.off_Aout);
  uint64_t* C = (uint64_t*)(w + P.off_C);
  uint64_t* Cout = (uint64_t*)(w + P.off_Cout);
  void* tmp = w + P.off_tmp;
  const GenArgs a = make_gen_args(spec, P, w);
  const int n = spec->n;

  GEN_LAUNCH(k_zero_i64, dim3(1), dim3(kGenBlock), 0, s, hdr, (int64_t)kHdrWords);
  if (spec->t > 0) {
    // targets and pattern to the device (small; the host arrays may go away after the call)
    std::vector<int32_t> host((size_t)spec->t + 2 * (size_t)spec->pattern_edges);
    std::copy(spec->targets, spec->targets + spec->t, host.begin());
    if (spec->pattern_edges > 0)
      std::copy(spec->pattern, spec->pattern + 2 * spec->pattern_edges, host.begin() + spec->t);
    GEN_HIP(hipMemcpyAsync(w + P.off_host, host.data(), host.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    GEN_HIP(hipStreamSynchronize(s));
    GEN_LAUNCH(k_zero_u8, dim3(grid(n)), dim3(kGenBlock), 0, s, (uint8_t*)(w + P.off_inside), (int64_t)n);
    GEN_LAUNCH(k_mark, dim3(1), dim3(kGenBlock), 0, s, (const int32_t*)(w + P.off_host), spec->t,
               (uint8_t*)(w + P.off_inside));
  }
  if (spec->family == EBTC_GEN_ER) {
    GEN_LAUNCH(k_er_rows<false>, dim3(grid(P.rows)), dim3(kGenBlock), 0, s, a, cnt, (const int64_t*)nullptr,
               (uint64_t*)nullptr, (int64_t)0);
    GEN_HIP(scan_i32_i64(tmp, (const int32_t*)cnt, S, P.rows, s));
    GEN_LAUNCH(k_er_total, dim3(1), dim3(1), 0, s, (const int32_t*)cnt, (const int64_t*)S, P.rows, P.cap_bg, hdr);
    GEN_LAUNCH(k_er_rows<true>, dim3(grid(P.rows)), dim3(kGenBlock), 0, s, a, cnt, (const int64_t*)S, A, P.cap_bg);
    if (P.cap_bg > 0) GEN_LAUNCH(k_er_tail, dim3(grid(P.cap_bg)), dim3(kGenBlock), 0, s, (const int64_t*)hdr, A, P.cap_bg);
  } else if (spec->family == EBTC_GEN_WS) {
    GEN_LAUNCH(k_ws_edges, dim3(grid(P.cap_bg)), dim3(kGenBlock), 0, s, a, A);
  } else {
    GEN_LAUNCH(k_ba_edges, dim3(grid(P.cap_bg)), dim3(kGenBlock), 0, s, a, A);
  }
  if (spec->pattern_edges > 0) {
    const int32_t* tg = (const int32_t*)(w + P.off_host);
    GEN_LAUNCH(k_pattern, dim3(grid((int64_t)spec->count * spec->pattern_edges)), dim3(kGenBlock), 0, s, n,
               spec->count, spec->pattern_edges, tg, tg + spec->t, A + P.cap_bg);
  }
  const size_t cap = (size_t)P.cap;
  if (cap > 0) {
    GEN_HIP(radix_sort_u64(tmp, A, Aout, P.cap, P.end_bit, s));
    GEN_LAUNCH(k_unique_flags, dim3(grid(P.cap)), dim3(kGenBlock), 0, s, (const uint64_t*)Aout, P.cap, P.limit, flags);
    GEN_HIP(scan_i32_i64(tmp, (const int32_t*)flags, pos, P.cap, s));
    GEN_LAUNCH(k_unique_scatter, dim3(grid(P.cap)), dim3(kGenBlock), 0, s, (const uint64_t*)Aout,
               (const int32_t*)flags, (const int64_t*)pos, P.cap, A, hdr);
  }
  GEN_LAUNCH(k_zero_i32, dim3(grid(P.rows)), dim3(kGenBlock), 0, s, cnt, P.rows);
  if (cap > 0)
    GEN_LAUNCH(k_degrees, dim3(grid(P.cap)), dim3(kGenBlock), 0, s, (const uint64_t*)A, (const int64_t*)hdr, P.cap, n,
               cnt);
  GEN_HIP(scan_i32_i64(tmp, (const int32_t*)cnt, S, P.rows, s));
  GEN_LAUNCH(k_row_ptr, dim3(grid((int64_t)spec->count * (n + 1))), dim3(kGenBlock), 0, s, (const int32_t*)cnt,
             (const int64_t*)S, n, spec->count, (const int64_t*)hdr, row_ptr, nnz, (int32_t*)(w + P.off_ok));
  if (cap > 0) {
    GEN_LAUNCH(k_directed, dim3(grid(P.cap)), dim3(kGenBlock), 0, s, (const uint64_t*)A, (const int64_t*)hdr, P.cap,
               n, C);
    GEN_HIP(radix_sort_u64(tmp, C, Cout, 2 * P.cap, P.end_bit, s));
  }
  return EBTC_OK;
}

extern "C" int ebtc_generate_fill(const ebtc_gen_spec* spec, void* ws, size_t ws_bytes, const int64_t* dest_off,
                                  int32_t* col_idx, void* stream) {
  GenPlan P;
  int rc = make_plan(spec, &P);
  if (rc) return rc;
  if (!ws || !dest_off || !col_idx) return report_error(EBTC_EINVAL, "NULL pointer");
  if (ws_bytes < P.total) return report_error(EBTC_EWORKSPACE, "workspace smaller than ebtc_generate_plan reported");
  for (int r = 0; r < spec->count; ++r)
    if (dest_off[r] < 0) return report_error(EBTC_EINVAL, "dest_off must be >= 0");
  if (P.cap == 0) return EBTC_OK;
  const hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  GEN_HIP(hipMemcpyAsync(w + P.off_dest, dest_off, sizeof(int64_t) * (size_t)spec->count, hipMemcpyHostToDevice, s));
  GEN_HIP(hipStreamSynchronize(s));
  GEN_LAUNCH(k_scatter_cols, dim3(grid(2 * P.cap)), dim3(kGenBlock), 0, s, (const uint64_t*)(w + P.off_Cout),
             (const int64_t*)(w + P.off_hdr), 2 * P.cap, spec->n, (const int64_t*)(w + P.off_S),
             (const int64_t*)(w + P.off_dest), (const int32_t*)(w + P.off_ok), col_idx);
  return EBTC_OK;
}
