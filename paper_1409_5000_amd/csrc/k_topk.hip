// Top-K selection per graph: the K largest summed scores are the candidate target nodes
// ("The total communicability": the largest 20 EBTC values; the paper sorts with Introsort,
// O(n log n); a radix select finds the same set in O(n)).
//
// One 1024-thread workgroup per graph:
//   1. radix select on order-preserving integer keys of the scores, 8 bits per pass from the top,
//      finds the key t of the K-th largest score and how many entries equal to t are needed;
//   2. one pass collects every entry above t, plus the lowest-id entries equal to t (an ordered
//      block scan in id order when there are more ties than needed);
//   3. a bitonic sort in LDS orders the K candidates by descending score, then ascending id.
// A graph of at most kTopkSortAll nodes skips 1 and 2: all its entries are sorted and the first K kept.
#include "internal.h"

namespace ebtc {
namespace {

constexpr int kTopkThreads = 1024;
// Graphs up to this many nodes are sorted whole (within the candidate arrays' EBTC_TOPK_LIMIT).
constexpr int kTopkSortAll = 2048;
static_assert(kTopkSortAll <= EBTC_TOPK_LIMIT, "candidate arrays");

// Bitonic sort of P2 (a power of two) keys with their ids in LDS: larger key first, then smaller id.
// Ends with a barrier.
template <typename K>
__device__ inline void bitonic_desc(K* ckey, int* cid, int P2) {
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < P2; i += kTopkThreads) {
        const int p = i ^ stride;
        if (p > i) {
          const bool desc = (i & size) == 0;
          const K ka = ckey[i], kb = ckey[p];
          const int ia = cid[i], ib = cid[p];
          const bool a_first = (ka > kb) || (ka == kb && ia < ib);
          if (a_first != desc) {
            ckey[i] = kb;
            ckey[p] = ka;
            cid[i] = ib;
            cid[p] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
}

__device__ inline uint32_t key_of(float v) {
  const uint32_t b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline uint64_t key_of(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

template <typename T, typename K>
__global__ __launch_bounds__(kTopkThreads) void k_topk(const GraphInfo* graphs, const int32_t* kvec,
                                                       const int64_t* koff, const T* scores, int32_t* idx_out,
                                                       T* val_out) {
  constexpr int NH = 4;  // count rows: wave w adds to row w % NH, so that waves rarely contend
  __shared__ uint32_t hist[256];
  __shared__ uint32_t whist[NH][256];
  __shared__ K s_prefix, s_mask;
  __shared__ int s_remaining, s_eq_total, s_ngt, s_eq_seen;
  __shared__ int wave_cnt[kTopkThreads / 64];
  __shared__ K ckey[EBTC_TOPK_LIMIT];
  __shared__ int cid[EBTC_TOPK_LIMIT];
  const int g = blockIdx.x, tid = threadIdx.x;
  const GraphInfo gi = graphs[g];
  const int K_ = kvec[g];
  if (K_ <= 0) return;
  const int n = gi.n;
  const T* s = scores + gi.score_off;
  constexpr int BITS = (int)sizeof(K) * 8;
  const int64_t o = koff[g];
  if (n <= kTopkSortAll) {  // a small graph: every entry sorted, the first K taken (no radix passes)
    int P2 = 1;
    while (P2 < n) P2 <<= 1;
    for (int i = tid; i < P2; i += kTopkThreads) {
      ckey[i] = i < n ? key_of(s[i]) : (K)0;
      cid[i] = i < n ? i : 0x7fffffff;
    }
    __syncthreads();
    bitonic_desc<K>(ckey, cid, P2);
    for (int r = tid; r < K_; r += kTopkThreads) {
      idx_out[o + r] = cid[r];
      if (val_out) val_out[o + r] = s[cid[r]];
    }
    return;
  }
  if (tid == 0) {
    s_prefix = 0;
    s_mask = 0;
    s_remaining = K_;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  for (int shift = BITS - 8; shift >= 0; shift -= 8) {
    for (int i = tid; i < NH * 256; i += kTopkThreads) (&whist[0][0])[i] = 0;
    __syncthreads();
    const K prefix = s_prefix, mask = s_mask;
    for (int i0 = 0; i0 < n; i0 += kTopkThreads) {  // uniform trip count: the ballots below need all lanes
      const int i = i0 + tid;
      const K k = i < n ? key_of(s[i]) : (K)0;
      const bool in = i < n && (k & mask) == prefix;
      const int bin = (int)((k >> shift) & 255);
      // the lanes sharing the first counted lane's bin (most of them in the leading passes, where
      // scores of one magnitude share their top key bits) add their count with one atomic
      const unsigned long long act = __ballot(in);
      if (act) {
        const int lead = __ffsll((long long)act) - 1;
        const int lbin = __shfl(bin, lead, 64);
        const unsigned long long same = __ballot(in && bin == lbin);
        if (lane == lead) atomicAdd(&whist[wave % NH][lbin], (uint32_t)__popcll(same));
        if (in && bin != lbin) atomicAdd(&whist[wave % NH][bin], 1u);
      }
    }
    __syncthreads();
    if (tid < 256) {
      uint32_t c = 0;
#pragma unroll
      for (int w = 0; w < NH; ++w) c += whist[w][tid];
      hist[tid] = c;
    }
    __syncthreads();
    if (tid < 64) {
      // the bin b of the K-th largest: the largest b whose count from b up reaches the entries still
      // needed (bin 0 when none does). Lane l holds bins 4l..4l+3; a suffix sum over the lanes gives
      // every bin's count from it up, and the bins that reach the need are counted.
      const int rem = s_remaining;
      int h[4], suf[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) h[q] = (int)hist[4 * tid + q];
      const int mine = h[0] + h[1] + h[2] + h[3];
      int incl = mine;  // inclusive suffix over lanes l..63
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_down(incl, o, 64);
        if (tid + o < 64) incl += t;
      }
      const int above = incl - mine;  // the bins of the lanes above this one
      suf[3] = above + h[3];
      suf[2] = suf[3] + h[2];
      suf[1] = suf[2] + h[1];
      suf[0] = suf[1] + h[0];
      int reach = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) reach += (suf[q] >= rem) ? 1 : 0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) reach += __shfl_xor(reach, o, 64);
      const int b = reach > 0 ? reach - 1 : 0;
      if (tid == (b >> 2)) {
        const int q = b & 3;
        const int cum = suf[q] - h[q];  // the entries in the bins above b
        s_remaining = rem - cum;
        s_prefix = prefix | ((K)b << shift);
        s_mask = mask | ((K)255 << shift);
        if (shift == 0) s_eq_total = h[q];
        s_ngt = 0;
        s_eq_seen = 0;
      }
    }
    __syncthreads();
  }
  const K t = s_prefix;
  const int need = s_remaining;         // entries equal to t to take
  const int gt_total = K_ - need;       // entries strictly above t
  const bool all_ties = (s_eq_total == need);
  for (int base = 0; base < n; base += kTopkThreads) {
    const int i = base + tid;
    const K k = (i < n) ? key_of(s[i]) : (K)0;
    const bool gt = (i < n) && k > t;
    const bool eq = (i < n) && k == t;
    if (gt) {
      const int slot = atomicAdd(&s_ngt, 1);
      ckey[slot] = k;
      cid[slot] = i;
    }
    if (all_ties) {
      if (eq) {
        const int slot = gt_total + atomicAdd(&s_eq_seen, 1);
        ckey[slot] = k;
        cid[slot] = i;
      }
    } else {
      const int seen = s_eq_seen;  // uniform: updated only between the barriers below
      if (seen < need) {
        const unsigned long long bal = __ballot(eq);
        if (lane == 0) wave_cnt[wave] = __popcll(bal);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < kTopkThreads / 64; ++w) {
          before += (w < wave) ? wave_cnt[w] : 0;
          total += wave_cnt[w];
        }
        const int rank = seen + before + __popcll(bal & ((1ull << lane) - 1ull));
        if (eq && rank < need) {
          ckey[gt_total + rank] = k;
          cid[gt_total + rank] = i;
        }
        __syncthreads();
        if (tid == 0) s_eq_seen = seen + total;
        __syncthreads();
      }
    }
  }
  __syncthreads();
  int P2 = 1;
  while (P2 < K_) P2 <<= 1;
  for (int i = K_ + tid; i < P2; i += kTopkThreads) {
    ckey[i] = (K)0;
    cid[i] = 0x7fffffff;
  }
  __syncthreads();
  bitonic_desc<K>(ckey, cid, P2);
  for (int r = tid; r < K_; r += kTopkThreads) {
    idx_out[o + r] = cid[r];
    if (val_out) val_out[o + r] = s[cid[r]];
  }
}

// ------------------------------------------------------------------------------- chunked selection
// The same selection with many workgroups per graph (the single-workgroup kernel reads a graph's
// scores five times on one CU, milliseconds at n = 1e6). Per radix pass, k_tk_hist counts the digits
// of one chunk of a graph's scores (those under the prefix chosen so far) and adds its histogram to the
// graph's (integer atomics: the counts, and so every choice, are the same whatever the order), then
// k_tk_select takes the pass's digit with one wave per graph. k_tk_collect places the entries above
// the final key t and counts each chunk's ties; k_tk_ties turns the tie counts into each chunk's first
// rank in id order; k_tk_collect_ties places the lowest-id ties still needed; k_tk_sort orders the K
// candidates of each graph by descending score, then ascending id. Candidate slots are taken by
// atomics, so their order varies, but the sort makes the output unique.
constexpr int kTkThreads = 256;
constexpr int kTkU = 8;  // scores loaded per thread before any is counted

__global__ void k_tk_init(const int32_t* kvec, TkState* st, uint32_t* hist, int passes) {
  const int g = blockIdx.x;
  if (threadIdx.x == 0) {
    TkState z;
    z.prefix = 0;
    z.mask = 0;
    z.remaining = kvec[g];
    z.eq_total = 0;
    z.ngt = 0;
    z.pad = 0;
    st[g] = z;
  }
  for (int i = threadIdx.x; i < passes * 256; i += blockDim.x) hist[(size_t)g * passes * 256 + i] = 0;
}

// Adds the wave's counted lanes to whist[row]: the lanes sharing the first counted lane's bin with one
// atomic (in the leading passes most of them do), the others one by one.
__device__ inline void wave_count(bool in, int bin, uint32_t* row) {
  const int lane = threadIdx.x & 63;
  const unsigned long long act = __ballot(in);
  if (act) {
    const int lead = __ffsll((long long)act) - 1;
    const int lbin = __shfl(bin, lead, 64);
    const unsigned long long same = __ballot(in && bin == lbin);
    if (lane == lead) atomicAdd(&row[lbin], (uint32_t)__popcll(same));
    if (in && bin != lbin) atomicAdd(&row[bin], 1u);
  }
}

template <typename T, typename K>
__global__ __launch_bounds__(kTkThreads) void k_tk_hist(const GraphInfo* graphs, const int32_t* kvec, const T* scores,
                                                        const int32_t* chunk_graph, const int32_t* chunk_begin,
                                                        const TkState* st, uint32_t* hist, int pass, int passes) {
  constexpr int NH = 4, BITS = (int)sizeof(K) * 8;
  __shared__ uint32_t whist[NH][256];
  const int c = blockIdx.x, g = chunk_graph[c];
  if (kvec[g] <= 0) return;
  const GraphInfo gi = graphs[g];
  const int n = gi.n, i0 = (c - chunk_begin[g]) * kTkChunk, i1 = min(n, i0 + kTkChunk);
  const T* s = scores + gi.score_off;
  const K prefix = (K)st[g].prefix, mask = (K)st[g].mask;
  const int shift = BITS - 8 - 8 * pass, tid = threadIdx.x;
  uint32_t* row = whist[(tid >> 6) % NH];
  for (int i = tid; i < NH * 256; i += kTkThreads) (&whist[0][0])[i] = 0;
  __syncthreads();
  for (int b0 = i0; b0 < i0 + kTkChunk; b0 += kTkThreads * kTkU) {  // uniform trip count: ballots
    K k[kTkU];
#pragma unroll
    for (int u = 0; u < kTkU; ++u) {
      const int i = b0 + u * kTkThreads + tid;
      k[u] = i < i1 ? key_of(s[i]) : (K)0;
    }
#pragma unroll
    for (int u = 0; u < kTkU; ++u) {
      const int i = b0 + u * kTkThreads + tid;
      wave_count(i < i1 && (k[u] & mask) == prefix, (int)((k[u] >> shift) & 255), row);
    }
  }
  __syncthreads();
  for (int b = tid; b < 256; b += kTkThreads) {
    uint32_t cnt = 0;
#pragma unroll
    for (int w = 0; w < NH; ++w) cnt += whist[w][b];
    if (cnt) atomicAdd(&hist[((size_t)g * passes + pass) * 256 + b], cnt);
  }
}

// One wave per graph: the digit of the K-th largest among the entries under the prefix (the largest
// bin b whose count from b up reaches the entries still needed), as in the single-workgroup kernel.
template <typename K>
__global__ __launch_bounds__(64) void k_tk_select(const int32_t* kvec, TkState* st, const uint32_t* hist, int pass,
                                                  int passes) {
  constexpr int BITS = (int)sizeof(K) * 8;
  const int g = blockIdx.x, tid = threadIdx.x;
  if (kvec[g] <= 0) return;
  const int shift = BITS - 8 - 8 * pass;
  const uint32_t* hg = hist + ((size_t)g * passes + pass) * 256;
  const int rem = st[g].remaining;
  int h[4], suf[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) h[q] = (int)hg[4 * tid + q];
  const int mine = h[0] + h[1] + h[2] + h[3];
  int incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_down(incl, o, 64);
    if (tid + o < 64) incl += t;
  }
  const int above = incl - mine;
  suf[3] = above + h[3];
  suf[2] = suf[3] + h[2];
  suf[1] = suf[2] + h[1];
  suf[0] = suf[1] + h[0];
  int reach = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) reach += (suf[q] >= rem) ? 1 : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) reach += __shfl_xor(reach, o, 64);
  const int b = reach > 0 ? reach - 1 : 0;
  if (tid == (b >> 2)) {
    const int q = b & 3;
    TkState x = st[g];
    x.remaining = rem - (suf[q] - h[q]);
    x.prefix |= (uint64_t)b << shift;
    x.mask |= (uint64_t)255 << shift;
    if (pass == passes - 1) x.eq_total = h[q];
    st[g] = x;
  }
}

// Entries above the final key t to candidate slots; each chunk's count of entries equal to t.
template <typename T, typename K>
__global__ __launch_bounds__(kTkThreads) void k_tk_collect(const GraphInfo* graphs, const int32_t* kvec,
                                                           const T* scores, const int32_t* chunk_graph,
                                                           const int32_t* chunk_begin, TkState* st, K* ckey,
                                                           int32_t* cid, int32_t* tiecnt) {
  __shared__ int wsum[kTkThreads / 64];
  const int c = blockIdx.x, g = chunk_graph[c];
  if (kvec[g] <= 0) return;
  const GraphInfo gi = graphs[g];
  const int n = gi.n, i0 = (c - chunk_begin[g]) * kTkChunk, i1 = min(n, i0 + kTkChunk);
  const T* s = scores + gi.score_off;
  const K t = (K)st[g].prefix;
  const int tid = threadIdx.x;
  int ties = 0;
  for (int b0 = i0; b0 < i1; b0 += kTkThreads * kTkU) {
    K k[kTkU];
#pragma unroll
    for (int u = 0; u < kTkU; ++u) {
      const int i = b0 + u * kTkThreads + tid;
      k[u] = i < i1 ? key_of(s[i]) : (K)0;
    }
#pragma unroll
    for (int u = 0; u < kTkU; ++u) {
      const int i = b0 + u * kTkThreads + tid;
      if (i >= i1) continue;
      if (k[u] > t) {
        const int slot = atomicAdd(&st[g].ngt, 1);
        ckey[(size_t)g * EBTC_TOPK_LIMIT + slot] = k[u];
        cid[(size_t)g * EBTC_TOPK_LIMIT + slot] = i;
      }
      ties += k[u] == t ? 1 : 0;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ties += __shfl_xor(ties, o, 64);
  if ((tid & 63) == 0) wsum[tid >> 6] = ties;
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (int w = 0; w < kTkThreads / 64; ++w) tot += wsum[w];
    tiecnt[c] = tot;
  }
}

// Each chunk's first tie rank: the ties of the graph's earlier chunks (chunks follow node ids).
__global__ void k_tk_ties(const int32_t* kvec, const int32_t* chunk_begin, const int32_t* tiecnt, int32_t* tiebase,
                          int32_t G) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G || kvec[g] <= 0) return;
  int run = 0;
  for (int c = chunk_begin[g]; c < chunk_begin[g + 1]; ++c) {
    tiebase[c] = run;
    run += tiecnt[c];
  }
}

// The ties still needed, lowest ids first: ranks in id order from the chunk's first rank.
template <typename T, typename K>
__global__ __launch_bounds__(kTkThreads) void k_tk_collect_ties(const GraphInfo* graphs, const int32_t* kvec,
                                                                const T* scores, const int32_t* chunk_graph,
                                                                const int32_t* chunk_begin, const TkState* st,
                                                                const int32_t* tiebase, K* ckey, int32_t* cid) {
  __shared__ int wcnt[kTkThreads / 64];
  const int c = blockIdx.x, g = chunk_graph[c];
  const int K_ = kvec[g];
  if (K_ <= 0) return;
  const int need = st[g].remaining, gt_total = K_ - need;
  int seen = tiebase[c];
  if (seen >= need) return;  // uniform
  const GraphInfo gi = graphs[g];
  const int n = gi.n, i0 = (c - chunk_begin[g]) * kTkChunk, i1 = min(n, i0 + kTkChunk);
  const T* s = scores + gi.score_off;
  const K t = (K)st[g].prefix;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int b0 = i0; b0 < i1 && seen < need; b0 += kTkThreads) {  // uniform: seen is the same in every thread
    const int i = b0 + tid;
    const bool eq = i < i1 && key_of(s[i]) == t;
    const unsigned long long bal = __ballot(eq);
    if (lane == 0) wcnt[wave] = __popcll(bal);
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < kTkThreads / 64; ++w) {
      before += w < wave ? wcnt[w] : 0;
      total += wcnt[w];
    }
    const int rank = seen + before + __popcll(bal & ((1ull << lane) - 1ull));
    if (eq && rank < need) {
      ckey[(size_t)g * EBTC_TOPK_LIMIT + gt_total + rank] = t;
      cid[(size_t)g * EBTC_TOPK_LIMIT + gt_total + rank] = i;
    }
    seen += total;
    __syncthreads();  // wcnt is rewritten by the next round
  }
}

template <typename T, typename K>
__global__ __launch_bounds__(kTopkThreads) void k_tk_sort(const GraphInfo* graphs, const int32_t* kvec,
                                                          const int64_t* koff, const T* scores, const K* ckey_g,
                                                          const int32_t* cid_g, int32_t* idx_out, T* val_out) {
  __shared__ K ckey[EBTC_TOPK_LIMIT];
  __shared__ int cid[EBTC_TOPK_LIMIT];
  const int g = blockIdx.x, tid = threadIdx.x;
  const int K_ = kvec[g];
  if (K_ <= 0) return;
  int P2 = 1;
  while (P2 < K_) P2 <<= 1;
  for (int i = tid; i < P2; i += kTopkThreads) {
    ckey[i] = i < K_ ? ckey_g[(size_t)g * EBTC_TOPK_LIMIT + i] : (K)0;
    cid[i] = i < K_ ? cid_g[(size_t)g * EBTC_TOPK_LIMIT + i] : 0x7fffffff;
  }
  __syncthreads();
  bitonic_desc<K>(ckey, cid, P2);
  const T* s = scores + graphs[g].score_off;
  const int64_t o = koff[g];
  for (int r = tid; r < K_; r += kTopkThreads) {
    idx_out[o + r] = cid[r];
    if (val_out) val_out[o + r] = s[cid[r]];
  }
}

// Scratch sections after the two host tables: byte offsets, then the pointers for a given base.
struct TkLayout {
  size_t st, hist, ckey, cid, tiecnt, tiebase, bytes;
};
TkLayout tk_layout(int32_t G, int64_t nchunks) {
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  TkLayout l{};
  size_t off = 0;
  l.st = off;
  off = up(off + sizeof(TkState) * (size_t)G);
  l.hist = off;
  off = up(off + sizeof(uint32_t) * 256 * 8 * (size_t)G);  // up to 8 passes (FP64 keys)
  l.ckey = off;
  off = up(off + sizeof(uint64_t) * EBTC_TOPK_LIMIT * (size_t)G);
  l.cid = off;
  off = up(off + sizeof(int32_t) * EBTC_TOPK_LIMIT * (size_t)G);
  l.tiecnt = off;
  off = up(off + sizeof(int32_t) * (size_t)nchunks);
  l.tiebase = off;
  off = up(off + sizeof(int32_t) * (size_t)nchunks);
  l.bytes = off;
  return l;
}
struct TkScratch {
  TkState* st;
  uint32_t* hist;
  void* ckey;
  int32_t* cid;
  int32_t* tiecnt;
  int32_t* tiebase;
};
TkScratch tk_scratch(char* base, int32_t G, int64_t nchunks) {
  const TkLayout l = tk_layout(G, nchunks);
  return {(TkState*)(base + l.st), (uint32_t*)(base + l.hist), base + l.ckey, (int32_t*)(base + l.cid),
          (int32_t*)(base + l.tiecnt), (int32_t*)(base + l.tiebase)};
}

template <typename T, typename K>
hipError_t topk_multi_t(const GraphInfo* graphs, int32_t G, const int32_t* kvec, const int64_t* koff, const T* scores,
                        int32_t* idx_out, T* val_out, const int32_t* chunk_graph, const int32_t* chunk_begin,
                        int64_t nchunks, void* scratch, hipStream_t s) {
  constexpr int passes = (int)sizeof(K);  // 8-bit digits
  const TkScratch x = tk_scratch((char*)scratch, G, nchunks);
  K* ckey = (K*)x.ckey;
  hipLaunchKernelGGL(k_tk_init, dim3((unsigned)G), dim3(256), 0, s, kvec, x.st, x.hist, passes);
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL((k_tk_hist<T, K>), dim3((unsigned)nchunks), dim3(kTkThreads), 0, s, graphs, kvec, scores,
                       chunk_graph, chunk_begin, (const TkState*)x.st, x.hist, p, passes);
    hipLaunchKernelGGL((k_tk_select<K>), dim3((unsigned)G), dim3(64), 0, s, kvec, x.st, (const uint32_t*)x.hist, p,
                       passes);
  }
  hipLaunchKernelGGL((k_tk_collect<T, K>), dim3((unsigned)nchunks), dim3(kTkThreads), 0, s, graphs, kvec, scores,
                     chunk_graph, chunk_begin, x.st, ckey, x.cid, x.tiecnt);
  hipLaunchKernelGGL(k_tk_ties, dim3((unsigned)((G + 63) / 64)), dim3(64), 0, s, kvec, chunk_begin,
                     (const int32_t*)x.tiecnt, x.tiebase, G);
  hipLaunchKernelGGL((k_tk_collect_ties<T, K>), dim3((unsigned)nchunks), dim3(kTkThreads), 0, s, graphs, kvec, scores,
                     chunk_graph, chunk_begin, (const TkState*)x.st, (const int32_t*)x.tiebase, ckey, x.cid);
  hipLaunchKernelGGL((k_tk_sort<T, K>), dim3((unsigned)G), dim3(kTopkThreads), 0, s, graphs, kvec, koff, scores,
                     (const K*)ckey, (const int32_t*)x.cid, idx_out, val_out);
  return hipGetLastError();
}

// Phase 1: row_ptr of each realization starts at 0, is non-decreasing and ends at its entry count.
__global__ void k_validate_rowptr(const int32_t* row_ptr, const Task* tasks, const int64_t* nnz, int32_t* bad) {
  const Task tk = tasks[blockIdx.x];
  const int32_t* rp = row_ptr + tk.rowptr_off;
  const int64_t z = nnz[blockIdx.x];
  int b = 0;
  for (int i = threadIdx.x; i < tk.n; i += blockDim.x)
    if (rp[i] > rp[i + 1] || rp[i] < 0) b = 1;
  if (threadIdx.x == 0 && (rp[0] != 0 || (int64_t)rp[tk.n] != z)) b = 1;
  if (__syncthreads_or(b) && threadIdx.x == 0) bad[blockIdx.x] = 1;
}

// Phase 2 (only where phase 1 passed): columns in range, strictly increasing, no self-loop, and the
// transposed entry exists (binary search in the column's row).
__global__ void k_validate_entries(const int32_t* row_ptr, const int32_t* col_idx, const Task* tasks, int32_t* bad) {
  const int r = blockIdx.y;
  if (bad[r]) return;
  const Task tk = tasks[r];
  const int32_t* rp = row_ptr + tk.rowptr_off;
  const int32_t* ci = col_idx + tk.nnz_off;
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0;
  if (row < tk.n) {
    const int s = rp[row], e = rp[row + 1];
    for (int k = s; k < e && !b; ++k) {
      const int c = ci[k];
      if (c < 0 || c >= tk.n || c == row || (k > s && ci[k - 1] >= c)) {
        b = 1;
        break;
      }
      int lo = rp[c], hi = rp[c + 1];
      bool found = false;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int v = ci[mid];
        if (v == row) {
          found = true;
          break;
        }
        if (v < row) lo = mid + 1; else hi = mid;
      }
      if (!found) b = 1;
    }
  }
  if (b) bad[r] = 1;
}

}  // namespace

hipError_t launch_topk(int dtype, const GraphInfo* graphs, int32_t G, const int32_t* kvec, const int64_t* koff,
                       const void* scores, int32_t* idx_out, void* val_out, hipStream_t s) {
  if (dtype == EBTC_F64)
    hipLaunchKernelGGL((k_topk<double, uint64_t>), dim3((unsigned)G), dim3(kTopkThreads), 0, s, graphs, kvec, koff,
                       (const double*)scores, idx_out, (double*)val_out);
  else
    hipLaunchKernelGGL((k_topk<float, uint32_t>), dim3((unsigned)G), dim3(kTopkThreads), 0, s, graphs, kvec, koff,
                       (const float*)scores, idx_out, (float*)val_out);
  return hipGetLastError();
}

size_t topk_multi_scratch_bytes(int32_t G, int64_t nchunks) { return tk_layout(G, nchunks).bytes; }

hipError_t launch_topk_multi(int dtype, const GraphInfo* graphs, int32_t G, const int32_t* kvec, const int64_t* koff,
                             const void* scores, int32_t* idx_out, void* val_out, const int32_t* chunk_graph,
                             const int32_t* chunk_begin, int64_t nchunks, void* scratch, hipStream_t s) {
  if (G < 1 || nchunks < G || nchunks > INT32_MAX) return hipErrorInvalidValue;
  if (dtype == EBTC_F64)
    return topk_multi_t<double, uint64_t>(graphs, G, kvec, koff, (const double*)scores, idx_out, (double*)val_out,
                                          chunk_graph, chunk_begin, nchunks, scratch, s);
  return topk_multi_t<float, uint32_t>(graphs, G, kvec, koff, (const float*)scores, idx_out, (float*)val_out,
                                       chunk_graph, chunk_begin, nchunks, scratch, s);
}

hipError_t launch_validate(const int32_t* row_ptr, const int32_t* col_idx, const Task* tasks, const int64_t* nnz,
                           int64_t R, int32_t max_n, int32_t* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_validate_rowptr, dim3((unsigned)R), dim3(256), 0, s, row_ptr, tasks, nnz, bad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_validate_entries, dim3((unsigned)((max_n + 255) / 256), (unsigned)R), dim3(256), 0, s, row_ptr,
                     col_idx, tasks, bad);
  return hipGetLastError();
}

}  // namespace ebtc
