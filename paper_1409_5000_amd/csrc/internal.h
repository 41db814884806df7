// Internal types and launchers of the EBTC library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/ebtc.h"

namespace ebtc {

// Records msg as ebtc_last_error() and returns code (shared by every entry point of the library).
int report_error(int code, const std::string& msg);

constexpr int kBlock = 256;          // threads of a streaming workgroup (4 waves of 64)
constexpr int kDotsThreads = 1024;   // threads of a workgroup forming a row block's dot partials
constexpr int kRowsPerBlock = 2048;  // CSR rows owned by one workgroup in the Lanczos kernels
constexpr int kRowsPerThread = kRowsPerBlock / kBlock;
constexpr int kStagedThreads = 1024; // threads of the LDS-staged SpMV workgroup (16 waves)
constexpr int kLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950
constexpr int kMLimit = EBTC_M_LIMIT;
constexpr int kPartStride = kMLimit; // doubles per workgroup in the dot-partial arena (one per basis vector)
constexpr int kMaxChunks = 32;       // chunks of the canonical partial-sum order

// One realization of the batch as the kernels see it (device table, 64 bytes).
struct Task {
  int64_t rowptr_off;  // start of the realization's local row_ptr block
  int64_t nnz_off;     // start of its entries in col_idx / values
  int64_t vec_off;     // element offset of its basis block (m_slots x n, vector-major) in the V arena
  int64_t w_off;       // element offset of its product vector w [n] in the W arena
  int64_t u_off;       // element offset of its combined vector u [n] in the U arena
  int64_t part_off;    // double offset of its per-workgroup dot partials (nblk x kPartStride); the
                       // norm partials (nblk) sit at the same offset / kPartStride in the norm arena
  int32_t n;
  int32_t graph;
  int32_t nblk;        // row blocks of kRowsPerBlock rows
  int32_t blk_begin;   // first flattened workgroup id of this realization in a batched launch
  int64_t aux_off;     // first entry of the realization in its SpMV form's entry arenas (sorted columns,
                       // values, products): entries of the realizations of the same form before it
  int32_t aux_blk;     // its first row block in the form's per-block arenas and in the form's launches
  int32_t form;        // index of its SpMV form in the batch's plan
};
static_assert(sizeof(Task) == 80, "Task layout");

// Per row block of the column-segmented form, written by the sort: what the first loads of a product
// need, so that they wait on one load instead of the chain workgroup map -> realization -> row
// pointers -> band table.
struct SegBlock {
  int64_t entries;   // index of the block's first slot in seg_col / seg_val (a multiple of four)
  int64_t vec_off;   // Task::vec_off of its realization
  int32_t n;         // order of its realization
  int32_t nnz;       // slots of the block: its entries and the zero padding of its wave bands
  int16_t rows;      // rows of the block
  int16_t flag;      // the block's seg_flag
  uint16_t wo0[17];  // band starts of segment 0 (the first 17 entries of its seg_woff table)
  uint16_t quads;    // quad slots (four entries each, 256 per wave) of its largest padded band, 1..3
};
static_assert(sizeof(SegBlock) == 64, "SegBlock layout");

// One workgroup's share of the entry-balanced SpMV form: the rows of realization `task` whose first
// entry falls in its entries [q * E, (q + 1) * E), E = LzArgs::bal_entries (the last share of a
// realization also takes its trailing empty rows). Row bounds written once per call.
struct BalPart {
  int32_t task;
  int32_t q;
  int32_t r_begin;
  int32_t r_end;
};
static_assert(sizeof(BalPart) == 16, "BalPart layout");
// Share sizes of the entry-balanced form: the default is the largest power of two in this range that
// still gives a batch about 8192 shares (two or more workgroups per CU in flight, few launches' worth
// of row walks per workgroup).
constexpr int kBalEntriesMin = 4096, kBalEntriesMax = 16384, kBalTargetShares = 8192;

// One work item of the panel form's products pass: panel `panel` of row units [b0, b1) of
// realization `task` (unit indices local to the realization). The once-per-call scan takes the same
// struct for a group of units (panel unused).
struct PanItem {
  int32_t task;
  int32_t panel;
  int32_t b0;
  int32_t b1;
};
static_assert(sizeof(PanItem) == 16, "PanItem layout");
// Panel form: the row-sum pass's LDS for one unit's products (at most 128 KB), the largest unit
// (rows), and the largest number of panels per realization (the sort's count table).
constexpr int kPanCapBytes = 128 * 1024;
constexpr int kPanMaxUnit = 256;
constexpr int kPanMaxPanels = 1024;

struct GraphInfo {
  int64_t score_off;   // offset of the graph's block in the score output
  int32_t n;
  int32_t first;       // first realization index
  int32_t count;       // realizations of this graph
  int32_t pad;
};
static_assert(sizeof(GraphInfo) == 24, "GraphInfo layout");

// Per-realization Lanczos state (FP64 scalars), one per realization in the workspace.
// Basis vectors are stored unnormalised: v_i = s[i] * Vraw_i (the normalisation of step j is folded
// into the scale instead of a separate pass over the vector).
struct RState {
  double alpha[kMLimit];
  double beta[kMLimit];
  double s[kMLimit + 1];
  double y[kMLimit];       // exp(T - theta I) e1
  double scal[kMLimit];    // scal[j] = max(|alpha_0..j|, beta_0..j-1): the breakdown reference of step j
  double theta;
  double est;
  double spare;
  double beta0;            // ||start vector|| = sqrt(n)
  int32_t m_used;
  int32_t flags;
  int32_t done;            // 1 once the realization stopped (breakdown, estimate met, cap)
  int32_t pad0;
};

// Arguments shared by the Lanczos streaming kernels.
struct LzArgs {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const void* values;      // nullptr = all ones
  const Task* tasks;
  const int32_t* blkmap;   // flattened workgroup -> task; nullptr = single-task launch
  const int32_t* sub_blocks;  // the launch's row blocks (batch-wide ids) when an SpMV form covers part of
                              // the batch; nullptr = every block in order
  int32_t single_task;
  int32_t hub_threshold;
  RState* state;
  void* V;
  void* W;
  void* U;
  double* part;            // dot partials
  double* npart;           // norm partials
  int32_t seglen;          // > 0: LDS-staged SpMV with column segments of this many elements
  int32_t m_fixed;         // fixed m, or 0 (adaptive)
  int32_t m_max;
  double eps;              // unit roundoff of the working precision
  ebtc_diag* diag;         // optional diagnostics output (combine flags non-finite results there)
  // column-segmented SpMV (seg_cols > 0): the entries of every row block sorted by column segment
  int32_t seg_cols;        // columns per segment
  int32_t seg_stride;      // bytes of per-(segment, row) counts per row block: max segments x kRowsPerBlock
  int32_t* seg_flag;       // [row blocks] 1 = sorted, 0 = the block uses the CSR-stream form
  uint8_t* seg_cnt;        // [row blocks][seg_stride] entries of row r in segment s at [s * rows2 + r],
                           // rows2 = the block's rows rounded up to even (the pad row's count is 0)
  uint16_t* seg_col;       // [slots] column - s * seg_cols, a block's entries ordered by (segment, row);
                           // each (segment, wave band) run padded with zeros to a multiple of four
                           // entries, each block's first slot a multiple of four
  void* seg_val;           // [slots] values in the same order (nullptr for pattern-only graphs)
  int32_t seg_vec;         // 1: every n and seg_cols are multiples of 16 bytes / element size (16-byte
                           // slice loads and stores)
  uint16_t* seg_woff;      // [row blocks][seg_wstride] wave bands: entries of rows [128 w, 128 w + 128) in
                           // segment s at [woff[s * 17 + w], woff[s * 17 + w + 1])
  int32_t seg_wstride;     // max segments x 17
  SegBlock* seg_blk;       // [row blocks] descriptors for the first loads of a product
  // entry-balanced SpMV (bal != nullptr): one workgroup per share of bal_entries entries
  BalPart* bal;            // [nbal] shares, realization by realization
  const int64_t* bal_begin;  // [R + 1] first share of each realization (host-computed)
  int32_t nbal;
  int32_t bal_entries;     // entries per share
  // panel form (pan_cols > 0): each group of row units' entries put in (panel, unit) order once per
  // call; each step a products pass (one vector slice in LDS serves a group's entries of a panel) and a
  // row-sum pass per unit
  int32_t pan_cols;        // columns per panel
  int32_t pan_pmax;        // most panels of a realization in the launch (the stride of pan_run)
  int32_t pan_unit;        // rows per unit (64, 128 or 256)
  int32_t pan_lds;         // entries of a unit the row-sum pass holds in LDS (more: stream arithmetic)
  int32_t* pan_flag;       // [units] 1 = sorted, 0 = the unit uses the CSR-stream arithmetic
  int2* pan_run;           // [units][pan_pmax] {first entry, count} of the unit's run of panel p, entries
                           // counted from the realization's first
  uint16_t* pan_col;       // [entries] column - p * pan_cols
  uint16_t* pan_perm;      // [entries] the entry's position in its unit's CSR range
  void* pan_val;           // [entries] values in the same order (nullptr for pattern-only graphs)
  void* pan_prod;          // [entries] the step's products, same order
  const PanItem* pan_items;  // products-pass work items
  const PanItem* pan_groups;  // [groups] unit groups of the once-per-call scan (panel unused)
  int32_t pan_nitems;
  // memory-bounded form (window > 0): Gram-Schmidt against the last `window` basis vectors only, the
  // raw basis kept in a ring of window + 1 slots (vector i in slot i % (window + 1))
  int32_t window;
  int32_t stop_mused;      // second pass of the memory-bounded form: steps j >= m_used - 1 are skipped
  // adaptive batched pass: live[j] = realizations still running after step j's check (zeroed by the
  // start kernel, counted by the check); every kernel of step j + 1 returns at once when it is 0
  int32_t* live;
  int32_t unit_start;      // 1: v_0 is the raw all-ones vector, so step 0's product is A's row sums
  int32_t first_in_prepare;  // 1: the column-segmented sort also writes step 0's product (weighted
                             // graphs), so the step sequence launches none for it
};

// Slot of basis vector i in a realization's V block.
__host__ __device__ inline size_t vslot(const LzArgs& a, int i) {
  return a.window > 0 ? (size_t)(i % (a.window + 1)) : (size_t)i;
}

// ---- launchers (k_lanczos.hip, k_spmv.hip)
hipError_t launch_blkmap(const Task* tasks, int64_t R, int32_t* blkmap, hipStream_t s);
// Largest row length of each realization (out: device [R]).
hipError_t launch_row_max(const Task* tasks, const int32_t* row_ptr, int64_t R, int32_t* out, hipStream_t s);
hipError_t launch_start(int dtype, const LzArgs& a, int64_t nblocks, hipStream_t s);
// Subgraph centrality: processes started at e_{nodes[r]}, and SC = e^{theta} y_0 per process.
hipError_t launch_start_unit(int dtype, const LzArgs& a, const int32_t* nodes, int64_t nblocks, hipStream_t s);
hipError_t launch_sc_out(const RState* state, const Task* tasks, const int32_t* nodes, int64_t count, double* out,
                         hipStream_t s);
// Phase A: the SpMV kernel (column-segmented when a.seg_cols > 0, LDS-staged when a.seglen > 0, else
// the CSR stream for lanes == 0 and lane groups otherwise).
hipError_t launch_spmv_step(int dtype, bool has_val, int lanes, int j, const LzArgs& a, int64_t nblocks,
                            hipStream_t s);
hipError_t launch_dots_step(int dtype, int j, const LzArgs& a, int64_t nblocks, hipStream_t s);

hipError_t launch_dots_again(int dtype, int j, const LzArgs& a, int64_t nblocks, hipStream_t s);
hipError_t launch_update(int dtype, int j, bool from_w, bool final_pass, bool second_pass, const LzArgs& a,
                         int64_t nblocks, hipStream_t s);
// Dots and update of step j in one launch; every realization must fit one row block (n <= kRowsPerBlock)
// and the basis window must be the whole basis (one Gram-Schmidt pass).
hipError_t launch_dots_update_1(int dtype, int j, const LzArgs& a, int64_t nblocks, hipStream_t s);
// Largest Gram-Schmidt window one dot-partial launch (and the fused dots-and-update kernel) covers;
// wider windows take one dot launch per 64 basis vectors.
constexpr int kDotsWindow = 64;
hipError_t launch_combine(int dtype, const LzArgs& a, int64_t nblocks, hipStream_t s);
// Single-kernel solve (k_solve.hip): `count` realizations (one workgroup each, n <= kRowsPerBlock, the
// whole basis, one Gram-Schmidt pass) from the start vector to u = beta0 V y, with diag and checkpoint
// as the final small exponential writes them.
hipError_t launch_solve_1(int dtype, bool has_val, const LzArgs& a, int64_t count, int steps, int shift, double tol,
                          ebtc_diag* diag, double* ckpt, int n_max, int64_t z_max, hipStream_t s);
// Opts the single-kernel solve in to the full LDS; once per process, before any stream capture.
hipError_t prepare_solve_kernels();
// Memory-bounded form, second pass: restart from the start vector keeping theta, y, m_used, flags;
// before step j, u (+)= beta0 y_j s_j Vraw_j (j = 0 assigns) and the realization stops after m_used.
hipError_t launch_restart(int dtype, const LzArgs& a, int64_t nblocks, hipStream_t s);
hipError_t launch_accum(int dtype, const LzArgs& a, int j, int64_t nblocks, hipStream_t s);
hipError_t launch_sum(int dtype, const GraphInfo* graphs, int32_t G, int32_t max_blocks, const Task* tasks,
                      const RState* state, const void* U, void* scores, double* log_scale, hipStream_t s);
hipError_t launch_spmv(int dtype, bool has_val, int lanes, int hub, int seglen, int32_t n, const int32_t* row_ptr,
                       const int32_t* col_idx, const void* values, const void* x, void* y, hipStream_t s);
// Largest column segment (elements) the staged SpMV can hold in LDS next to its per-row state.
int staged_max_seglen(int dtype);
// Opts the staged kernels in to the full LDS once per process (call before any stream capture).
hipError_t prepare_staged_kernels();
// Column-segmented SpMV: at most kSegMax segments per realization; largest segment that fits in LDS.
constexpr int kSegMax = 32;
// Slots of the column-segmented arenas per row block beyond its entries: up to three zeros after each
// of its (segment, wave band) runs, and the rounding of its first slot up to a multiple of four.
constexpr int kSegSlack = 3 * 16 * kSegMax + 8;
int seg_max_cols(int dtype);
hipError_t prepare_seg_kernels();
// Sorts every row block's entries by column segment (a.seg_* arrays); smax = max segments in the launch.
hipError_t launch_seg_prepare(int dtype, bool has_val, const LzArgs& a, int64_t nblocks, int smax, hipStream_t s);
// Row bounds of the entry-balanced form's shares of realizations [t0, t0 + count).
hipError_t launch_bal_rows(const LzArgs& a, int t0, int count, hipStream_t s);
// Panel form: largest panel (columns) for the products pass's LDS slice, largest LDS budget of the
// row-sum pass (entries), and the once-per-call sort (count, scan over `groups`, place).
int pan_max_cols(int dtype);
int pan_max_lds(int dtype);
// Entries of the CSR-stream arithmetic's LDS buffer (rows beyond it are summed as hub rows).
int stream_cap(int dtype);
hipError_t prepare_pan_kernels();
hipError_t launch_pan_prepare(int dtype, bool has_val, const LzArgs& a, int64_t nblocks, const PanItem* groups,
                              int ngroups, hipStream_t s);

// ---- launchers (k_tridiag.hip)
// mode 0: final (closes step m_steps-1 when still open; writes y/theta/est, diag, checkpoint);
// mode 1: adaptive check after step j (closes step j, stops on breakdown, estimate < tol or m_max).
hipError_t launch_tridiag_state(const LzArgs& a, int64_t first, int64_t count, int mode, int j, int m_steps,
                                int shift, double tol, ebtc_diag* diag, double* ckpt, hipStream_t s);
hipError_t launch_tridiag_arrays(int32_t count, int32_t k, const double* alpha, const double* beta, double* y,
                                 double* theta, int32_t shift, hipStream_t s);

// ---- launchers (k_topk.hip)
hipError_t launch_topk(int dtype, const GraphInfo* graphs, int32_t G, const int32_t* kvec, const int64_t* koff,
                       const void* scores, int32_t* idx_out, void* val_out, hipStream_t s);
// Top-K with many workgroups per graph, for batches holding a graph of at least kTopkMultiMin nodes:
// the radix passes count chunks of kTkChunk scores per workgroup into per-graph histograms, one wave
// per graph picks each pass's digit, the candidates are collected by chunk and sorted per graph.
constexpr int kTopkMultiMin = 32768;
constexpr int kTkChunk = 16384;
// Per-graph state of the chunked selection: the digits chosen so far (prefix under mask), the entries
// still needed at the prefix, the ties at the final key, and the entries above it placed so far.
struct TkState {
  uint64_t prefix, mask;
  int32_t remaining, eq_total, ngt, pad;
};
static_assert(sizeof(TkState) == 32, "TkState layout");
// Scratch of the chunked top-K (device, 256-byte aligned sections): chunk_graph [nchunks] (graph of
// each chunk, host-built), chunk_begin [G + 1] (first chunk of each graph, host-built), then the
// kernels' own arrays. topk_multi_scratch_bytes gives the size of the part after the two host tables.
size_t topk_multi_scratch_bytes(int32_t G, int64_t nchunks);
hipError_t launch_topk_multi(int dtype, const GraphInfo* graphs, int32_t G, const int32_t* kvec, const int64_t* koff,
                             const void* scores, int32_t* idx_out, void* val_out, const int32_t* chunk_graph,
                             const int32_t* chunk_begin, int64_t nchunks, void* scratch, hipStream_t s);

// ---- launchers (k_topk.hip, structural check)
hipError_t launch_validate(const int32_t* row_ptr, const int32_t* col_idx, const Task* tasks, const int64_t* nnz,
                           int64_t R, int32_t max_n, int32_t* bad, hipStream_t s);

// ---- launchers (k_adjoint.hip)
int adjoint_max_m();
hipError_t launch_start_vec(int dtype, const LzArgs& a, const GraphInfo* graphs, const void* g, int64_t nblocks,
                            hipStream_t s);
hipError_t launch_start_norm(const LzArgs& a, int64_t R, hipStream_t s);
hipError_t launch_block_exp(const RState* fwd, const RState* adj, const Task* tasks, const double* log_scale,
                            double* xout, int64_t R, hipStream_t s);
hipError_t launch_build_zv(int dtype, const LzArgs& fwd, const LzArgs& adj, const double* x, void* Z, void* Vn,
                           int ld, int64_t nblocks, hipStream_t s);
hipError_t launch_sddmm(int dtype, int ld, const LzArgs& fwd, const void* Z, const void* Vn, void* grad,
                        int64_t nblocks, hipStream_t s);
// Counts the realizations whose recomputed forward state differs bit for bit from the forward call's
// checkpoint (ckpt: [R][kCkptDoubles]) into *mismatch (device int32, cleared first).
hipError_t launch_ckpt_check(const RState* st, const double* ckpt, int64_t R, int32_t* mismatch, hipStream_t s);

// Leading dimension of the adjoint's block-exponential output per realization (the adjoint's Krylov
// dimension is at most adjoint_max_m() <= kXLd).
constexpr int kXLd = 64;

// checkpoint layout per realization (doubles): alpha[kMLimit], beta[kMLimit], theta, beta0, m_used, flags
constexpr int kCkptDoubles = 2 * kMLimit + 4;

}  // namespace ebtc
