/*
 * ebtc.h -- C ABI of the MI355X (gfx950) Estrada-Benzi total-communicability library.
 *
 * What the library computes (Fioriti & Chinnici, arXiv 1409.5000, "Identification algorithm"):
 *   for each graph g with realizations A_{g,1..N_g} on the same n_g nodes,
 *     EBTC_{g,k} = exp(A_{g,k}) 1                      eq. (4), row sums of the matrix exponential,
 *                                                      by an m-step Lanczos (Krylov) approximation
 *     S_g        = sum_k EBTC_{g,k}                     eq. (5), plain sum over realizations
 *     top-K(S_g)                                       the K largest summed scores are the candidate
 *                                                      target nodes ("The total communicability")
 *   To keep exp(A) finite the sum is returned in scaled form: S_g = e^{Sigma_g} * S~_g with one FP64
 *   log-scale Sigma_g per graph (Sigma_g = max_k theta*_k, theta*_k the largest Ritz value).
 *
 * Conventions
 *   - Every call returns an int status (EBTC_OK = 0). Arguments are checked before anything is
 *     enqueued, so a failing call has no side effect and leaves every output untouched;
 *     ebtc_last_error() then holds a thread-local message.
 *   - "device" pointers are HIP device allocations on the current device; "host" pointers are
 *     ordinary host memory. The library never allocates device memory: the caller passes a workspace
 *     whose size ebtc_plan() reports. Device pointers in a batch are borrowed and must outlive it.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream). Calls that take a stream
 *     are asynchronous on it unless stated otherwise.
 *   - Conditions found on the device never fail a call; they set ebtc_diag.flags.
 *   - A batch is not thread-safe; distinct batches are. Two calls that share a workspace race.
 */
#ifndef EBTC_H
#define EBTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EBTC_VERSION_MAJOR 0
#define EBTC_VERSION_MINOR 1
#define EBTC_M_LIMIT 128     /* largest Krylov dimension (fixed m or adaptive cap) */
#define EBTC_TOPK_LIMIT 4096 /* largest K per graph in ebtc_topk */

enum ebtc_status {
  EBTC_OK = 0,
  EBTC_EINVAL = 1,        /* bad argument: NULL where not allowed, size or option out of range   */
  EBTC_EBADGRAPH = 2,     /* inconsistent batch description, or ebtc_validate found a bad graph  */
  EBTC_EWORKSPACE = 3,    /* workspace (or checkpoint) smaller than ebtc_plan reported           */
  EBTC_EHIP = 4,          /* a HIP runtime call failed                                           */
  EBTC_ENOTSUPPORTED = 5  /* well-formed request outside what this library implements            */
};

enum ebtc_dtype { EBTC_F32 = 0, EBTC_F64 = 1 };

enum ebtc_schedule {
  EBTC_SCHED_AUTO = 0,     /* library picks: SINGLE when the batch allows it, else BATCHED         */
  EBTC_SCHED_PLAIN = 1,    /* one realization at a time: per Lanczos step an SpMV, a Gram-Schmidt dot
                              and an update launch (dots and update are one launch when every
                              realization has at most 2048 nodes), plus a few per realization     */
  EBTC_SCHED_BATCHED = 2,  /* all realizations of all graphs advance together, one launch per
                              Lanczos phase, optionally replayed from a captured hipGraph          */
  EBTC_SCHED_SINGLE = 3    /* all realizations in one launch, one workgroup running each
                              realization's whole Lanczos process (then one launch for the sum):
                              needs every n_g <= 2048, m (adaptive: m_max) <= 64, reorth = 1 and
                              the SpMV form AUTO, STREAM, SEGMENTED or BALANCED
                              (EBTC_ENOTSUPPORTED otherwise). Same results as BATCHED with the
                              CSR-stream arithmetic, bit for bit                                 */
};

enum ebtc_flags {
  EBTC_FLAG_BREAKDOWN = 1, /* Krylov space closed early (beta_j ~ 0): result exact, informational */
  EBTC_FLAG_CAPPED = 2,    /* adaptive mode reached m_max before the estimate met tol             */
  EBTC_FLAG_NONFINITE = 4  /* a non-finite value appeared (e.g. overflow with shift = 0)          */
};

typedef struct ebtc_batch ebtc_batch; /* opaque */

/*
 * A batch: G graphs, graph g has n_g nodes and N_g realizations; R = sum_g N_g realizations in
 * graph order (all realizations of graph 0, then graph 1, ...). Each realization is a CSR matrix of
 * a simple undirected graph ("Signal processing on graphs": symmetric 0/1 adjacency), stored
 * symmetrically (both (i,j) and (j,i)), columns sorted within a row, no self-loops.
 */
typedef struct {
  int32_t dtype;               /* EBTC_F32 or EBTC_F64: type of values, vectors and scores          */
  int32_t num_graphs;          /* G >= 1                                                           */
  int64_t num_realizations;    /* R = sum_g graph_nreal[g]                                         */
  const int32_t* graph_n;      /* host [G]: n_g >= 1                                               */
  const int32_t* graph_nreal;  /* host [G]: N_g >= 1                                               */
  const int64_t* rowptr_off;   /* host [R]: realization r's row pointers are row_ptr[rowptr_off[r] ..
                                  rowptr_off[r] + n_g], local (first entry 0, last = its nnz)       */
  const int64_t* nnz_off;      /* host [R+1]: realization r's entries are [nnz_off[r], nnz_off[r+1])
                                  of col_idx / values; nnz_off[0] = 0, non-decreasing               */
  const int32_t* row_ptr;      /* device int32                                                     */
  const int32_t* col_idx;      /* device int32, local node ids in [0, n_g)                         */
  const void* values;          /* device, dtype, one weight per stored entry; NULL = all ones      */
} ebtc_batch_desc;

typedef struct {
  int32_t m;             /* fixed Krylov dimension 1..EBTC_M_LIMIT; 0 = adaptive                  */
  int32_t m_max;         /* adaptive cap 1..EBTC_M_LIMIT                                          */
  double tol;            /* adaptive stop: Saad's relative estimate beta_j |y_j| / ||y|| < tol     */
  int32_t reorth;        /* classical Gram-Schmidt passes per step against the whole basis: 1 or 2;
                            0 = memory-bounded form: one pass against v_{j-1} and v_j only (the
                            three-term recurrence), three basis vectors per realization in the
                            workspace, and a second run of the same steps that regenerates the
                            basis bit for bit and accumulates u = beta0 V y (about twice the work
                            of reorth 1 at m / 3 of its basis memory; no adjoint)               */
  int32_t schedule;      /* enum ebtc_schedule                                                    */
  int32_t use_hipgraph;  /* batched schedule: capture the launch sequence once, replay it after    */
  int32_t shift;         /* 1 (default): factor out theta*; 0: theta* = 0 (overflow-prone, tests)  */
  int32_t spmv;          /* SpMV form (enum ebtc_spmv_form): 0 = auto (the form ebtc_tune picked for
                            this batch, else the CSR-stream form)                                 */
  int32_t lanes_per_row; /* lane-group form: lanes per CSR row, 4, 8, 16 or 32 (0 = 8)            */
  int32_t hub_threshold; /* rows with more entries are reduced by a whole workgroup; 0 = auto     */
  int32_t seg_len;       /* LDS-staged and column-segmented forms: vector segment length in
                            elements (0 = the form's default: the largest that fits for LDS-staged,
                            12288 FP32 / 6144 FP64 for column-segmented); for the entry-balanced
                            form, entries per share, 256..2^24 (0 = the largest power of two in
                            4096..16384 that leaves the batch 8192 shares)                        */
} ebtc_opts;

enum ebtc_spmv_form {
  EBTC_SPMV_AUTO = 0,
  EBTC_SPMV_STREAM = 1,      /* each workgroup streams its rows' contiguous entries, gathers, sums
                                every row in FP64 from LDS                                         */
  EBTC_SPMV_LANE_GROUPS = 2, /* L lanes per row, two rows and four entries per lane in flight      */
  EBTC_SPMV_LDS_STAGED = 3,  /* the gathered vector streams through LDS in column segments         */
  EBTC_SPMV_SEGMENTED = 4,   /* each call first sorts every row block's entries by column segment
                                (stable; 16-bit in-segment columns, 8-bit per-row counts); each step
                                then stages one vector segment at a time in LDS and serves every
                                gather of that segment from it. Needs ceil(n / seg_len) <= 32;
                                row blocks with more than 65535 entries, or a row with more than 255
                                entries in one segment, use the CSR-stream form                     */
  EBTC_SPMV_BALANCED = 5,    /* the CSR-stream arithmetic with workgroups over equal shares of a
                                realization's entries (seg_len each) instead of equal row counts: rows
                                stay whole, so the sums are the stream form's; for graphs whose
                                first rows hold most entries (preferential attachment). Each call
                                first finds every share's rows                                     */
  EBTC_SPMV_PANELED = 6      /* for vectors too large for the column-segmented form: each call first
                                puts the entries of groups of row units (64-256 rows) in column-panel
                                order (seg_len columns per panel, 0 = 12288 FP32 / 6144 FP64); each
                                step then forms the products panel by panel, one vector slice in LDS
                                serving a group's entries, and a second pass sums every row's products
                                in entry order (the stream form's sums, bit for bit). Units with more
                                entries than the row-sum pass holds in LDS (1.5 times the densest
                                realization's mean per unit, at most 32768 FP32 / 16384 FP64) or a row
                                beyond the stream form's LDS capacity use the CSR-stream arithmetic;
                                at most 1024 panels per realization                                */
};
#define EBTC_TUNE_SLOTS 10 /* entries of ebtc_tune's ms_out */

/* Per-realization diagnostics (device array [R], written by ebtc_scores). */
typedef struct {
  int32_t m_used;  /* Lanczos steps taken (size of T)                                              */
  int32_t flags;   /* enum ebtc_flags                                                              */
  double theta;    /* theta*: the largest Ritz value, the realization's log-scale                  */
  double est;      /* Saad's relative error estimate at the last step (0 after a breakdown)        */
} ebtc_diag;

/* ---------------------------------------------------------------- library information            */
int ebtc_version(int* major, int* minor);
const char* ebtc_status_str(int status);
/* Message of the last failing call on this thread ("" if none). Valid until the next call. */
const char* ebtc_last_error(void);
/* Fills defaults: m = 30, m_max = 60, tol = 1e-6, reorth = 1, schedule AUTO, hipgraph on, shift on. */
void ebtc_default_opts(ebtc_opts* opts);

/* ---------------------------------------------------------------- batch                          */
/* Host-only. Copies the host arrays of `desc`, checks counts and offsets (n_g >= 1, N_g >= 1,
 * R = sum N_g, nnz_off non-decreasing from 0, each realization's nnz < 2^31, dtype known) and
 * records the borrowed device pointers. EBTC_EINVAL for NULL or out-of-range fields,
 * EBTC_EBADGRAPH for inconsistent offsets. The O(nnz) structural check is ebtc_validate. */
int ebtc_batch_create(const ebtc_batch_desc* desc, ebtc_batch** out);
/* Frees host-side state (and captured graphs). NULL-safe. Never frees caller memory. */
void ebtc_batch_destroy(ebtc_batch* batch);

/* Host-only. Workspace bytes ebtc_scores needs for `opts` (all realizations resident), and the
 * checkpoint bytes ebtc_scores_backward needs (0 if not requested). Also validates opts. */
int ebtc_plan(ebtc_batch* batch, const ebtc_opts* opts, size_t* ws_bytes, size_t* ckpt_bytes);

/* ---------------------------------------------------------------- forward                        */
/* Scaled summed scores, eq. (4)-(5), asynchronous on `stream`.
 *   ws, ws_bytes   device workspace of at least the planned size (contents need no initialisation)
 *   scores_out     device [sum_g n_g] of dtype: S~_g for graph 0, then graph 1, ...
 *   log_scale_out  device [G] double: Sigma_g; the summed score is e^{Sigma_g} S~_g
 *   ckpt_out       device checkpoint of the planned size for ebtc_scores_backward, or NULL
 *   diag_out       device [R] ebtc_diag, or NULL
 * Lanczos: start vector 1/sqrt(n), full reorthogonalisation against the whole basis (reorth 0: the
 * three-term recurrence, two passes), FP64 tridiagonal exponential; breakdown
 * (beta_j <= 64 eps max(|alpha|, beta)) ends a realization early.
 * Realizations of a graph are summed in k order with FP64 weights e^{theta*_k - Sigma_g}. */
int ebtc_scores(ebtc_batch* batch, const ebtc_opts* opts, void* ws, size_t ws_bytes, void* scores_out,
                double* log_scale_out, void* ckpt_out, ebtc_diag* diag_out, void* stream);

/* For callers that cannot allocate device memory -- code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation: ebtc_scores with the workspace taken from a fixed device
 * array of the library (64 MiB per GPU, EBTC_NOALLOC_WS_BYTES, held on every GPU the library runs on
 * until the process ends) instead of a caller buffer. Calls no allocating routine: the launches are
 * eager (use_hipgraph is ignored; instantiating a graph would allocate), and the array's device address
 * is looked up once per GPU on the first call there. Arguments, outputs, results and errors as for
 * ebtc_scores, plus EBTC_EWORKSPACE when ebtc_plan's size for (batch, opts) exceeds the array (nothing
 * is enqueued then). Every call on one GPU uses that GPU's one array: calls that overlap on a GPU
 * (other threads, other streams, or a second call enqueued before the first has run on another
 * stream) race and give undefined results; calls in order on one stream do not. */
#define EBTC_NOALLOC_WS_BYTES ((size_t)64 << 20)
int ebtc_scores_noalloc(ebtc_batch* batch, const ebtc_opts* opts, void* scores_out, double* log_scale_out,
                        void* ckpt_out, ebtc_diag* diag_out, void* stream);

/* ---------------------------------------------------------------- adjoint                        */
/* Workspace bytes for ebtc_scores_backward (host-only). EBTC_ENOTSUPPORTED when the Krylov
 * dimension (m, or m_max in adaptive mode) exceeds 40. */
int ebtc_plan_backward(ebtc_batch* batch, const ebtc_opts* opts, size_t* ws_bytes);
/* Gradient of L = sum_g <grad_scores_g, S~_g> with respect to every stored CSR entry, with the
 * log-scales held fixed, asynchronous on `stream`:
 *   grad_values[e] = dL/dA_k(i, j) for entry e = (i, j) of realization k,
 *                  ~ e^{-Sigma_g} [int_0^1 e^{sA} g 1^T e^{(1-s)A} ds]_{ij}
 * (Frechet derivative of exp(A) 1, eq. (4), through the sum of eq. (5)). An undirected edge weight
 * that feeds both (i, j) and (j, i) has gradient grad(i, j) + grad(j, i); tying is the caller's.
 * Both exponential actions use their Lanczos approximations: the forward basis is recomputed from
 * scratch with the forward's kernels (bitwise the same: every reduction runs in a fixed order), an
 * adjoint Lanczos starts at the cotangent, the m x m coupling comes from the upper-right block of an
 * FP64 block exponential, and an SDDMM over the CSR pattern forms the entries.
 *   opts         the options of the forward call
 *   log_scale    device [G] double, the forward's Sigma_g
 *   grad_scores  device [sum_g n_g] of dtype, the cotangent of the scores
 *   grad_values  device [nnz_off[R]] of dtype, written
 *   ws, ws_bytes device workspace of at least ebtc_plan_backward's size
 *   ckpt         device [R][2 EBTC_M_LIMIT + 4] doubles (nullable): the forward call's ckpt_out. The
 *                recomputed forward process is compared with it bit for bit (alpha, beta, theta*,
 *                beta0, steps, flags of every realization), which holds exactly when the batch's
 *                values and the options are the forward's
 *   ckpt_mismatch device int32 (required with ckpt): the number of realizations that differ
 * Errors: EINVAL (NULL arguments, ckpt without ckpt_mismatch, bad opts), ENOTSUPPORTED (reorth 0, or
 * a Krylov dimension above the adjoint's), EWORKSPACE, EHIP. */
int ebtc_scores_backward(ebtc_batch* batch, const ebtc_opts* opts, const double* log_scale, const void* grad_scores,
                         void* grad_values, void* ws, size_t ws_bytes, const double* ckpt, int32_t* ckpt_mismatch,
                         void* stream);

/* ---------------------------------------------------------------- selection                      */
/* Device workspace bytes for ebtc_topk (host-only). */
int ebtc_topk_ws_bytes(ebtc_batch* batch, size_t* ws_bytes);
/* K_g largest entries of each graph's score block ("The total communicability": the largest
 * values are the candidates), asynchronous on `stream`.
 *   scores       device [sum_g n_g] of dtype (as written by ebtc_scores)
 *   k_per_graph  host [G], 0 <= K_g <= min(n_g, EBTC_TOPK_LIMIT)
 *   idx_out      device int32 [sum_g K_g]: graph 0's K_0 ids, then graph 1's ...; each block sorted
 *                by descending score, equal scores by ascending node id
 *   val_out      device [sum_g K_g] of dtype, or NULL
 * NaN scores are not supported (ordering undefined). */
int ebtc_topk(ebtc_batch* batch, const void* scores, const int32_t* k_per_graph, int32_t* idx_out,
              void* val_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- component entry points         */
/* y = A x for one CSR matrix (the Krylov step's product), asynchronous. Same CSR rules as a batch;
 * values NULL = all ones; x, y device [n] of dtype, distinct. lanes_per_row / hub_threshold /
 * seg_len as in ebtc_opts (seg_len 0 here means gather without staging). */
int ebtc_spmv(int32_t dtype, int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const void* values,
              const void* x, void* y, int32_t lanes_per_row, int32_t hub_threshold, int32_t seg_len, void* stream);

/* For `count` symmetric tridiagonal matrices of size k (1 <= k <= EBTC_M_LIMIT), FP64, asynchronous:
 * theta_out[c] = largest eigenvalue (0 when shift == 0) and y_out[c*k ..] = exp(T_c - theta I) e1.
 *   alpha  device [count*k] diagonals;  beta device [count*k] off-diagonals (entry i couples rows
 *   i and i+1; entry k-1 of each matrix is ignored). */
int ebtc_tridiag_expv(int32_t count, int32_t k, const double* alpha, const double* beta, double* y_out,
                      double* theta_out, int32_t shift, void* stream);

/* ---------------------------------------------------------------- subgraph centrality            */
/* Subgraph centrality SC(i) = [exp(A)]_ii (eq. 3) of selected nodes of one graph, by the Gauss
 * quadrature rule of the m-step Lanczos process started at e_i: SC(i) ~ e1^T exp(T_m) e1 = e^{theta*}
 * y_0 (theta* = lambda_max(T_m), y = exp(T_m - theta* I) e1 in FP64). The m-point rule bounds SC(i)
 * from below and is exact once the Krylov space of e_i closes (breakdown stops the process there).
 * Every node's process is one realization of a batched launch over the same CSR (stream SpMV form,
 * one classical Gram-Schmidt pass), so the cost is that of `count` realizations of m steps.
 *   dtype, n, row_ptr, col_idx, values  the graph, device CSR as for ebtc_spmv (values NULL = ones)
 *   count, nodes   device int32 [count] node ids; an id outside [0, n) yields NaN
 *   m              Krylov dimension, 1..EBTC_M_LIMIT
 *   sc_out         device double [count]
 *   ws, ws_bytes   device workspace of ebtc_subgraph_centrality_ws_bytes() bytes, 256-byte aligned
 * Synchronises `stream` once (after uploading its task table), then enqueues the rest
 * asynchronously. Errors: EINVAL, EWORKSPACE, ENOTSUPPORTED (too many row blocks), EHIP. */
int ebtc_subgraph_centrality_ws_bytes(int32_t dtype, int32_t n, int32_t count, int32_t m, size_t* ws_bytes);
int ebtc_subgraph_centrality(int32_t dtype, int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                             const void* values, int32_t count, const int32_t* nodes, int32_t m, double* sc_out,
                             void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- autotuning                     */
/* Chooses the batch's SpMV form by timing. Each graph falls in a bucket given by precision, weights,
 * the octave of n, the half-octave of the mean degree, the octave of the largest row over the mean
 * degree (measured on the device) and the octave of the Krylov steps; the sorted list of the batch's
 * buckets is its composition. Unless the composition is in the process-wide cache (ebtc_tune_cache_*),
 * the forms are timed with HIP events on the whole batch: the CSR stream, lane groups of 4, 8, 16 and
 * 32 lanes per row, the LDS-staged form when the largest vector passes through LDS in at most eight
 * segments, the column-segmented form with 6144 and 12288 FP32 (3072 and 6144 FP64) columns when at
 * most 32 segments, the entry-balanced and the paneled form; each form whose plan fits ws_bytes gets
 * its once-per-call preparation, one warm-up and three timed launches of the first Lanczos product.
 * The fastest per launch, with its preparation spread over the call's m steps, is recorded in the
 * cache under the composition and in the batch; later calls with opts->spmv == EBTC_SPMV_AUTO use it
 * (a form named in opts overrides it). Plan the later calls after tuning: the chosen form sets their
 * workspace size. Synchronous on the stream. Overwrites the workspace (the largest ebtc_plan size over
 * the forms to try, 256-byte aligned; forms whose plan does not fit are skipped); not thread-safe with
 * other calls on the same batch.
 *   form_out, lanes_out, seglen_out  host (nullable): the chosen form and its parameters
 *   ms_out  host [EBTC_TUNE_SLOTS] (nullable): ms per launch of stream, lanes 4, 8, 16, 32,
 *           LDS-staged, column-segmented with 6144 and 12288 FP32 (3072 and 6144 FP64) columns per
 *           segment, entry-balanced and paneled, the segmented, balanced and paneled figures with
 *           their preparation spread over the m steps (-1 where the form was not timed, as for a
 *           composition found in the cache)
 * Errors: EINVAL (NULL batch or workspace, bad opts), EWORKSPACE, EHIP. On error the batch keeps its
 * previous choice. */
int ebtc_tune(ebtc_batch* batch, const ebtc_opts* opts, void* ws, size_t ws_bytes, int32_t* form_out,
              int32_t* lanes_out, int32_t* seglen_out, double* ms_out, void* stream);

/* Each graph's SpMV form and parameters as recorded by ebtc_tune (the same for every graph) or
 * ebtc_set_forms (form 0 for every graph when none is recorded).
 *   form_out, lanes_out, seglen_out  host int32 [G] (lanes_out, seglen_out nullable)
 * Errors: EINVAL. */
int ebtc_tuned_forms(ebtc_batch* batch, int32_t* form_out, int32_t* lanes_out, int32_t* seglen_out);

/* Records an SpMV form for every graph for calls with opts->spmv == EBTC_SPMV_AUTO (for callers that
 * know their graphs, or that tuned an equal batch before). One launch sequence runs one form: while
 * the graphs' forms differ, the plan and compute calls with EBTC_SPMV_AUTO refuse the batch with
 * EBTC_ENOTSUPPORTED.
 *   form     host int32 [G]: EBTC_SPMV_STREAM .. EBTC_SPMV_PANELED
 *   lanes    host int32 [G] (nullable = 0): lanes per row of the lane-group form (0 = 8)
 *   seg_len  host int32 [G] (nullable = 0): the form's ebtc_opts::seg_len parameter (0 = default)
 * Errors: EINVAL (NULL batch or form, a form out of range, lanes not 0/4/8/16/32, seg_len < 0). */
int ebtc_set_forms(ebtc_batch* batch, const int32_t* form, const int32_t* lanes, const int32_t* seg_len);

/* The autotuner's process-wide cache of decisions, as text: one line per batch composition (its
 * buckets joined by '+'), "<key> <form> <lanes> <seg_len>". ebtc_tune_cache_get writes it with a
 * terminating NUL into buf
 * (cap bytes; buf NULL: only *len, the text's length without the NUL, is set); ebtc_tune_cache_put
 * merges such text (later lines win; a saved cache restored in a new process skips the timing of the
 * compositions it holds); ebtc_tune_cache_clear empties it. Thread-safe.
 * Errors: EINVAL (NULL len or text, buffer too small, a malformed line: a form outside the enum, lanes
 * other than 0, 4, 8, 16 or 32, a negative seg_len; the whole text is then refused). */
int ebtc_tune_cache_get(char* buf, size_t cap, size_t* len);
int ebtc_tune_cache_put(const char* text);
int ebtc_tune_cache_clear(void);

/* ---------------------------------------------------------------- measurement                    */
enum ebtc_phase {
  EBTC_PHASE_START = 0,      /* start vector and state initialisation                           */
  EBTC_PHASE_SPMV = 1,       /* w = A v_j (with the dots too when the vector is staged in LDS)  */
  EBTC_PHASE_DOTS = 2,       /* partial dots <v_i, w> (both Gram-Schmidt passes)               */
  EBTC_PHASE_UPDATE = 3,     /* Gram-Schmidt update, norm, breakdown test                       */
  EBTC_PHASE_TRIDIAG = 4,    /* FP64 tridiagonal exponential (final and adaptive checks)        */
  EBTC_PHASE_COMBINE = 5,    /* u = beta0 V y                                                    */
  EBTC_PHASE_SUM = 6,        /* realization sum with per-graph log-scale                        */
  EBTC_PHASE_PREPARE = 7,    /* once per call: the column-segment sort of the entries
                                (column-segmented SpMV) or the rows of every share (entry-balanced) */
  EBTC_PHASE_FIRST = 8,      /* step 0's product A 1 of the all-ones start: row sums, no gathers
                                (the entry-balanced form computes a weighted graph's row sums with
                                its own SpMV kernel over the ones, in equal shares of entries)     */
  EBTC_PHASE_SOLVE = 9,      /* the single-kernel schedule's one launch (every phase above from
                                start to combine)                                                 */
  EBTC_PHASE_COUNT = 10
};
/* Measurement only: runs ebtc_scores' batched launch sequence once, eagerly (no hipGraph), with a
 * HIP event recorded on `stream` before and after every kernel launch, then synchronises the
 * stream. Outputs are those of ebtc_scores (ckpt and diag not written).
 *   phase_ms        host [EBTC_PHASE_COUNT]: summed kernel milliseconds per phase (overwritten)
 *   phase_launches  host [EBTC_PHASE_COUNT]: number of launches per phase (overwritten) */
int ebtc_profile_phases(ebtc_batch* batch, const ebtc_opts* opts, void* ws, size_t ws_bytes, void* scores_out,
                        double* log_scale_out, double* phase_ms, int64_t* phase_launches, void* stream);

/* ---------------------------------------------------------------- checking                       */
/* Synchronous structural check of every realization on the device: columns in [0, n), strictly
 * increasing within a row (no duplicates), no self-loops, symmetric pattern, row_ptr monotone from 0.
 * *first_bad = index of the first bad realization, or -1. ws: device, >= ebtc_validate_ws_bytes. */
int ebtc_validate_ws_bytes(ebtc_batch* batch, size_t* ws_bytes);
int ebtc_validate(ebtc_batch* batch, void* ws, size_t ws_bytes, int64_t* first_bad, void* stream);

/* ---------------------------------------------------------------- realization generator          */
/* Background graphs drawn on the device and written as the batch's CSR: the families of the
 * experiments (Introduction, "Multiple backgrounds scenario", "Single background scenario",
 * Tables 1-3), N independent draws on one node set ("Signal processing on graphs"), the target
 * pattern embedded (edges among the target nodes replaced by the pattern). Random numbers:
 * Philox4x32-10 (Salmon et al., SC 2011) keyed by `seed`, counter (c0, c1, realization, family tag),
 * so the result depends only on the spec, never on launch shapes. Definitions:
 *   ER  row i visits j > i by geometric skips j <- j + 1 + floor(ln U / ln(1 - p)), U = (w + 1/2) 2^-32
 *       for the words of counters (i, 0, r, 1), (i, 1, r, 1), ... in order; ln is evaluated with
 *       correctly rounded operations only (frexp, atanh series, no fused multiply-add), so the skips
 *       are reproducible bit for bit on any IEEE machine. Each pair is an edge with probability p.
 *   WS  ring lattice of degree k; lattice edge e = (i, i + 1 + e mod (k/2)), i = e div (k/2), is
 *       rewired iff w0 < floor(beta 2^32) (counter (e, 0, r, 2)) to the far end
 *       (i + 1 + floor(w1 (n - 1) / 2^32)) mod n; coinciding edges are kept once.
 *   BA  seed star on k + 1 nodes; each later node attaches k edges to endpoint slots drawn uniformly
 *       (64-bit, counter (e, 0, r, 3)) from the endpoint list of all earlier edges
 *       (degree-proportional); a node's repeated picks collapse to one edge.
 * Realization r of the call is the spec's realization first + r (counter word 2). */
enum ebtc_gen_family { EBTC_GEN_ER = 0, EBTC_GEN_WS = 1, EBTC_GEN_BA = 2 };

typedef struct {
  int32_t family;         /* enum ebtc_gen_family                                                */
  int32_t n;              /* nodes: ER >= 1; WS >= k + 2; BA >= k + 2                            */
  double p;               /* ER: edge probability in [0, 1]                                      */
  int32_t k;              /* WS: even lattice degree >= 2; BA: edges per new node >= 1            */
  int32_t count;          /* realizations drawn by this call, >= 1                               */
  double beta;            /* WS: rewiring probability in [0, 1]                                  */
  uint64_t seed;          /* Philox key (low word, high word)                                    */
  int64_t first;          /* realization index of the call's first realization; first + count <= 2^32 */
  int32_t t;              /* target nodes, 0 = no target                                         */
  int32_t pattern_edges;  /* edges of the target pattern                                         */
  const int32_t* targets; /* host [t]: distinct node ids in [0, n), in pattern order              */
  const int32_t* pattern; /* host [pattern_edges][2]: local ends a != b in [0, t)                 */
} ebtc_gen_spec;

/* Workspace bytes for one ebtc_generate_count / ebtc_generate_fill pair (host call; needs no device:
 * the sizes, the radix sort's and scan's temporary storage included, follow from the spec alone).
 * Validates the spec: EBTC_EINVAL for out-of-range fields, repeated targets or bad pattern ends; EBTC_ENOTSUPPORTED
 * when the keys (realization, a, b) would not fit 63 bits (count n^2 >= 2^63: draw fewer
 * realizations per call). For G(n, p) the candidate buffer holds the mean edge count plus 8
 * standard deviations per realization. */
int ebtc_generate_plan(const ebtc_gen_spec* spec, size_t* ws_bytes);
/* Draws the spec's realizations, asynchronously on `stream`, and writes their row pointers:
 *   ws        device, >= ebtc_generate_plan bytes; it carries the drawn graphs to ebtc_generate_fill
 *             and must not be reused in between
 *   row_ptr   device int32 [count][n + 1]: realization r's local row pointers (first entry 0)
 *   nnz       device int64 [count]: stored entries of realization r (twice its edges), or -1 if its
 *             draw overflowed the candidate buffer or it would hold 2^31 entries or more
 * The caller reads nnz to size col_idx. Errors: EINVAL, EWORKSPACE, EHIP. */
int ebtc_generate_count(const ebtc_gen_spec* spec, void* ws, size_t ws_bytes, int32_t* row_ptr, int64_t* nnz,
                        void* stream);
/* Writes the columns of the realizations counted by the preceding ebtc_generate_count on the same
 * ws and spec, asynchronously on `stream`:
 *   dest_off  host [count]: offset of realization r's first entry in col_idx
 *   col_idx   device int32: realization r's nnz[r] columns at col_idx[dest_off[r] ...], sorted
 *             within each row, both (i, j) and (j, i) stored, no self-loops
 * Errors: EINVAL, EWORKSPACE, EHIP. */
int ebtc_generate_fill(const ebtc_gen_spec* spec, void* ws, size_t ws_bytes, const int64_t* dest_off,
                       int32_t* col_idx, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* EBTC_H */
