// Host side of the EBTC C ABI: argument checks, workspace layout, launch sequences, hipGraph cache.
#include <algorithm>
#include <array>
#include <map>
#include <sstream>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

using namespace ebtc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

// Error reporting for entry points defined in other translation units.
int ebtc::report_error(int code, const std::string& msg) { return fail(code, msg); }

namespace {

#define EBTC_HIP(call)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return fail(EBTC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// One SpMV form's share of the workspace: its launch's block list (when it covers part of the batch)
// and its arenas, sized for its realizations only.
struct FormLayout {
  int64_t blocks = 0, z = 0;  // row blocks and entries of the form's realizations
  size_t off_sub = 0;         // [blocks] batch-wide block ids (mixed plans only)
  // column-segmented SpMV arenas
  size_t off_segflag = 0, off_segcnt = 0, off_segwoff = 0, off_segblk = 0, off_segcol = 0, off_segval = 0;
  // entry-balanced SpMV arenas
  size_t off_bal = 0, off_balbeg = 0;
  int64_t nbal = 0;  // shares over the form's realizations
  // panel-form arenas
  size_t off_panflag = 0, off_panrun = 0, off_pancol = 0, off_panperm = 0, off_panval = 0, off_panprod = 0,
         off_panitems = 0, off_pangroups = 0;
  int64_t npan_items = 0, npan_groups = 0;
};

// Host tables of one SpMV form (uploaded with every call; kept in the batch for the async copies).
struct FormHost {
  std::vector<int32_t> sub;          // [blocks] the form's row blocks, batch-wide ids (mixed plans only)
  std::vector<int64_t> bal_begin;    // [R + 1] first entry-balanced share of each realization (0 elsewhere)
  std::vector<PanItem> pan_items;    // products-pass work items, realization by realization
  std::vector<int64_t> pan_begin;    // [R + 1] first work item of each realization
  std::vector<PanItem> pan_groups;   // unit groups of the sort's scan, realization by realization
  std::vector<int64_t> pan_gbegin;   // [R + 1] first group of each realization
};

struct Layout {
  int m_slots = 0;
  size_t off_tasks = 0, off_graphs = 0, off_blkmap = 0, off_state = 0, off_part = 0, off_npart = 0, off_V = 0,
         off_W = 0, off_U = 0, off_live = 0;
  std::vector<FormLayout> fl;  // per SpMV form of the plan
  size_t total = 0;
  int64_t total_blocks = 0;
};

struct ExecKey {
  void* ws;
  void* scores;
  double* log_scale;
  void* ckpt;
  ebtc_diag* diag;
  int m, m_max, reorth, shift, sched;
  double tol;
  std::string plan;  // the SpMV plan's signature (forms, parameters, each graph's form)
  bool operator==(const ExecKey& o) const {
    return ws == o.ws && scores == o.scores && log_scale == o.log_scale && ckpt == o.ckpt && diag == o.diag &&
           m == o.m && m_max == o.m_max && reorth == o.reorth && shift == o.shift && sched == o.sched &&
           tol == o.tol && plan == o.plan;
  }
};

struct ExecEntry {
  ExecKey key;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

int elem_size(int dtype) { return dtype == EBTC_F64 ? 8 : 4; }

}  // namespace

struct ebtc_batch {
  int dtype = EBTC_F32;
  int32_t G = 0;
  int64_t R = 0;
  std::vector<int32_t> n, nreal, first;
  std::vector<int64_t> rowptr_off, nnz_off, score_off;
  const int32_t* row_ptr = nullptr;
  const int32_t* col_idx = nullptr;
  const void* values = nullptr;
  int64_t total_scores = 0;  // sum_g n_g
  int64_t total_rows = 0;    // sum_r n_r
  int32_t n_max = 0;
  int64_t z_max = 0;         // largest realization's entry count
  double mean_degree = 0.0;
  std::vector<Task> tasks;          // host staging of the device task table (kept alive for async copies)
  std::vector<GraphInfo> graphs;
  std::vector<int64_t> nnz_r;       // per-realization entry counts (validation upload)
  // host tables of the current SpMV plan's forms (kept alive for async uploads), and the plan they
  // were built for
  std::vector<FormHost> fh;
  std::string fh_sig;
  std::vector<int32_t> topk_k;
  std::vector<int64_t> topk_off;
  std::vector<int32_t> topk_cgraph, topk_cbegin;  // chunked top-K: each chunk's graph, each graph's first chunk
  std::vector<ExecEntry> execs;
  hipStream_t capture_stream = nullptr;
  // SpMV forms chosen by ebtc_tune (empty = not tuned), used when opts->spmv is EBTC_SPMV_AUTO:
  // {form, lanes, seg_len parameter} per form and each graph's form
  std::vector<std::array<int32_t, 3>> tuned;
  std::vector<int32_t> tuned_graph;
};

namespace {

// Chunks of the chunked top-K: kTkChunk scores each, at least one per graph.
int64_t topk_chunks(const ebtc_batch* b) {
  int64_t c = 0;
  for (int32_t g = 0; g < b->G; ++g) c += (b->n[g] + kTkChunk - 1) / kTkChunk;
  return c;
}

int check_opts(const ebtc_opts* o) {
  if (!o) return fail(EBTC_EINVAL, "opts is NULL");
  if (o->m < 0 || o->m > EBTC_M_LIMIT)
    return fail(EBTC_EINVAL, "m must be in [0, " + std::to_string(EBTC_M_LIMIT) + "] (0 = adaptive)");
  if (o->m == 0 && (o->m_max < 1 || o->m_max > EBTC_M_LIMIT))
    return fail(EBTC_EINVAL, "m_max must be in [1, " + std::to_string(EBTC_M_LIMIT) + "]");
  if (o->m == 0 && !(o->tol > 0.0)) return fail(EBTC_EINVAL, "adaptive mode needs tol > 0");
  if (o->reorth < 0 || o->reorth > 2)
    return fail(EBTC_EINVAL, "reorth must be 0 (memory-bounded two-pass), 1 or 2");
  if (o->schedule < EBTC_SCHED_AUTO || o->schedule > EBTC_SCHED_SINGLE) return fail(EBTC_EINVAL, "unknown schedule");
  if (o->spmv < EBTC_SPMV_AUTO || o->spmv > EBTC_SPMV_PANELED) return fail(EBTC_EINVAL, "unknown spmv form");
  if (o->lanes_per_row != 0 && o->lanes_per_row != 4 && o->lanes_per_row != 8 && o->lanes_per_row != 16 &&
      o->lanes_per_row != 32)
    return fail(EBTC_EINVAL, "lanes_per_row must be 0, 4, 8, 16 or 32");
  if (o->hub_threshold < 0) return fail(EBTC_EINVAL, "hub_threshold must be >= 0");
  if (o->seg_len < 0) return fail(EBTC_EINVAL, "seg_len must be >= 0");
  return EBTC_OK;
}

// Schedule of the SpMV for a set of graphs: the form and its parameters.
struct SpmvPlan {
  int form = EBTC_SPMV_STREAM;
  int lanes = 0, hub = 0;
  int seglen = 0;   // LDS-staged: segment length
  int segcols = 0;  // column-segmented: columns per segment
  int smax = 0;     // column-segmented: segments of the largest realization
  int balent = 0;   // entry-balanced: entries per share
  int pancols = 0;  // paneled: columns per panel
  int pmax = 0;     // paneled: panels of the largest realization
  int panunit = 0;  // paneled: rows per unit
  int panlds = 0;   // paneled: entries of a unit held by the row-sum pass
  // the parameter ebtc_opts::seg_len carries for this form
  int param() const {
    return form == EBTC_SPMV_SEGMENTED ? segcols
           : form == EBTC_SPMV_BALANCED ? balent
           : form == EBTC_SPMV_PANELED  ? pancols
                                        : seglen;
  }
};

// The SpMV plan of a batch: one or more forms, each over a set of graphs (every realization of a graph
// takes the graph's form). With several forms each step launches one SpMV per form, over its graphs'
// row blocks; every other phase still runs once over the whole batch.
struct BatchPlan {
  std::vector<SpmvPlan> forms;
  std::vector<int32_t> graph_form;  // [G] index into forms
  bool mixed() const { return forms.size() > 1; }
  std::string sig() const {
    std::string t;
    for (const SpmvPlan& p : forms)
      t += std::to_string(p.form) + "," + std::to_string(p.lanes) + "," + std::to_string(p.hub) + "," +
           std::to_string(p.seglen) + "," + std::to_string(p.segcols) + "," + std::to_string(p.smax) + "," +
           std::to_string(p.balent) + "," + std::to_string(p.pancols) + "," + std::to_string(p.pmax) + "," +
           std::to_string(p.panunit) + "," + std::to_string(p.panlds) + ";";
    if (mixed())
      for (int32_t f : graph_form) t += std::to_string(f) + ",";
    return t;
  }
};

// Graph membership of a form: nullptr = every graph.
using Members = std::vector<char>;
bool member(const Members* m, int32_t g) { return m == nullptr || (*m)[g] != 0; }

std::vector<int64_t> bal_shares(const ebtc_batch* b, int e, const Members* m);

int check_form(const ebtc_batch* b, const SpmvPlan& p, const Members* m) {
  if (p.form == EBTC_SPMV_LANE_GROUPS && p.lanes != 4 && p.lanes != 8 && p.lanes != 16 && p.lanes != 32)
    return fail(EBTC_EINVAL, "the lane-group SpMV takes 4, 8, 16 or 32 lanes per row");
  if (p.form == EBTC_SPMV_BALANCED) {
    if (p.balent < 256 || p.balent > (1 << 24))
      return fail(EBTC_EINVAL, "the entry-balanced SpMV takes shares of 256 to 2^24 entries (seg_len)");
    if (bal_shares(b, p.balent, m).back() > INT32_MAX) return fail(EBTC_EINVAL, "too many entry-balanced shares");
  }
  if (p.form == EBTC_SPMV_PANELED && p.pmax > kPanMaxPanels)
    return fail(EBTC_EINVAL, "the paneled SpMV takes at most " + std::to_string(kPanMaxPanels) + " panels: n " +
                                 std::to_string(p.pmax * (int64_t)p.pancols) + " > " + std::to_string(kPanMaxPanels) +
                                 " x " + std::to_string(p.pancols));
  if (p.form == EBTC_SPMV_SEGMENTED && p.smax > kSegMax)
    return fail(EBTC_EINVAL, "the column-segmented SpMV needs at most " + std::to_string(kSegMax) +
                                 " segments: n " + std::to_string(p.smax * (int64_t)p.segcols) + " > " +
                                 std::to_string(kSegMax) + " x " + std::to_string(p.segcols));
  return EBTC_OK;
}

Members members_of(const BatchPlan& bp, size_t f) {
  Members m(bp.graph_form.size(), 0);
  for (size_t g = 0; g < bp.graph_form.size(); ++g) m[g] = bp.graph_form[g] == (int32_t)f ? 1 : 0;
  return m;
}

int check_plan(const ebtc_batch* b, const BatchPlan& bp) {
  // Several SpMV forms in one launch sequence (one launch per form over its graphs' row blocks) are
  // switched off: a batch of six graphs on six forms did not complete its first eager pass on the
  // GPU, and the cause is not found. The host side (block lists, per-form arenas) stays, and the
  // autotuner decides per batch.
  if (bp.mixed())
    return fail(EBTC_ENOTSUPPORTED, "several SpMV forms in one batch are not supported in this version: record the "
                                    "same form for every graph (or name one in opts->spmv)");
  for (size_t f = 0; f < bp.forms.size(); ++f) {
    const Members m = members_of(bp, f);
    const int rc = check_form(b, bp.forms[f], bp.mixed() ? &m : nullptr);
    if (rc) return rc;
  }
  return EBTC_OK;
}

// First entry-balanced share of each realization ([R + 1]): one share per e entries, at least one
// per realization of a member graph, none for the others.
std::vector<int64_t> bal_shares(const ebtc_batch* b, int e, const Members* m) {
  std::vector<int64_t> v((size_t)b->R + 1, 0);
  int64_t r = 0;
  for (int32_t g = 0; g < b->G; ++g)
    for (int32_t k = 0; k < b->nreal[g]; ++k, ++r) {
      const int64_t z = b->nnz_r[r];
      v[r + 1] = v[r] + (member(m, g) ? std::max<int64_t>(1, (z + e - 1) / e) : 0);
    }
  return v;
}

// Default share size: the largest power of two in [kBalEntriesMin, kBalEntriesMax] that leaves the
// member graphs' realizations at least kBalTargetShares shares.
int bal_default(const ebtc_batch* b, const Members* m) {
  int64_t z = 0, r = 0;
  for (int32_t g = 0; g < b->G; ++g)
    for (int32_t k = 0; k < b->nreal[g]; ++k, ++r)
      if (member(m, g)) z += b->nnz_r[r];
  int e = kBalEntriesMax;
  while (e > kBalEntriesMin && z / e < kBalTargetShares) e >>= 1;
  return e;
}

// The panel form's unit groups and products-pass work items: per member realization, groups of units
// sized so that staging a panel's slice costs at most about a tenth of the product traffic of the
// group's run of that panel (2 + 2 s bytes per entry: column, value, product), halved while the form
// has fewer than 1536 items; items panel by panel, group by group.
void pan_tables(const ebtc_batch* b, int S, int U, const Members* m, FormHost& h) {
  const double es = elem_size(b->dtype);
  auto build = [&](int shrink) {
    h.pan_items.clear();
    h.pan_groups.clear();
    h.pan_begin.assign((size_t)b->R + 1, 0);
    h.pan_gbegin.assign((size_t)b->R + 1, 0);
    int64_t r = 0;
    for (int32_t g = 0; g < b->G; ++g) {
      const int32_t nr = b->n[g];
      const int units = (nr + U - 1) / U, P = (nr + S - 1) / S;
      for (int32_t k = 0; k < b->nreal[g]; ++k, ++r) {
        if (member(m, g)) {
          const double per = std::max(1.0, (double)b->nnz_r[r] / ((double)units * P));  // entries per (unit, panel)
          int gsz = (int)std::ceil(10.0 * S * es / ((2.0 + 2.0 * es) * per));
          gsz = std::max(1, std::min(units, gsz >> shrink));
          const size_t g0 = h.pan_groups.size();
          for (int u0 = 0; u0 < units; u0 += gsz) h.pan_groups.push_back({(int32_t)r, 0, u0, std::min(units, u0 + gsz)});
          for (int p = 0; p < P; ++p)
            for (size_t q = g0; q < h.pan_groups.size(); ++q)
              h.pan_items.push_back({(int32_t)r, p, h.pan_groups[q].b0, h.pan_groups[q].b1});
        }
        h.pan_begin[r + 1] = (int64_t)h.pan_items.size();
        h.pan_gbegin[r + 1] = (int64_t)h.pan_groups.size();
      }
    }
  };
  int shrink = 0;
  build(shrink);
  while (h.pan_items.size() < 1536 && shrink < 16) {
    ++shrink;
    const size_t before = h.pan_items.size();
    build(shrink);
    if (h.pan_items.size() == before) break;
  }
}

// The batch's host tables for plan bp (rebuilt when the plan changes).
const std::vector<FormHost>& form_host(const ebtc_batch* cb, const BatchPlan& bp) {
  ebtc_batch* b = const_cast<ebtc_batch*>(cb);
  const std::string sig = bp.sig();
  if (b->fh_sig == sig && b->fh.size() == bp.forms.size()) return b->fh;
  b->fh.assign(bp.forms.size(), FormHost{});
  for (size_t f = 0; f < bp.forms.size(); ++f) {
    const SpmvPlan& p = bp.forms[f];
    FormHost& h = b->fh[f];
    const Members m = members_of(bp, f);
    const Members* mp = bp.mixed() ? &m : nullptr;
    if (bp.mixed()) {
      int64_t r = 0;
      int32_t blk = 0;
      for (int32_t g = 0; g < b->G; ++g) {
        const int32_t nb = (b->n[g] + kRowsPerBlock - 1) / kRowsPerBlock;
        for (int32_t k = 0; k < b->nreal[g]; ++k, ++r, blk += nb)
          if (member(mp, g))
            for (int32_t i = 0; i < nb; ++i) h.sub.push_back(blk + i);
      }
    }
    if (p.form == EBTC_SPMV_BALANCED) h.bal_begin = bal_shares(b, p.balent, mp);
    if (p.form == EBTC_SPMV_PANELED) pan_tables(b, p.pancols, p.panunit, mp, h);
  }
  b->fh_sig = sig;
  return b->fh;
}

Layout make_layout(const ebtc_batch* b, const ebtc_opts* o, const BatchPlan& bp) {
  Layout L;
  // the memory-bounded form keeps the last three basis vectors only
  L.m_slots = o->reorth == 0 ? 3 : (o->m > 0 ? o->m : o->m_max) + 1;
  const size_t es = elem_size(b->dtype);
  int64_t blocks = 0;
  int64_t rows = 0;
  for (int32_t g = 0; g < b->G; ++g) {
    const int64_t nb = (b->n[g] + kRowsPerBlock - 1) / kRowsPerBlock;
    blocks += nb * b->nreal[g];
    rows += (int64_t)b->n[g] * b->nreal[g];
  }
  L.total_blocks = blocks;
  size_t off = 0;
  L.off_tasks = off;
  off = align_up(off + sizeof(Task) * b->R);
  L.off_graphs = off;
  off = align_up(off + sizeof(GraphInfo) * b->G);
  L.off_blkmap = off;
  off = align_up(off + sizeof(int32_t) * blocks);
  L.off_state = off;
  off = align_up(off + sizeof(RState) * b->R);
  L.off_part = off;
  off = align_up(off + sizeof(double) * kPartStride * blocks);
  L.off_npart = off;
  off = align_up(off + sizeof(double) * blocks);
  L.off_live = off;
  off = align_up(off + sizeof(int32_t) * kMLimit);
  L.off_V = off;
  off = align_up(off + es * (size_t)L.m_slots * rows);
  L.off_W = off;
  off = align_up(off + es * rows);
  L.off_U = off;
  off = align_up(off + es * rows);
  const std::vector<FormHost>& fh = form_host(b, bp);
  for (size_t f = 0; f < bp.forms.size(); ++f) {
    const SpmvPlan& sp = bp.forms[f];
    FormLayout F;
    int64_t r = 0;
    for (int32_t g = 0; g < b->G; ++g) {
      const int64_t nb = (b->n[g] + kRowsPerBlock - 1) / kRowsPerBlock;
      for (int32_t k = 0; k < b->nreal[g]; ++k, ++r)
        if (bp.graph_form[g] == (int32_t)f) {
          F.blocks += nb;
          F.z += b->nnz_r[r];
        }
    }
    const size_t z = (size_t)F.z;
    if (bp.mixed()) {
      F.off_sub = off;
      off = align_up(off + sizeof(int32_t) * (size_t)F.blocks);
    }
    if (sp.form == EBTC_SPMV_SEGMENTED) {
      F.off_segflag = off;
      off = align_up(off + sizeof(int32_t) * F.blocks);
      F.off_segcnt = off;
      off = align_up(off + (size_t)sp.smax * kRowsPerBlock * F.blocks);
      F.off_segwoff = off;
      off = align_up(off + sizeof(uint16_t) * (size_t)sp.smax * 17 * F.blocks);
      F.off_segblk = off;
      off = align_up(off + sizeof(SegBlock) * F.blocks);
      // the entries, the zero padding of every (segment, wave band) run and the rounding of every
      // block's first slot to a multiple of four
      const size_t slots = z + (size_t)F.blocks * kSegSlack + 8;
      F.off_segcol = off;
      off = align_up(off + sizeof(uint16_t) * slots);
      F.off_segval = off;
      if (b->values) off = align_up(off + es * slots);
    }
    if (sp.form == EBTC_SPMV_PANELED) {
      const int64_t units = F.blocks * (kRowsPerBlock / sp.panunit);
      F.npan_items = (int64_t)fh[f].pan_items.size();
      F.npan_groups = (int64_t)fh[f].pan_groups.size();
      F.off_panflag = off;
      off = align_up(off + sizeof(int32_t) * (size_t)units);
      F.off_panrun = off;
      off = align_up(off + sizeof(int2) * (size_t)sp.pmax * (size_t)units);
      F.off_pancol = off;
      off = align_up(off + sizeof(uint16_t) * z);
      F.off_panperm = off;
      off = align_up(off + sizeof(uint16_t) * z);
      F.off_panval = off;
      if (b->values) off = align_up(off + es * z);
      F.off_panprod = off;
      off = align_up(off + es * z);
      F.off_panitems = off;
      off = align_up(off + sizeof(PanItem) * (size_t)F.npan_items);
      F.off_pangroups = off;
      off = align_up(off + sizeof(PanItem) * (size_t)F.npan_groups);
    }
    if (sp.form == EBTC_SPMV_BALANCED) {
      F.nbal = fh[f].bal_begin.back();
      F.off_bal = off;
      off = align_up(off + sizeof(BalPart) * (size_t)F.nbal);
      F.off_balbeg = off;
      off = align_up(off + sizeof(int64_t) * (size_t)(b->R + 1));
    }
    L.fl.push_back(F);
  }
  L.total = off;
  return L;
}

// The task table; each realization's offsets in its form's arenas count the entries and blocks of the
// realizations of the same form before it.
void fill_tables(ebtc_batch* b, const Layout& L, const BatchPlan& bp) {
  b->tasks.resize(b->R);
  int64_t vec = 0, row = 0, part = 0;
  int32_t blk = 0;
  int64_t r = 0;
  std::vector<int64_t> aux_off(bp.forms.size(), 0);
  std::vector<int32_t> aux_blk(bp.forms.size(), 0);
  for (int32_t g = 0; g < b->G; ++g) {
    const int32_t f = bp.graph_form[g];
    for (int32_t k = 0; k < b->nreal[g]; ++k, ++r) {
      Task& t = b->tasks[r];
      const int32_t n = b->n[g];
      const int32_t nb = (n + kRowsPerBlock - 1) / kRowsPerBlock;
      t.rowptr_off = b->rowptr_off[r];
      t.nnz_off = b->nnz_off[r];
      t.vec_off = vec;
      t.w_off = row;
      t.u_off = row;
      t.part_off = part;
      t.n = n;
      t.graph = g;
      t.nblk = nb;
      t.blk_begin = blk;
      t.aux_off = aux_off[f];
      t.aux_blk = aux_blk[f];
      t.form = f;
      aux_off[f] += b->nnz_r[r];
      aux_blk[f] += nb;
      vec += (int64_t)L.m_slots * n;
      row += n;
      part += (int64_t)nb * kPartStride;
      blk += nb;
    }
  }
}

int upload_tables(ebtc_batch* b, char* ws, const Layout& L, const BatchPlan& bp, hipStream_t s) {
  fill_tables(b, L, bp);
  const std::vector<FormHost>& fh = form_host(b, bp);
  EBTC_HIP(hipMemcpyAsync(ws + L.off_tasks, b->tasks.data(), sizeof(Task) * b->R, hipMemcpyHostToDevice, s));
  EBTC_HIP(hipMemcpyAsync(ws + L.off_graphs, b->graphs.data(), sizeof(GraphInfo) * b->G, hipMemcpyHostToDevice, s));
  for (size_t f = 0; f < bp.forms.size(); ++f) {
    const FormLayout& F = L.fl[f];
    if (bp.mixed() && F.blocks > 0)
      EBTC_HIP(hipMemcpyAsync(ws + F.off_sub, fh[f].sub.data(), sizeof(int32_t) * (size_t)F.blocks,
                              hipMemcpyHostToDevice, s));
    if (F.npan_items > 0) {
      EBTC_HIP(hipMemcpyAsync(ws + F.off_panitems, fh[f].pan_items.data(), sizeof(PanItem) * (size_t)F.npan_items,
                              hipMemcpyHostToDevice, s));
      EBTC_HIP(hipMemcpyAsync(ws + F.off_pangroups, fh[f].pan_groups.data(),
                              sizeof(PanItem) * (size_t)F.npan_groups, hipMemcpyHostToDevice, s));
    }
    if (bp.forms[f].form == EBTC_SPMV_BALANCED)
      EBTC_HIP(hipMemcpyAsync(ws + F.off_balbeg, fh[f].bal_begin.data(), sizeof(int64_t) * (b->R + 1),
                              hipMemcpyHostToDevice, s));
  }
  return EBTC_OK;
}

// One form over the member graphs (nullptr: all); the parameters follow the largest member.
SpmvPlan spmv_form(const ebtc_batch* b, int form, int lanes, int seg_len, int hub, const Members* m = nullptr) {
  SpmvPlan p;
  p.form = form;
  int32_t n_max = 1;
  double deg = 0.0;  // the densest member realization's mean degree
  {
    int64_t r = 0;
    for (int32_t g = 0; g < b->G; ++g)
      for (int32_t k = 0; k < b->nreal[g]; ++k, ++r)
        if (member(m, g)) {
          n_max = std::max(n_max, b->n[g]);
          deg = std::max(deg, (double)b->nnz_r[r] / std::max(1, b->n[g]));
        }
  }
  if (form == EBTC_SPMV_LANE_GROUPS) p.lanes = lanes ? lanes : 8;
  if (form == EBTC_SPMV_LDS_STAGED) {
    const int maxseg = staged_max_seglen(b->dtype);
    p.seglen = seg_len > 0 ? std::min(seg_len, maxseg) : maxseg;
  }
  if (form == EBTC_SPMV_SEGMENTED) {
    p.segcols = std::min(seg_len > 0 ? seg_len : seg_max_cols(b->dtype), seg_max_cols(b->dtype));
    p.smax = (n_max + p.segcols - 1) / p.segcols;
  }
  if (form == EBTC_SPMV_BALANCED) p.balent = seg_len > 0 ? seg_len : bal_default(b, m);
  if (form == EBTC_SPMV_PANELED) {
    p.pancols = std::min(seg_len > 0 ? seg_len : pan_max_cols(b->dtype), pan_max_cols(b->dtype));
    p.pmax = (n_max + p.pancols - 1) / p.pancols;
    // units: the most rows (256, 128 or 64) whose entries, at 1.5 times the densest realization's mean
    // degree, fit the stream arithmetic's LDS buffer, which the row-sum pass holds anyway; the budget
    // is that buffer, or 1.5 times a 64-row unit's mean entries when even those do not fit
    const int cap = stream_cap(b->dtype);
    p.panunit = 256;
    while (p.panunit > 64 && p.panunit * deg * 1.5 > cap) p.panunit >>= 1;
    const double need = std::ceil(p.panunit * deg * 1.5 / 256.0) * 256.0;
    p.panlds = (int)std::min<double>(pan_max_lds(b->dtype), std::max<double>(cap, need));
  }
  p.hub = hub ? hub : 16 * (p.lanes ? p.lanes : 8);
  return p;
}

BatchPlan one_form(const ebtc_batch* b, const SpmvPlan& p) {
  BatchPlan bp;
  bp.forms.push_back(p);
  bp.graph_form.assign((size_t)b->G, 0);
  return bp;
}

// The CSR-stream form unless the caller names one or ebtc_tune measured others on this batch.
BatchPlan spmv_plan(const ebtc_batch* b, const ebtc_opts* o) {
  if (o->spmv != EBTC_SPMV_AUTO)
    return one_form(b, spmv_form(b, o->spmv, o->lanes_per_row, o->seg_len, o->hub_threshold));
  if (b->tuned.empty()) return one_form(b, spmv_form(b, EBTC_SPMV_STREAM, 0, 0, o->hub_threshold));
  BatchPlan bp;
  bp.graph_form = b->tuned_graph;
  for (size_t f = 0; f < b->tuned.size(); ++f) {
    const Members m = members_of(bp, f);
    bp.forms.push_back(spmv_form(b, b->tuned[f][0], b->tuned[f][1], b->tuned[f][2], o->hub_threshold,
                                 b->tuned.size() > 1 ? &m : nullptr));
  }
  return bp;
}

LzArgs make_args(const ebtc_batch* b, const ebtc_opts* o, char* ws, const Layout& L) {
  LzArgs a{};
  a.row_ptr = b->row_ptr;
  a.col_idx = b->col_idx;
  a.values = b->values;
  a.tasks = (const Task*)(ws + L.off_tasks);
  a.blkmap = (const int32_t*)(ws + L.off_blkmap);
  a.sub_blocks = nullptr;
  a.single_task = 0;
  a.hub_threshold = 128;
  a.state = (RState*)(ws + L.off_state);
  a.V = ws + L.off_V;
  a.W = ws + L.off_W;
  a.U = ws + L.off_U;
  a.part = (double*)(ws + L.off_part);
  a.npart = (double*)(ws + L.off_npart);
  a.m_fixed = o->m;
  a.m_max = o->m > 0 ? o->m : o->m_max;
  a.eps = b->dtype == EBTC_F64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
  a.window = o->reorth == 0 ? 2 : 0;
  a.stop_mused = 0;
  a.live = nullptr;
  return a;
}

// One SpMV launch's arguments: the base arguments plus one form's fields.
struct FArgs {
  LzArgs a;
  SpmvPlan sp;
  int64_t nb = 0;  // row blocks the launch covers (batched schedule)
};

std::vector<FArgs> form_args(const ebtc_batch* b, const LzArgs& base, char* ws, const Layout& L, const BatchPlan& bp) {
  std::vector<FArgs> out;
  for (size_t f = 0; f < bp.forms.size(); ++f) {
    const SpmvPlan& sp = bp.forms[f];
    const FormLayout& F = L.fl[f];
    FArgs x;
    x.sp = sp;
    x.nb = F.blocks;
    LzArgs& a = x.a;
    a = base;
    a.sub_blocks = bp.mixed() ? (const int32_t*)(ws + F.off_sub) : nullptr;
    a.hub_threshold = sp.hub;
    a.seglen = sp.seglen;
    // the column-segmented sort of weighted graphs also writes step 0's product
    a.first_in_prepare = base.unit_start && sp.form == EBTC_SPMV_SEGMENTED && b->values != nullptr ? 1 : 0;
    if (sp.form == EBTC_SPMV_SEGMENTED) {
      a.seg_cols = sp.segcols;
      a.seg_stride = sp.smax * kRowsPerBlock;
      a.seg_flag = (int32_t*)(ws + F.off_segflag);
      a.seg_cnt = (uint8_t*)(ws + F.off_segcnt);
      a.seg_woff = (uint16_t*)(ws + F.off_segwoff);
      a.seg_wstride = sp.smax * 17;
      a.seg_blk = (SegBlock*)(ws + F.off_segblk);
      a.seg_col = (uint16_t*)(ws + F.off_segcol);
      a.seg_val = b->values ? (void*)(ws + F.off_segval) : nullptr;
      // 16-byte slice stores need every slice length to be a whole number of vectors: n and the
      // segment length multiples of the vector width (else a store would pass the slice's end, into
      // the other LDS buffer)
      const int vw = 16 / elem_size(b->dtype);
      a.seg_vec = sp.segcols % vw == 0 ? 1 : 0;
      for (int32_t g = 0; g < b->G; ++g)
        if (bp.graph_form[g] == (int32_t)f && b->n[g] % vw != 0) a.seg_vec = 0;
    }
    if (sp.form == EBTC_SPMV_PANELED) {
      a.pan_cols = sp.pancols;
      a.pan_pmax = sp.pmax;
      a.pan_unit = sp.panunit;
      a.pan_lds = sp.panlds;
      a.pan_flag = (int32_t*)(ws + F.off_panflag);
      a.pan_run = (int2*)(ws + F.off_panrun);
      a.pan_col = (uint16_t*)(ws + F.off_pancol);
      a.pan_perm = (uint16_t*)(ws + F.off_panperm);
      a.pan_val = b->values ? (void*)(ws + F.off_panval) : nullptr;
      a.pan_prod = ws + F.off_panprod;
      a.pan_items = (const PanItem*)(ws + F.off_panitems);
      a.pan_nitems = (int32_t)F.npan_items;
      a.pan_groups = (const PanItem*)(ws + F.off_pangroups);
    }
    if (sp.form == EBTC_SPMV_BALANCED) {
      a.bal = (BalPart*)(ws + F.off_bal);
      a.bal_begin = (const int64_t*)(ws + F.off_balbeg);
      a.nbal = (int32_t)F.nbal;
      a.bal_entries = sp.balent;
    }
    out.push_back(x);
  }
  return out;
}

// The same launch restricted to one realization (the plain schedule).
FArgs one_task(const ebtc_batch* b, const FArgs& x, size_t f, int64_t r) {
  FArgs y = x;
  y.a.single_task = (int32_t)r;
  y.a.blkmap = nullptr;
  y.a.sub_blocks = nullptr;
  y.nb = b->tasks[r].nblk;
  const FormHost& h = b->fh[f];
  if (y.a.bal != nullptr) y.a.nbal = (int32_t)(h.bal_begin[r + 1] - h.bal_begin[r]);
  if (y.a.pan_cols > 0) {
    y.a.pan_items = x.a.pan_items + h.pan_begin[r];
    y.a.pan_nitems = (int32_t)(h.pan_begin[r + 1] - h.pan_begin[r]);
  }
  return y;
}

// The autotuner's decisions, process-wide: bucket key -> {form, lanes, seg_len parameter}.
std::mutex g_tune_mu;
std::map<std::string, std::array<int32_t, 3>> g_tune_cache;

// A graph's autotuning bucket: precision, weights, octave of n, half-octave of the mean degree, octave
// of the largest row over the mean degree (hub rows), octave of the Krylov steps (which spread the
// once-per-call preparations).
std::string tune_key(int dtype, bool has_val, int32_t n, double mean_deg, int32_t row_max, int steps) {
  const int nl = (int)std::floor(std::log2(std::max(1, n)));
  const int dl = (int)std::floor(2.0 * std::log2(std::max(1.0, mean_deg)));
  const int hl = (int)std::floor(std::log2(std::max(1.0, row_max / std::max(1.0, mean_deg))));
  const int sl = (int)std::floor(std::log2(std::max(1, steps)));
  return std::string(dtype == EBTC_F64 ? "f64" : "f32") + (has_val ? "v" : "p") + "-n" + std::to_string(nl) + "-d" +
         std::to_string(dl) + "-h" + std::to_string(hl) + "-s" + std::to_string(sl);
}

// Kernel opt-ins to the full LDS; once per process, before any stream capture.
int prepare_kernels(const BatchPlan& bp) {
  for (const SpmvPlan& sp : bp.forms) {
    if (sp.seglen > 0) EBTC_HIP(prepare_staged_kernels());
    if (sp.segcols > 0) EBTC_HIP(prepare_seg_kernels());
    if (sp.pancols > 0) EBTC_HIP(prepare_pan_kernels());
  }
  EBTC_HIP(prepare_solve_kernels());
  return EBTC_OK;
}

// Optional per-launch event recording (ebtc_profile_phases).
struct Prof {
  struct Rec {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  hipStream_t s;
  int before(int phase) {
    Rec r{phase, nullptr, nullptr};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return EBTC_EHIP;
    recs.push_back(r);
    return hipEventRecord(r.a, s) == hipSuccess ? EBTC_OK : EBTC_EHIP;
  }
  int after() { return hipEventRecord(recs.back().b, s) == hipSuccess ? EBTC_OK : EBTC_EHIP; }
  ~Prof() {
    for (auto& r : recs) {
      if (r.a) (void)hipEventDestroy(r.a);
      if (r.b) (void)hipEventDestroy(r.b);
    }
  }
};

#define EBTC_LAUNCH(call)                                                                              \
  do {                                                                                                 \
    hipError_t e_ = (call);                                                                            \
    if (e_ != hipSuccess) return fail(EBTC_EHIP, std::string("launch ") + #call + ": " + hipGetErrorString(e_)); \
  } while (0)

#define EBTC_PHASE(prof, phase, call)                                                   \
  do {                                                                                  \
    if (prof && prof->before(phase)) return fail(EBTC_EHIP, "event record failed");    \
    EBTC_LAUNCH(call);                                                                  \
    if (prof && prof->after()) return fail(EBTC_EHIP, "event record failed");          \
  } while (0)

// Whether the single-kernel schedule can run this batch: one row block per realization, the whole
// basis with one Gram-Schmidt pass, and an SpMV form whose arithmetic is the CSR stream's (the
// single-kernel solve computes those bits).
bool single_ok(const ebtc_batch* b, const ebtc_opts* o) {
  const bool stream_bits = o->spmv == EBTC_SPMV_AUTO || o->spmv == EBTC_SPMV_STREAM ||
                           o->spmv == EBTC_SPMV_SEGMENTED || o->spmv == EBTC_SPMV_BALANCED;
  const int steps = o->m > 0 ? o->m : o->m_max;
  return b->n_max <= kRowsPerBlock && o->reorth == 1 && stream_bits && steps <= kDotsWindow;
}

// The schedule a call runs: AUTO takes the single-kernel form where it applies.
int resolve_schedule(const ebtc_batch* b, const ebtc_opts* o, int* sched) {
  *sched = o->schedule;
  if (*sched == EBTC_SCHED_AUTO) *sched = single_ok(b, o) ? EBTC_SCHED_SINGLE : EBTC_SCHED_BATCHED;
  if (*sched == EBTC_SCHED_SINGLE && !single_ok(b, o))
    return fail(EBTC_ENOTSUPPORTED, "the single-kernel schedule needs every n <= " + std::to_string(kRowsPerBlock) +
                                        ", m (or m_max) <= " + std::to_string(kDotsWindow) +
                                        ", reorth = 1 and the stream, segmented, balanced or auto SpMV form");
  return EBTC_OK;
}

// Lanczos steps for the launches described by (a, nblocks); a.blkmap / a.single_task select the scope.
// fa: the SpMV launches of each step, one per form of the plan.
int run_steps(const ebtc_batch* b, const ebtc_opts* o, const LzArgs& a, const std::vector<FArgs>& fa, int64_t nblocks,
              int64_t first, int64_t count, hipStream_t s, Prof* prof, bool with_start = true) {
  const bool has_val = b->values != nullptr;
  const int steps = o->m > 0 ? o->m : o->m_max;
  // every realization in one row block: dots and update of a step in one launch (one workgroup each)
  const bool one_block = b->n_max <= kRowsPerBlock && o->reorth == 1 && a.window == 0 && steps <= kDotsWindow;
  if (with_start) EBTC_PHASE(prof, EBTC_PHASE_START, launch_start(b->dtype, a, nblocks, s));
  for (int j = 0; j < steps; ++j) {
    for (const FArgs& x : fa) {
      if (x.nb == 0 || (j == 0 && x.a.unit_start && x.a.first_in_prepare)) continue;
      EBTC_PHASE(prof, j == 0 && x.a.unit_start ? EBTC_PHASE_FIRST : EBTC_PHASE_SPMV,
                 launch_spmv_step(b->dtype, has_val, x.sp.lanes, j, x.a, x.nb, s));
    }
    if (one_block) {
      EBTC_PHASE(prof, EBTC_PHASE_DOTS, launch_dots_update_1(b->dtype, j, a, nblocks, s));
    } else if (o->reorth == 2) {
      EBTC_PHASE(prof, EBTC_PHASE_DOTS, launch_dots_step(b->dtype, j, a, nblocks, s));
      EBTC_PHASE(prof, EBTC_PHASE_UPDATE, launch_update(b->dtype, j, true, false, false, a, nblocks, s));
      EBTC_PHASE(prof, EBTC_PHASE_DOTS, launch_dots_again(b->dtype, j, a, nblocks, s));
      EBTC_PHASE(prof, EBTC_PHASE_UPDATE, launch_update(b->dtype, j, false, true, true, a, nblocks, s));
    } else {
      EBTC_PHASE(prof, EBTC_PHASE_DOTS, launch_dots_step(b->dtype, j, a, nblocks, s));
      EBTC_PHASE(prof, EBTC_PHASE_UPDATE, launch_update(b->dtype, j, true, true, false, a, nblocks, s));
    }
    if (o->m == 0)
      EBTC_PHASE(prof, EBTC_PHASE_TRIDIAG,
                 launch_tridiag_state(a, first, count, 1, j, steps, o->shift, o->tol, nullptr, nullptr, s));
  }
  return EBTC_OK;
}

// The once-per-call preparation of one form's launch: the column-segmented sort, the entry-balanced
// shares or the panel order (nothing for the other forms). f: the form's index in the plan.
int enqueue_prepare(const ebtc_batch* b, const FArgs& x, size_t f, hipStream_t s, Prof* prof) {
  const LzArgs& a = x.a;
  if (x.nb == 0) return EBTC_OK;
  if (x.sp.form == EBTC_SPMV_BALANCED) {
    const bool one = a.blkmap == nullptr;  // the plain schedule: one realization
    EBTC_PHASE(prof, EBTC_PHASE_PREPARE, launch_bal_rows(a, one ? a.single_task : 0, one ? 1 : (int)b->R, s));
    return EBTC_OK;
  }
  if (x.sp.form == EBTC_SPMV_PANELED) {
    const FormHost& h = b->fh[f];
    const bool one = a.blkmap == nullptr;
    const int64_t g0 = one ? h.pan_gbegin[a.single_task] : 0;
    const int64_t g1 = one ? h.pan_gbegin[a.single_task + 1] : h.pan_gbegin[b->R];
    EBTC_PHASE(prof, EBTC_PHASE_PREPARE,
               launch_pan_prepare(b->dtype, b->values != nullptr, a, x.nb, a.pan_groups + g0, (int)(g1 - g0), s));
    return EBTC_OK;
  }
  if (x.sp.form != EBTC_SPMV_SEGMENTED) return EBTC_OK;
  EBTC_PHASE(prof, EBTC_PHASE_PREPARE, launch_seg_prepare(b->dtype, b->values != nullptr, a, x.nb, x.sp.smax, s));
  return EBTC_OK;
}

int enqueue_prepare_all(const ebtc_batch* b, const std::vector<FArgs>& fa, hipStream_t s, Prof* prof) {
  for (size_t f = 0; f < fa.size(); ++f) {
    const int rc = enqueue_prepare(b, fa[f], f, s, prof);
    if (rc) return rc;
  }
  return EBTC_OK;
}

// Second pass of the memory-bounded form (reorth 0): the first pass kept only a ring of three basis
// vectors, so u = beta0 V y is accumulated while the same kernels regenerate the same basis (same
// launches in the same order: bitwise the same vectors), one term before each step.
int run_pass2(const ebtc_batch* b, const ebtc_opts* o, const LzArgs& a1, const std::vector<FArgs>& fa1,
              int64_t nblocks, hipStream_t s, Prof* prof) {
  LzArgs a = a1;
  a.stop_mused = 1;
  a.live = nullptr;  // the live counts belong to the first pass
  std::vector<FArgs> fa = fa1;
  for (FArgs& x : fa) {
    x.a.stop_mused = 1;
    x.a.live = nullptr;
  }
  const bool has_val = b->values != nullptr;
  const int steps = o->m > 0 ? o->m : o->m_max;
  EBTC_PHASE(prof, EBTC_PHASE_START, launch_restart(b->dtype, a, nblocks, s));
  for (int j = 0; j < steps; ++j) {
    EBTC_PHASE(prof, EBTC_PHASE_COMBINE, launch_accum(b->dtype, a, j, nblocks, s));
    if (j + 1 == steps) break;  // the last vector needed is v_{steps-1}
    for (const FArgs& x : fa) {
      if (x.nb == 0) continue;
      // the second pass never skips step 0: the sort's product of the first pass is gone
      LzArgs xa = x.a;
      xa.first_in_prepare = 0;
      EBTC_PHASE(prof, j == 0 && xa.unit_start ? EBTC_PHASE_FIRST : EBTC_PHASE_SPMV,
                 launch_spmv_step(b->dtype, has_val, x.sp.lanes, j, xa, x.nb, s));
    }
    EBTC_PHASE(prof, EBTC_PHASE_DOTS, launch_dots_step(b->dtype, j, a, nblocks, s));
    EBTC_PHASE(prof, EBTC_PHASE_UPDATE, launch_update(b->dtype, j, true, true, false, a, nblocks, s));
  }
  return EBTC_OK;
}

int enqueue_batched(ebtc_batch* b, const ebtc_opts* o, char* ws, const Layout& L, const BatchPlan& bp, void* scores,
                    double* log_scale, void* ckpt, ebtc_diag* diag, int sched, hipStream_t s, Prof* prof = nullptr) {
  LzArgs a = make_args(b, o, ws, L);
  a.unit_start = 1;  // k_start (and k_restart) set v_0 = 1
  a.diag = diag;
  // adaptive m: the checks count the realizations still running, and once none is, the launches of
  // the remaining steps up to the cap return at once
  if (o->m == 0 && sched != EBTC_SCHED_SINGLE) a.live = (int32_t*)(ws + L.off_live);
  const std::vector<FArgs> fa = form_args(b, a, ws, L, bp);
  EBTC_LAUNCH(launch_blkmap(a.tasks, b->R, (int32_t*)(ws + L.off_blkmap), s));
  const int32_t maxblk = (b->n_max + kRowsPerBlock - 1) / kRowsPerBlock;
  if (sched == EBTC_SCHED_SINGLE) {
    EBTC_PHASE(prof, EBTC_PHASE_SOLVE,
               launch_solve_1(b->dtype, b->values != nullptr, a, b->R, o->m > 0 ? o->m : o->m_max, o->shift, o->tol,
                              diag, (double*)ckpt, b->n_max, b->z_max, s));
    EBTC_PHASE(prof, EBTC_PHASE_SUM, launch_sum(b->dtype, (const GraphInfo*)(ws + L.off_graphs), b->G, maxblk,
                                                a.tasks, a.state, a.U, scores, log_scale, s));
    return EBTC_OK;
  }
  int rc = enqueue_prepare_all(b, fa, s, prof);
  if (rc) return rc;
  rc = run_steps(b, o, a, fa, L.total_blocks, 0, b->R, s, prof);
  if (rc) return rc;
  const int steps = o->m > 0 ? o->m : o->m_max;
  EBTC_PHASE(prof, EBTC_PHASE_TRIDIAG,
             launch_tridiag_state(a, 0, b->R, 0, 0, steps, o->shift, o->tol, diag, (double*)ckpt, s));
  if (o->reorth == 0) {
    rc = run_pass2(b, o, a, fa, L.total_blocks, s, prof);
    if (rc) return rc;
  } else {
    EBTC_PHASE(prof, EBTC_PHASE_COMBINE, launch_combine(b->dtype, a, L.total_blocks, s));
  }
  EBTC_PHASE(prof, EBTC_PHASE_SUM, launch_sum(b->dtype, (const GraphInfo*)(ws + L.off_graphs), b->G, maxblk, a.tasks,
                                              a.state, a.U, scores, log_scale, s));
  return EBTC_OK;
}

int enqueue_plain(ebtc_batch* b, const ebtc_opts* o, char* ws, const Layout& L, const BatchPlan& bp, void* scores,
                  double* log_scale, void* ckpt, ebtc_diag* diag, hipStream_t s) {
  LzArgs a = make_args(b, o, ws, L);
  a.unit_start = 1;
  a.blkmap = nullptr;
  a.diag = diag;
  const std::vector<FArgs> fa = form_args(b, a, ws, L, bp);
  for (int64_t r = 0; r < b->R; ++r) {
    a.single_task = (int32_t)r;
    const size_t f = (size_t)bp.graph_form[b->tasks[r].graph];
    const std::vector<FArgs> fr{one_task(b, fa[f], f, r)};
    const int64_t nb = b->tasks[r].nblk;
    int rc = enqueue_prepare(b, fr[0], f, s, nullptr);
    if (rc) return rc;
    rc = run_steps(b, o, a, fr, nb, r, 1, s, nullptr);
    if (rc) return rc;
    EBTC_LAUNCH(launch_tridiag_state(a, r, 1, 0, 0, o->m > 0 ? o->m : o->m_max, o->shift, o->tol, diag,
                                     (double*)ckpt, s));
    if (o->reorth == 0) {
      rc = run_pass2(b, o, a, fr, nb, s, nullptr);
      if (rc) return rc;
    } else {
      EBTC_LAUNCH(launch_combine(b->dtype, a, nb, s));
    }
  }
  const int32_t maxblk = (b->n_max + kRowsPerBlock - 1) / kRowsPerBlock;
  EBTC_LAUNCH(launch_sum(b->dtype, (const GraphInfo*)(ws + L.off_graphs), b->G, maxblk, a.tasks, a.state, a.U, scores,
                         log_scale, s));
  return EBTC_OK;
}

}  // namespace

namespace {

// Backward workspace: the forward layout (recomputed forward), then the adjoint Lanczos state and
// basis, the per-realization block exponentials and the node-major Z and normalised V.
struct BwdLayout {
  Layout fwd;
  size_t off_astate = 0, off_aV = 0, off_X = 0, off_Z = 0, off_Vn = 0, total = 0;
  int ld = 0;
};

BwdLayout make_bwd_layout(const ebtc_batch* b, const ebtc_opts* o) {
  BwdLayout B;
  B.fwd = make_layout(b, o, spmv_plan(b, o));
  const size_t es = elem_size(b->dtype);
  const int steps = o->m > 0 ? o->m : o->m_max;
  B.ld = (steps + 7) / 8 * 8;
  size_t off = B.fwd.total;
  B.off_astate = off;
  off = align_up(off + sizeof(RState) * b->R);
  B.off_aV = off;
  off = align_up(off + es * (size_t)B.fwd.m_slots * b->total_rows);
  B.off_X = off;
  off = align_up(off + sizeof(double) * kXLd * kXLd * b->R);
  B.off_Z = off;
  off = align_up(off + es * (size_t)B.ld * b->total_rows);
  B.off_Vn = off;
  off = align_up(off + es * (size_t)B.ld * b->total_rows);
  B.total = off;
  return B;
}

int check_bwd_opts(const ebtc_opts* o) {
  int rc = check_opts(o);
  if (rc) return rc;
  const int steps = o->m > 0 ? o->m : o->m_max;
  if (o->reorth == 0)
    return fail(EBTC_ENOTSUPPORTED, "the adjoint needs the stored basis: reorth 1 or 2");
  if (steps > adjoint_max_m())
    return fail(EBTC_ENOTSUPPORTED, "the adjoint supports Krylov dimensions up to " + std::to_string(adjoint_max_m()));
  return EBTC_OK;
}

}  // namespace

extern "C" {

int ebtc_version(int* major, int* minor) {
  if (!major || !minor) return fail(EBTC_EINVAL, "NULL output pointer");
  *major = EBTC_VERSION_MAJOR;
  *minor = EBTC_VERSION_MINOR;
  return EBTC_OK;
}

const char* ebtc_status_str(int status) {
  switch (status) {
    case EBTC_OK: return "ok";
    case EBTC_EINVAL: return "invalid argument";
    case EBTC_EBADGRAPH: return "bad graph batch";
    case EBTC_EWORKSPACE: return "workspace too small";
    case EBTC_EHIP: return "HIP runtime error";
    case EBTC_ENOTSUPPORTED: return "not supported";
    default: return "unknown status";
  }
}

const char* ebtc_last_error(void) { return g_err.c_str(); }

void ebtc_default_opts(ebtc_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->m = 30;
  o->m_max = 60;
  o->tol = 1e-6;
  o->reorth = 1;
  o->schedule = EBTC_SCHED_AUTO;
  o->use_hipgraph = 1;
  o->shift = 1;
  o->spmv = EBTC_SPMV_AUTO;
  o->lanes_per_row = 0;
  o->hub_threshold = 0;
  o->seg_len = 0;
}

int ebtc_batch_create(const ebtc_batch_desc* d, ebtc_batch** out) {
  g_err.clear();
  if (!d || !out) return fail(EBTC_EINVAL, "NULL descriptor or output");
  if (d->dtype != EBTC_F32 && d->dtype != EBTC_F64) return fail(EBTC_EINVAL, "dtype must be EBTC_F32 or EBTC_F64");
  if (d->num_graphs < 1) return fail(EBTC_EINVAL, "num_graphs must be >= 1");
  if (d->num_realizations < 1 || d->num_realizations >= (int64_t)1 << 31)
    return fail(EBTC_EINVAL, "num_realizations must be in [1, 2^31)");
  if (!d->graph_n || !d->graph_nreal || !d->rowptr_off || !d->nnz_off)
    return fail(EBTC_EINVAL, "NULL host array in the descriptor");
  if (!d->row_ptr || !d->col_idx) return fail(EBTC_EINVAL, "NULL device row_ptr or col_idx");
  ebtc_batch* b = new ebtc_batch();
  b->dtype = d->dtype;
  b->G = d->num_graphs;
  b->R = d->num_realizations;
  // the per-realization arrays are read only after R has been checked against graph_nreal, so an
  // inconsistent count is reported instead of read past the caller's arrays
  b->n.assign(d->graph_n, d->graph_n + b->G);
  b->nreal.assign(d->graph_nreal, d->graph_nreal + b->G);
  b->row_ptr = d->row_ptr;
  b->col_idx = d->col_idx;
  b->values = d->values;
  int64_t sum_real = 0, blocks = 0;
  b->first.resize(b->G);
  b->score_off.resize(b->G + 1);
  b->score_off[0] = 0;
  for (int32_t g = 0; g < b->G; ++g) {
    if (b->n[g] < 1) {
      delete b;
      return fail(EBTC_EINVAL, "graph " + std::to_string(g) + ": n must be >= 1");
    }
    if (b->nreal[g] < 1) {
      delete b;
      return fail(EBTC_EINVAL, "graph " + std::to_string(g) + ": realizations must be >= 1");
    }
    b->first[g] = (int32_t)sum_real;
    sum_real += b->nreal[g];
    b->score_off[g + 1] = b->score_off[g] + b->n[g];
    b->n_max = std::max(b->n_max, b->n[g]);
    b->total_rows += (int64_t)b->n[g] * b->nreal[g];
    blocks += (int64_t)((b->n[g] + kRowsPerBlock - 1) / kRowsPerBlock) * b->nreal[g];
  }
  if (sum_real != b->R) {
    delete b;
    return fail(EBTC_EBADGRAPH, "num_realizations differs from the sum of graph_nreal");
  }
  b->rowptr_off.assign(d->rowptr_off, d->rowptr_off + b->R);
  b->nnz_off.assign(d->nnz_off, d->nnz_off + b->R + 1);
  if (blocks >= (int64_t)1 << 31) {
    delete b;
    return fail(EBTC_ENOTSUPPORTED, "too many row blocks for one launch");
  }
  if (b->nnz_off[0] != 0) {
    delete b;
    return fail(EBTC_EBADGRAPH, "nnz_off[0] must be 0");
  }
  b->nnz_r.resize(b->R);
  int64_t r = 0;
  for (int32_t g = 0; g < b->G; ++g) {
    for (int32_t k = 0; k < b->nreal[g]; ++k, ++r) {
      const int64_t z = b->nnz_off[r + 1] - b->nnz_off[r];
      if (z < 0 || z >= (int64_t)1 << 31) {
        delete b;
        return fail(EBTC_EBADGRAPH, "realization " + std::to_string(r) + ": entry count out of range");
      }
      if (b->rowptr_off[r] < 0) {
        delete b;
        return fail(EBTC_EBADGRAPH, "realization " + std::to_string(r) + ": negative rowptr_off");
      }
      b->nnz_r[r] = z;
      b->z_max = std::max(b->z_max, z);
    }
  }
  b->total_scores = b->score_off[b->G];
  b->mean_degree = b->total_rows > 0 ? (double)b->nnz_off[b->R] / (double)b->total_rows : 0.0;
  b->graphs.resize(b->G);
  for (int32_t g = 0; g < b->G; ++g) {
    b->graphs[g].score_off = b->score_off[g];
    b->graphs[g].n = b->n[g];
    b->graphs[g].first = b->first[g];
    b->graphs[g].count = b->nreal[g];
    b->graphs[g].pad = 0;
  }
  *out = b;
  return EBTC_OK;
}

void ebtc_batch_destroy(ebtc_batch* b) {
  if (!b) return;
  for (auto& e : b->execs) {
    (void)hipGraphExecDestroy(e.exec);
    (void)hipGraphDestroy(e.graph);
  }
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  delete b;
}

int ebtc_plan(ebtc_batch* b, const ebtc_opts* o, size_t* ws_bytes, size_t* ckpt_bytes) {
  g_err.clear();
  if (!b || !ws_bytes) return fail(EBTC_EINVAL, "NULL batch or output");
  int rc = check_opts(o);
  if (rc) return rc;
  const BatchPlan bp = spmv_plan(b, o);
  rc = check_plan(b, bp);
  if (rc) return rc;
  *ws_bytes = make_layout(b, o, bp).total;
  if (ckpt_bytes) *ckpt_bytes = sizeof(double) * kCkptDoubles * (size_t)b->R;
  return EBTC_OK;
}

int ebtc_scores(ebtc_batch* b, const ebtc_opts* o, void* ws, size_t ws_bytes, void* scores_out, double* log_scale_out,
                void* ckpt_out, ebtc_diag* diag_out, void* stream) {
  g_err.clear();
  if (!b) return fail(EBTC_EINVAL, "NULL batch");
  int rc = check_opts(o);
  if (rc) return rc;
  if (!ws || !scores_out || !log_scale_out) return fail(EBTC_EINVAL, "NULL workspace, scores or log_scale output");
  const BatchPlan bp = spmv_plan(b, o);
  rc = check_plan(b, bp);
  if (rc) return rc;
  const Layout L = make_layout(b, o, bp);
  if (ws_bytes < L.total)
    return fail(EBTC_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(L.total));
  if (((uintptr_t)ws & 255) != 0) return fail(EBTC_EINVAL, "workspace must be 256-byte aligned");
  int sched = 0;
  rc = resolve_schedule(b, o, &sched);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  rc = prepare_kernels(bp);
  if (rc) return rc;
  char* w = (char*)ws;
  rc = upload_tables(b, w, L, bp, s);
  if (rc) return rc;
  if (sched == EBTC_SCHED_PLAIN)
    return enqueue_plain(b, o, w, L, bp, scores_out, log_scale_out, ckpt_out, diag_out, s);
  if (!o->use_hipgraph)
    return enqueue_batched(b, o, w, L, bp, scores_out, log_scale_out, ckpt_out, diag_out, sched, s);
  const ExecKey key{ws,       scores_out, log_scale_out, ckpt_out, diag_out, o->m,   o->m_max,
                    o->reorth, o->shift,  sched,         o->tol,   bp.sig()};
  for (auto& e : b->execs) {
    if (e.key == key) {
      EBTC_HIP(hipGraphLaunch(e.exec, s));
      return EBTC_OK;
    }
  }
  if (!b->capture_stream) EBTC_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
  EBTC_HIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
  rc = enqueue_batched(b, o, w, L, bp, scores_out, log_scale_out, ckpt_out, diag_out, sched, b->capture_stream);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(b->capture_stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess) return fail(EBTC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(EBTC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  if (b->execs.size() >= 4) {
    (void)hipGraphExecDestroy(b->execs.front().exec);
    (void)hipGraphDestroy(b->execs.front().graph);
    b->execs.erase(b->execs.begin());
  }
  b->execs.push_back({key, graph, exec});
  EBTC_HIP(hipGraphLaunch(exec, s));
  return EBTC_OK;
}

}  // extern "C"

// ---- workspace of ebtc_scores_noalloc: a fixed device array, one per GPU, held until the process ends
namespace {

constexpr size_t kScratchBytes = EBTC_NOALLOC_WS_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// Device address of the current GPU's copy of `scratch`, looked up once per device (the array's name
// is a host-side stand-in in host code; only this address may be passed to kernels or copies).
int scratch_address(void** out) {
  int dev = -1;
  EBTC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return fail(EBTC_ENOTSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    EBTC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr || ((uintptr_t)p & 255) != 0) return fail(EBTC_EHIP, "scratch address unusable");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return EBTC_OK;
}

}  // namespace

extern "C" {

int ebtc_scores_noalloc(ebtc_batch* b, const ebtc_opts* o, void* scores_out, double* log_scale_out, void* ckpt_out,
                        ebtc_diag* diag_out, void* stream) {
  g_err.clear();
  if (!b) return fail(EBTC_EINVAL, "NULL batch");
  int rc = check_opts(o);
  if (rc) return rc;
  if (!scores_out || !log_scale_out) return fail(EBTC_EINVAL, "NULL scores or log_scale output");
  const BatchPlan bp = spmv_plan(b, o);
  rc = check_plan(b, bp);
  if (rc) return rc;
  const Layout L = make_layout(b, o, bp);
  if (L.total > kScratchBytes)
    return fail(EBTC_EWORKSPACE, "the batch needs a workspace of " + std::to_string(L.total) +
                                     " bytes; the static scratch holds " + std::to_string(kScratchBytes) +
                                     " (use ebtc_scores with a caller workspace)");
  int sched = 0;
  rc = resolve_schedule(b, o, &sched);
  if (rc) return rc;
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  rc = prepare_kernels(bp);
  if (rc) return rc;
  char* w = (char*)ws;
  rc = upload_tables(b, w, L, bp, s);
  if (rc) return rc;
  // eager launches: instantiating a hipGraph would allocate
  if (sched == EBTC_SCHED_PLAIN)
    return enqueue_plain(b, o, w, L, bp, scores_out, log_scale_out, ckpt_out, diag_out, s);
  return enqueue_batched(b, o, w, L, bp, scores_out, log_scale_out, ckpt_out, diag_out, sched, s);
}

int ebtc_profile_phases(ebtc_batch* b, const ebtc_opts* o, void* ws, size_t ws_bytes, void* scores_out,
                        double* log_scale_out, double* phase_ms, int64_t* phase_launches, void* stream) {
  g_err.clear();
  if (!b || !phase_ms || !phase_launches) return fail(EBTC_EINVAL, "NULL batch or phase output");
  int rc = check_opts(o);
  if (rc) return rc;
  if (!ws || !scores_out || !log_scale_out) return fail(EBTC_EINVAL, "NULL workspace, scores or log_scale output");
  const BatchPlan bp = spmv_plan(b, o);
  rc = check_plan(b, bp);
  if (rc) return rc;
  const Layout L = make_layout(b, o, bp);
  if (ws_bytes < L.total) return fail(EBTC_EWORKSPACE, "workspace too small");
  if (((uintptr_t)ws & 255) != 0) return fail(EBTC_EINVAL, "workspace must be 256-byte aligned");
  int sched = 0;
  rc = resolve_schedule(b, o, &sched);
  if (rc) return rc;
  if (sched == EBTC_SCHED_PLAIN) sched = EBTC_SCHED_BATCHED;  // phases are measured on a batched pass
  hipStream_t s = (hipStream_t)stream;
  rc = prepare_kernels(bp);
  if (rc) return rc;
  char* w = (char*)ws;
  rc = upload_tables(b, w, L, bp, s);
  if (rc) return rc;
  Prof prof;
  prof.s = s;
  rc = enqueue_batched(b, o, w, L, bp, scores_out, log_scale_out, nullptr, nullptr, sched, s, &prof);
  if (rc) return rc;
  EBTC_HIP(hipStreamSynchronize(s));
  for (int p = 0; p < EBTC_PHASE_COUNT; ++p) {
    phase_ms[p] = 0.0;
    phase_launches[p] = 0;
  }
  for (auto& r : prof.recs) {
    float ms = 0.f;
    EBTC_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    phase_ms[r.phase] += ms;
    phase_launches[r.phase] += 1;
  }
  return EBTC_OK;
}

int ebtc_tune(ebtc_batch* b, const ebtc_opts* o, void* ws, size_t ws_bytes, int32_t* form_out, int32_t* lanes_out,
              int32_t* seglen_out, double* ms_out, void* stream) {
  g_err.clear();
  if (!b) return fail(EBTC_EINVAL, "NULL batch");
  int rc = check_opts(o);
  if (rc) return rc;
  if (!ws) return fail(EBTC_EINVAL, "NULL workspace");
  const BatchPlan base = one_form(b, spmv_form(b, EBTC_SPMV_STREAM, 0, 0, o->hub_threshold));
  const Layout L = make_layout(b, o, base);
  if (ws_bytes < L.total)
    return fail(EBTC_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(L.total));
  if (((uintptr_t)ws & 255) != 0) return fail(EBTC_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const bool has_val = b->values != nullptr;
  const int steps = o->m > 0 ? o->m : o->m_max;
  rc = upload_tables(b, w, L, base, s);
  if (rc) return rc;
  // 1. each graph's bucket: its largest row (over its realizations) measured on the device, in the
  //    norm-partial arena, which the start kernel below overwrites
  std::vector<int32_t> row_max((size_t)b->R, 0);
  if (b->R > 0) {
    int32_t* dmax = (int32_t*)(w + L.off_npart);
    EBTC_LAUNCH(launch_row_max((const Task*)(w + L.off_tasks), b->row_ptr, b->R, dmax, s));
    EBTC_HIP(hipMemcpyAsync(row_max.data(), dmax, sizeof(int32_t) * (size_t)b->R, hipMemcpyDeviceToHost, s));
    EBTC_HIP(hipStreamSynchronize(s));
  }
  std::vector<std::string> gkey((size_t)b->G);
  {
    int64_t r = 0;
    for (int32_t g = 0; g < b->G; ++g) {
      int64_t z = 0;
      int32_t mx = 0;
      for (int32_t k = 0; k < b->nreal[g]; ++k, ++r) {
        z += b->nnz_r[r];
        mx = std::max(mx, row_max[r]);
      }
      gkey[g] = tune_key(b->dtype, has_val, b->n[g], (double)z / std::max<int64_t>(1, (int64_t)b->nreal[g] * b->n[g]),
                         mx, steps);
    }
  }
  // the batch's composition: its buckets, sorted and joined (the cache key of the batch's form)
  std::vector<std::string> keys = gkey;
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  std::string bkey;
  for (const std::string& k : keys) bkey += (bkey.empty() ? "" : "+") + k;
  keys.assign(1, bkey);
  for (std::string& k : gkey) k = bkey;
  // 2. time the candidate forms on the whole batch (a composition already in the cache is not timed)
  LzArgs a0 = make_args(b, o, w, L);
  EBTC_LAUNCH(launch_blkmap(a0.tasks, b->R, (int32_t*)(w + L.off_blkmap), s));
  EBTC_LAUNCH(launch_start(b->dtype, a0, L.total_blocks, s));
  double ms[EBTC_TUNE_SLOTS];
  for (double& v : ms) v = -1.0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  for (auto& e : ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& f : ev)
        if (f) (void)hipEventDestroy(f);
      return fail(EBTC_EHIP, "hipEventCreate failed");
    }
  }
  std::map<std::string, std::array<int32_t, 3>> choice;
  constexpr int kReps = 3;
  for (const std::string& key : keys) {
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        choice[key] = it->second;
        continue;
      }
    }
    const Members* mp = nullptr;  // every graph
    struct Cand {
      SpmvPlan p;
      int slot;
    };
    std::vector<Cand> cands;
    cands.push_back({spmv_form(b, EBTC_SPMV_STREAM, 0, 0, o->hub_threshold, mp), 0});
    for (int i = 0; i < 4; ++i)
      cands.push_back({spmv_form(b, EBTC_SPMV_LANE_GROUPS, 4 << i, 0, o->hub_threshold, mp), 1 + i});
    int32_t nmax = 1;
    for (int32_t g = 0; g < b->G; ++g)
      if (member(mp, g)) nmax = std::max(nmax, b->n[g]);
    const int maxseg = staged_max_seglen(b->dtype);
    if ((nmax + maxseg - 1) / maxseg <= 8) cands.push_back({spmv_form(b, EBTC_SPMV_LDS_STAGED, 0, 0, 0, mp), 5});
    const int small_seg = seg_max_cols(b->dtype) / 2;
    for (int i = 0; i < 2; ++i) {
      const SpmvPlan p = spmv_form(b, EBTC_SPMV_SEGMENTED, 0, small_seg << i, 0, mp);
      if (p.smax <= kSegMax) cands.push_back({p, 6 + i});
    }
    cands.push_back({spmv_form(b, EBTC_SPMV_BALANCED, 0, 0, 0, mp), 8});
    {
      const SpmvPlan p = spmv_form(b, EBTC_SPMV_PANELED, 0, 0, 0, mp);
      if (p.pmax <= kPanMaxPanels) cands.push_back({p, 9});
    }
    int best = -1;
    double best_ms = 0.0;
    for (size_t c = 0; c < cands.size() && rc == EBTC_OK; ++c) {
      const SpmvPlan& p = cands[c].p;
      const BatchPlan bp = one_form(b, p);
      if (check_plan(b, bp) != EBTC_OK) {
        g_err.clear();
        continue;
      }
      const Layout Lc = make_layout(b, o, bp);  // the forms' arenas follow the common ones
      if (Lc.total > ws_bytes) continue;
      rc = prepare_kernels(bp);
      if (rc) break;
      rc = upload_tables(b, w, Lc, bp, s);
      if (rc) break;
      const std::vector<FArgs> fa = form_args(b, a0, w, Lc, bp);
      const FArgs& x = fa[0];
      // [ev0, ev1): the once-per-call preparation; [ev2, ev3): kReps products after a warm-up. Step 0
      // reads only the start vector and the state k_start wrote, so every launch does the same work.
      hipError_t e = hipEventRecord(ev[0], s);
      if (e == hipSuccess && enqueue_prepare(b, x, 0, s, nullptr) != EBTC_OK) e = hipErrorLaunchFailure;
      if (e == hipSuccess) e = hipEventRecord(ev[1], s);
      if (e == hipSuccess) e = launch_spmv_step(b->dtype, has_val, p.lanes, 0, x.a, x.nb, s);
      if (e == hipSuccess) e = hipEventRecord(ev[2], s);
      for (int k = 0; k < kReps && e == hipSuccess; ++k) e = launch_spmv_step(b->dtype, has_val, p.lanes, 0, x.a, x.nb, s);
      if (e == hipSuccess) e = hipEventRecord(ev[3], s);
      if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
      float t_prep = 0.f, t_spmv = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t_prep, ev[0], ev[1]);
      if (e == hipSuccess) e = hipEventElapsedTime(&t_spmv, ev[2], ev[3]);
      if (e != hipSuccess) {
        rc = fail(EBTC_EHIP, std::string("tuning launch: ") + (g_err.empty() ? hipGetErrorString(e) : g_err));
        break;
      }
      const bool prepared = p.form == EBTC_SPMV_SEGMENTED || p.form == EBTC_SPMV_BALANCED || p.form == EBTC_SPMV_PANELED;
      const double t = t_spmv / kReps + (prepared ? t_prep / steps : 0.0);
      ms[cands[c].slot] = (ms[cands[c].slot] < 0 ? 0.0 : ms[cands[c].slot]) + t;
      if (best < 0 || t < best_ms) {
        best = (int)c;
        best_ms = t;
      }
    }
    if (rc) break;
    if (best < 0) {
      rc = fail(EBTC_EHIP, "no SpMV form could be timed");
      break;
    }
    const SpmvPlan& p = cands[best].p;
    choice[key] = {p.form, p.lanes, p.param()};
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = choice[key];
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (rc) return rc;
  // 3. the plan: one form per distinct choice, each graph on its bucket's
  std::vector<std::array<int32_t, 3>> forms;
  std::vector<int32_t> gform((size_t)b->G, 0);
  for (int32_t g = 0; g < b->G; ++g) {
    const std::array<int32_t, 3>& c = choice[gkey[g]];
    size_t f = 0;
    while (f < forms.size() && forms[f] != c) ++f;
    if (f == forms.size()) forms.push_back(c);
    gform[g] = (int32_t)f;
  }
  b->tuned = forms;
  b->tuned_graph = gform;
  if (form_out) *form_out = forms.size() == 1 ? forms[0][0] : EBTC_SPMV_AUTO;
  if (lanes_out) *lanes_out = forms.size() == 1 ? forms[0][1] : 0;
  if (seglen_out) *seglen_out = forms.size() == 1 ? forms[0][2] : 0;
  if (ms_out)
    for (int i = 0; i < EBTC_TUNE_SLOTS; ++i) ms_out[i] = ms[i];
  return EBTC_OK;
}

int ebtc_tuned_forms(ebtc_batch* b, int32_t* form_out, int32_t* lanes_out, int32_t* seglen_out) {
  g_err.clear();
  if (!b || !form_out) return fail(EBTC_EINVAL, "NULL batch or output");
  for (int32_t g = 0; g < b->G; ++g) {
    const bool t = !b->tuned.empty();
    const std::array<int32_t, 3> c = t ? b->tuned[b->tuned_graph[g]] : std::array<int32_t, 3>{0, 0, 0};
    form_out[g] = c[0];
    if (lanes_out) lanes_out[g] = c[1];
    if (seglen_out) seglen_out[g] = c[2];
  }
  return EBTC_OK;
}

int ebtc_set_forms(ebtc_batch* b, const int32_t* form, const int32_t* lanes, const int32_t* seg_len) {
  g_err.clear();
  if (!b || !form) return fail(EBTC_EINVAL, "NULL batch or form");
  std::vector<std::array<int32_t, 3>> forms;
  std::vector<int32_t> gform((size_t)b->G, 0);
  for (int32_t g = 0; g < b->G; ++g) {
    const int32_t l = lanes ? lanes[g] : 0, q = seg_len ? seg_len[g] : 0;
    if (form[g] < EBTC_SPMV_STREAM || form[g] > EBTC_SPMV_PANELED)
      return fail(EBTC_EINVAL, "graph " + std::to_string(g) + ": unknown spmv form");
    if (l != 0 && l != 4 && l != 8 && l != 16 && l != 32)
      return fail(EBTC_EINVAL, "graph " + std::to_string(g) + ": lanes must be 0, 4, 8, 16 or 32");
    if (q < 0) return fail(EBTC_EINVAL, "graph " + std::to_string(g) + ": seg_len must be >= 0");
    const std::array<int32_t, 3> c{form[g], form[g] == EBTC_SPMV_LANE_GROUPS ? l : 0, q};
    size_t f = 0;
    while (f < forms.size() && forms[f] != c) ++f;
    if (f == forms.size()) forms.push_back(c);
    gform[g] = (int32_t)f;
  }
  b->tuned = forms;
  b->tuned_graph = gform;
  return EBTC_OK;
}

int ebtc_tune_cache_get(char* buf, size_t cap, size_t* len) {
  g_err.clear();
  if (!len) return fail(EBTC_EINVAL, "NULL length output");
  std::string t;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const auto& kv : g_tune_cache)
      t += kv.first + " " + std::to_string(kv.second[0]) + " " + std::to_string(kv.second[1]) + " " +
           std::to_string(kv.second[2]) + "\n";
  }
  *len = t.size();
  if (buf == nullptr) return EBTC_OK;
  if (cap < t.size() + 1) return fail(EBTC_EINVAL, "buffer of " + std::to_string(cap) + " bytes, need " +
                                                       std::to_string(t.size() + 1));
  std::memcpy(buf, t.c_str(), t.size() + 1);
  return EBTC_OK;
}

int ebtc_tune_cache_put(const char* text) {
  g_err.clear();
  if (!text) return fail(EBTC_EINVAL, "NULL text");
  std::map<std::string, std::array<int32_t, 3>> add;
  const char* p = text;
  while (*p) {
    const char* e = std::strchr(p, '\n');
    const std::string line = e ? std::string(p, e) : std::string(p);
    p = e ? e + 1 : p + line.size();
    if (line.empty()) continue;
    std::istringstream in(line);
    std::string key, rest;
    int f = 0, l = 0, q = 0;
    if (!(in >> key >> f >> l >> q) || (in >> rest) || f < EBTC_SPMV_STREAM || f > EBTC_SPMV_PANELED ||
        (l != 0 && l != 4 && l != 8 && l != 16 && l != 32) || q < 0)
      return fail(EBTC_EINVAL, "bad tune-cache line: " + line);
    add[key] = {f, l, q};
  }
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (const auto& kv : add) g_tune_cache[kv.first] = kv.second;
  return EBTC_OK;
}

int ebtc_tune_cache_clear(void) {
  g_err.clear();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache.clear();
  return EBTC_OK;
}

int ebtc_plan_backward(ebtc_batch* b, const ebtc_opts* o, size_t* ws_bytes) {
  g_err.clear();
  if (!b || !ws_bytes) return fail(EBTC_EINVAL, "NULL batch or output");
  int rc = check_bwd_opts(o);
  if (rc) return rc;
  rc = check_plan(b, spmv_plan(b, o));
  if (rc) return rc;
  *ws_bytes = make_bwd_layout(b, o).total;
  return EBTC_OK;
}

int ebtc_scores_backward(ebtc_batch* b, const ebtc_opts* o, const double* log_scale, const void* grad_scores,
                         void* grad_values, void* ws, size_t ws_bytes, const double* ckpt, int32_t* ckpt_mismatch,
                         void* stream) {
  g_err.clear();
  if (!b) return fail(EBTC_EINVAL, "NULL batch");
  int rc = check_bwd_opts(o);
  if (rc) return rc;
  if (!log_scale || !grad_scores || !grad_values || !ws)
    return fail(EBTC_EINVAL, "NULL log_scale, grad_scores, grad_values or workspace");
  if (ckpt && !ckpt_mismatch) return fail(EBTC_EINVAL, "a checkpoint to compare needs ckpt_mismatch");
  const BatchPlan bp = spmv_plan(b, o);
  rc = check_plan(b, bp);
  if (rc) return rc;
  const BwdLayout B = make_bwd_layout(b, o);
  if (ws_bytes < B.total)
    return fail(EBTC_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(B.total));
  if (((uintptr_t)ws & 255) != 0) return fail(EBTC_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  rc = prepare_kernels(bp);
  if (rc) return rc;
  char* w = (char*)ws;
  rc = upload_tables(b, w, B.fwd, bp, s);
  if (rc) return rc;
  // 1. forward recomputation (same kernels and order as ebtc_scores: bitwise the same basis)
  LzArgs fa = make_args(b, o, w, B.fwd);
  fa.unit_start = 1;
  const std::vector<FArgs> ffa = form_args(b, fa, w, B.fwd, bp);
  EBTC_LAUNCH(launch_blkmap(fa.tasks, b->R, (int32_t*)(w + B.fwd.off_blkmap), s));
  rc = enqueue_prepare_all(b, ffa, s, nullptr);  // the sorted entries serve both solves
  if (rc) return rc;
  rc = run_steps(b, o, fa, ffa, B.fwd.total_blocks, 0, b->R, s, nullptr);
  if (rc) return rc;
  const int steps = o->m > 0 ? o->m : o->m_max;
  EBTC_LAUNCH(launch_tridiag_state(fa, 0, b->R, 0, 0, steps, o->shift, o->tol, nullptr, nullptr, s));
  // the recomputation against the forward call's checkpoint: every reduction runs in a fixed order, so
  // any difference means the inputs or the options are not the forward's
  if (ckpt) EBTC_LAUNCH(launch_ckpt_check(fa.state, ckpt, b->R, ckpt_mismatch, s));
  // 2. adjoint Lanczos started at the cotangent (shares W and the partial-sum arenas)
  LzArgs aa = fa;
  aa.unit_start = 0;  // started at the cotangent
  aa.first_in_prepare = 0;
  aa.state = (RState*)(w + B.off_astate);
  aa.V = w + B.off_aV;
  const std::vector<FArgs> faa = form_args(b, aa, w, B.fwd, bp);
  EBTC_LAUNCH(launch_start_vec(b->dtype, aa, (const GraphInfo*)(w + B.fwd.off_graphs), grad_scores,
                               B.fwd.total_blocks, s));
  EBTC_LAUNCH(launch_start_norm(aa, b->R, s));
  rc = run_steps(b, o, aa, faa, B.fwd.total_blocks, 0, b->R, s, nullptr, false);
  if (rc) return rc;
  EBTC_LAUNCH(launch_tridiag_state(aa, 0, b->R, 0, 0, steps, 1, o->tol, nullptr, nullptr, s));
  // 3. block exponential, 4. node-major Z and V, 5. SDDMM on the pattern
  double* X = (double*)(w + B.off_X);
  EBTC_LAUNCH(launch_block_exp(fa.state, aa.state, fa.tasks, log_scale, X, b->R, s));
  EBTC_LAUNCH(launch_build_zv(b->dtype, fa, aa, X, w + B.off_Z, w + B.off_Vn, B.ld, B.fwd.total_blocks, s));
  EBTC_LAUNCH(launch_sddmm(b->dtype, B.ld, fa, w + B.off_Z, w + B.off_Vn, grad_values, B.fwd.total_blocks, s));
  return EBTC_OK;
}

// One graph, `count` Lanczos processes over its CSR (every task shares the graph's arrays).
namespace {
void shared_batch(ebtc_batch& b, int32_t dtype, int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                  const void* values, int32_t count) {
  b.dtype = dtype;
  b.G = 1;
  b.R = count;
  b.n = {n};
  b.nreal = {count};
  b.first = {0};
  b.rowptr_off.assign(count, 0);
  b.nnz_off.assign((size_t)count + 1, 0);
  b.nnz_r.assign((size_t)count, 0);  // the shared entries belong to no realization's arenas
  b.score_off = {0, n};
  b.row_ptr = row_ptr;
  b.col_idx = col_idx;
  b.values = values;
  b.total_scores = n;
  b.total_rows = (int64_t)n * count;
  b.n_max = n;
  b.graphs.resize(1);
  b.graphs[0] = GraphInfo{0, n, 0, count, 0};
}

int check_sc_args(int32_t dtype, int32_t n, int32_t count, int32_t m) {
  if (dtype != EBTC_F32 && dtype != EBTC_F64) return fail(EBTC_EINVAL, "dtype must be EBTC_F32 or EBTC_F64");
  if (n < 1) return fail(EBTC_EINVAL, "n must be >= 1");
  if (count < 1) return fail(EBTC_EINVAL, "count must be >= 1");
  if (m < 1 || m > EBTC_M_LIMIT) return fail(EBTC_EINVAL, "m must be in [1, " + std::to_string(EBTC_M_LIMIT) + "]");
  if ((int64_t)count * ((n + kRowsPerBlock - 1) / kRowsPerBlock) >= ((int64_t)1 << 31))
    return fail(EBTC_ENOTSUPPORTED, "too many row blocks for one launch");
  return EBTC_OK;
}

ebtc_opts sc_opts(int32_t m) {
  ebtc_opts o;
  ebtc_default_opts(&o);
  o.m = m;
  o.reorth = 1;
  o.schedule = EBTC_SCHED_BATCHED;
  o.use_hipgraph = 0;
  o.spmv = EBTC_SPMV_STREAM;
  return o;
}
}  // namespace

int ebtc_subgraph_centrality_ws_bytes(int32_t dtype, int32_t n, int32_t count, int32_t m, size_t* ws_bytes) {
  g_err.clear();
  if (!ws_bytes) return fail(EBTC_EINVAL, "NULL output");
  int rc = check_sc_args(dtype, n, count, m);
  if (rc) return rc;
  ebtc_batch b;
  shared_batch(b, dtype, n, nullptr, nullptr, nullptr, count);
  const ebtc_opts o = sc_opts(m);
  *ws_bytes = make_layout(&b, &o, spmv_plan(&b, &o)).total;
  return EBTC_OK;
}

int ebtc_subgraph_centrality(int32_t dtype, int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                             const void* values, int32_t count, const int32_t* nodes, int32_t m, double* sc_out,
                             void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int rc = check_sc_args(dtype, n, count, m);
  if (rc) return rc;
  if (!row_ptr || !col_idx || !nodes || !sc_out || !ws)
    return fail(EBTC_EINVAL, "NULL row_ptr, col_idx, nodes, output or workspace");
  ebtc_batch b;
  shared_batch(b, dtype, n, row_ptr, col_idx, values, count);
  const ebtc_opts o = sc_opts(m);
  const BatchPlan bp = spmv_plan(&b, &o);
  const Layout L = make_layout(&b, &o, bp);
  if (ws_bytes < L.total)
    return fail(EBTC_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(L.total));
  if (((uintptr_t)ws & 255) != 0) return fail(EBTC_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  rc = upload_tables(&b, w, L, bp, s);
  if (rc) return rc;
  // the task table lives on this call's stack: wait until the copy has read it
  EBTC_HIP(hipStreamSynchronize(s));
  LzArgs a = make_args(&b, &o, w, L);
  const std::vector<FArgs> fa = form_args(&b, a, w, L, bp);
  EBTC_LAUNCH(launch_blkmap(a.tasks, b.R, (int32_t*)(w + L.off_blkmap), s));
  EBTC_LAUNCH(launch_start_unit(dtype, a, nodes, L.total_blocks, s));
  rc = run_steps(&b, &o, a, fa, L.total_blocks, 0, b.R, s, nullptr, false);
  if (rc) return rc;
  EBTC_LAUNCH(launch_tridiag_state(a, 0, b.R, 0, 0, m, 1, 0.0, nullptr, nullptr, s));
  EBTC_LAUNCH(launch_sc_out(a.state, a.tasks, nodes, b.R, sc_out, s));
  return EBTC_OK;
}

int ebtc_topk_ws_bytes(ebtc_batch* b, size_t* ws_bytes) {
  g_err.clear();
  if (!b || !ws_bytes) return fail(EBTC_EINVAL, "NULL batch or output");
  *ws_bytes = align_up(sizeof(GraphInfo) * b->G) + align_up(sizeof(int32_t) * b->G) + align_up(sizeof(int64_t) * b->G);
  if (b->n_max >= kTopkMultiMin) {  // the chunked selection: chunk tables and its scratch
    const int64_t nchunks = topk_chunks(b);
    *ws_bytes += align_up(sizeof(int32_t) * (size_t)nchunks) + align_up(sizeof(int32_t) * ((size_t)b->G + 1)) +
                 topk_multi_scratch_bytes(b->G, nchunks);
  }
  return EBTC_OK;
}

int ebtc_topk(ebtc_batch* b, const void* scores, const int32_t* k_per_graph, int32_t* idx_out, void* val_out,
              void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!b || !scores || !k_per_graph || !idx_out || !ws) return fail(EBTC_EINVAL, "NULL argument");
  size_t need = 0;
  ebtc_topk_ws_bytes(b, &need);
  if (ws_bytes < need) return fail(EBTC_EWORKSPACE, "top-k workspace too small");
  if (((uintptr_t)ws & 255) != 0) return fail(EBTC_EINVAL, "workspace must be 256-byte aligned");
  b->topk_k.assign(k_per_graph, k_per_graph + b->G);
  b->topk_off.resize(b->G);
  int64_t off = 0;
  for (int32_t g = 0; g < b->G; ++g) {
    const int32_t k = b->topk_k[g];
    if (k < 0 || k > b->n[g] || k > EBTC_TOPK_LIMIT)
      return fail(k > EBTC_TOPK_LIMIT ? EBTC_ENOTSUPPORTED : EBTC_EINVAL,
                  "graph " + std::to_string(g) + ": K must be in [0, min(n, 4096)]");
    b->topk_off[g] = off;
    off += k;
  }
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const size_t o1 = align_up(sizeof(GraphInfo) * b->G), o2 = o1 + align_up(sizeof(int32_t) * b->G);
  EBTC_HIP(hipMemcpyAsync(w, b->graphs.data(), sizeof(GraphInfo) * b->G, hipMemcpyHostToDevice, s));
  EBTC_HIP(hipMemcpyAsync(w + o1, b->topk_k.data(), sizeof(int32_t) * b->G, hipMemcpyHostToDevice, s));
  EBTC_HIP(hipMemcpyAsync(w + o2, b->topk_off.data(), sizeof(int64_t) * b->G, hipMemcpyHostToDevice, s));
  const size_t o3 = o2 + align_up(sizeof(int64_t) * b->G);
  if (b->n_max < kTopkMultiMin) {  // one workgroup per graph
    EBTC_LAUNCH(launch_topk(b->dtype, (const GraphInfo*)w, b->G, (const int32_t*)(w + o1), (const int64_t*)(w + o2),
                            scores, idx_out, val_out, s));
    return EBTC_OK;
  }
  // chunks of kTkChunk scores, graph by graph (a graph's chunks follow its node ids)
  const int64_t nchunks = topk_chunks(b);
  b->topk_cgraph.resize((size_t)nchunks);
  b->topk_cbegin.resize((size_t)b->G + 1);
  int32_t c = 0;
  for (int32_t g = 0; g < b->G; ++g) {
    b->topk_cbegin[g] = c;
    const int32_t nc = (b->n[g] + kTkChunk - 1) / kTkChunk;
    for (int32_t i = 0; i < nc; ++i) b->topk_cgraph[c++] = g;
  }
  b->topk_cbegin[b->G] = c;
  const size_t o4 = o3 + align_up(sizeof(int32_t) * (size_t)nchunks), o5 = o4 + align_up(sizeof(int32_t) * ((size_t)b->G + 1));
  EBTC_HIP(hipMemcpyAsync(w + o3, b->topk_cgraph.data(), sizeof(int32_t) * (size_t)nchunks, hipMemcpyHostToDevice, s));
  EBTC_HIP(hipMemcpyAsync(w + o4, b->topk_cbegin.data(), sizeof(int32_t) * ((size_t)b->G + 1), hipMemcpyHostToDevice, s));
  EBTC_LAUNCH(launch_topk_multi(b->dtype, (const GraphInfo*)w, b->G, (const int32_t*)(w + o1), (const int64_t*)(w + o2),
                                scores, idx_out, val_out, (const int32_t*)(w + o3), (const int32_t*)(w + o4), nchunks,
                                w + o5, s));
  return EBTC_OK;
}

int ebtc_spmv(int32_t dtype, int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const void* values,
              const void* x, void* y, int32_t lanes_per_row, int32_t hub_threshold, int32_t seg_len, void* stream) {
  g_err.clear();
  if (dtype != EBTC_F32 && dtype != EBTC_F64) return fail(EBTC_EINVAL, "dtype must be EBTC_F32 or EBTC_F64");
  if (n < 1 || !row_ptr || !col_idx || !x || !y) return fail(EBTC_EINVAL, "n < 1 or NULL pointer");
  if (x == y) return fail(EBTC_EINVAL, "x and y must be distinct");
  const int lanes = lanes_per_row;
  if (lanes != 0 && lanes != 4 && lanes != 8 && lanes != 16 && lanes != 32)
    return fail(EBTC_EINVAL, "lanes_per_row must be 0, 4, 8, 16 or 32");
  if (hub_threshold < 0) return fail(EBTC_EINVAL, "hub_threshold must be >= 0");
  if (seg_len < -1) return fail(EBTC_EINVAL, "seg_len must be -1, 0 or > 0");
  const int hub = hub_threshold ? hub_threshold : 16 * (lanes ? lanes : 8);
  const int seg = seg_len > 0 ? std::min(seg_len, staged_max_seglen(dtype)) : 0;
  if (seg > 0) EBTC_HIP(prepare_staged_kernels());
  EBTC_LAUNCH(launch_spmv(dtype, values != nullptr, lanes, hub, seg, n, row_ptr, col_idx, values, x, y,
                          (hipStream_t)stream));
  return EBTC_OK;
}

int ebtc_tridiag_expv(int32_t count, int32_t k, const double* alpha, const double* beta, double* y_out,
                      double* theta_out, int32_t shift, void* stream) {
  g_err.clear();
  if (count < 0) return fail(EBTC_EINVAL, "count must be >= 0");
  if (k < 1 || k > EBTC_M_LIMIT) return fail(EBTC_EINVAL, "k must be in [1, " + std::to_string(EBTC_M_LIMIT) + "]");
  if (count == 0) return EBTC_OK;
  if (!alpha || !beta || !y_out || !theta_out) return fail(EBTC_EINVAL, "NULL pointer");
  EBTC_LAUNCH(launch_tridiag_arrays(count, k, alpha, beta, y_out, theta_out, shift, (hipStream_t)stream));
  return EBTC_OK;
}

int ebtc_validate_ws_bytes(ebtc_batch* b, size_t* ws_bytes) {
  g_err.clear();
  if (!b || !ws_bytes) return fail(EBTC_EINVAL, "NULL batch or output");
  *ws_bytes = align_up(sizeof(Task) * b->R) + align_up(sizeof(int64_t) * b->R) + align_up(sizeof(int32_t) * b->R);
  return EBTC_OK;
}

int ebtc_validate(ebtc_batch* b, void* ws, size_t ws_bytes, int64_t* first_bad, void* stream) {
  g_err.clear();
  if (!b || !ws || !first_bad) return fail(EBTC_EINVAL, "NULL argument");
  size_t need = 0;
  ebtc_validate_ws_bytes(b, &need);
  if (ws_bytes < need) return fail(EBTC_EWORKSPACE, "validate workspace too small");
  hipStream_t s = (hipStream_t)stream;
  Layout L;
  L.m_slots = 1;
  BatchPlan one;
  one.forms.resize(1);
  one.graph_form.assign((size_t)b->G, 0);
  fill_tables(b, L, one);
  char* w = (char*)ws;
  const size_t o1 = align_up(sizeof(Task) * b->R), o2 = o1 + align_up(sizeof(int64_t) * b->R);
  std::vector<int32_t> bad(b->R, 0);
  EBTC_HIP(hipMemcpyAsync(w, b->tasks.data(), sizeof(Task) * b->R, hipMemcpyHostToDevice, s));
  EBTC_HIP(hipMemcpyAsync(w + o1, b->nnz_r.data(), sizeof(int64_t) * b->R, hipMemcpyHostToDevice, s));
  EBTC_HIP(hipMemcpyAsync(w + o2, bad.data(), sizeof(int32_t) * b->R, hipMemcpyHostToDevice, s));
  EBTC_LAUNCH(launch_validate(b->row_ptr, b->col_idx, (const Task*)w, (const int64_t*)(w + o1), b->R, b->n_max,
                              (int32_t*)(w + o2), s));
  EBTC_HIP(hipMemcpyAsync(bad.data(), w + o2, sizeof(int32_t) * b->R, hipMemcpyDeviceToHost, s));
  EBTC_HIP(hipStreamSynchronize(s));
  *first_bad = -1;
  for (int64_t r = 0; r < b->R; ++r)
    if (bad[r]) {
      *first_bad = r;
      break;
    }
  return EBTC_OK;
}

}  // extern "C"
