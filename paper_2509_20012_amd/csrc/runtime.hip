// Host runtime and C ABI of the fredopt library (include/fredopt.h): workspace
// layout, matrix load (Table 2 step iii of Borys et al., arXiv 2509.20012), work
// lists for the kernels, one outer iteration of Fig. 3 as a fixed kernel sequence,
// HIP-graph capture of that sequence for fredopt_solve, measurement and tuning.
#include "fredopt.h"
#include "fredopt_device.h"
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

using namespace fo;

namespace {

thread_local std::string g_err;

fredopt_status fail(fredopt_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(FREDOPT_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int64_t kSortWindow = 8192;     // rows sorted by length inside such windows
constexpr int64_t kRowItemRows = 2048;
constexpr int64_t kTrChunkMin = 256;
constexpr int64_t kTrChunkDefault = 4096;
// Chunk cap of the gradient's column-major copy (objective rows only): its columns
// are short and few, so smaller chunks balance the waves of the single pass better.
constexpr int64_t kGradChunk = 512;
constexpr int64_t kBlockCountCap = int64_t(1) << 24;
constexpr int kTrWgsPerCu = 8;            // persistent grid of the column-major passes
constexpr size_t kProjectTwoPerCuLds = 72 * 1024;  // LDS sums that let two projection
                                                   // workgroups share a CU
constexpr int kObjWgsPerCu = 2;           // forward passes over the objective-row view
constexpr size_t kScatterLdsMax = 159744; // its LDS accumulator: C 64-bit sums

inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

inline bool scatter_fits(int64_t C) { return (size_t)C * sizeof(int64_t) <= kScatterLdsMax; }

int value_bytes(int storage) { return storage == FREDOPT_F32 ? 4 : 2; }
int index_bytes(int storage) { return index16(storage) ? 2 : 4; }  // row-major copy

int auto_lpr_log2(int64_t R, int64_t nnz) {
  const double avg = R > 0 ? (double)nnz / (double)R : 0.0;
  int lg = 0;
  while (lg < 4 && (double)(1 << (lg + 1)) <= avg / 64.0) ++lg;
  return lg;
}

bool lpr_log2_of(int32_t lanes, int64_t R, int64_t nnz, int* out) {
  if (lanes == 0) {
    *out = auto_lpr_log2(R, nnz);
    return true;
  }
  for (int lg = 0; lg <= 4; ++lg)
    if (lanes == (1 << lg)) {
      *out = lg;
      return true;
    }
  return false;
}

// Sliced-ELL geometry of one pattern.
struct Sell {
  int lpr_log2 = 0;
  int64_t n_slices = 0, slots = 0;
  std::vector<int64_t> base;   // n_slices + 1
  std::vector<int32_t> width;  // n_slices
  std::vector<int32_t> srow;   // n_slices * rpw
  std::vector<int32_t> rslice; // R
};

// Listed rows (row_id(i), length len(i), i = 0..n-1) sorted by length (descending,
// stable) inside windows of kSortWindow consecutive list positions, cut into slices
// of rpw rows; each slice is as wide as its longest row.  With full set, the slice
// tables are kept and pos[i] receives list entry i's slice position.
template <typename RowId, typename Len>
void build_sell_list(int64_t n, RowId row_id, Len len, int lpr_log2, bool full, Sell* S) {
  const int rpw = kWave >> lpr_log2;
  const int64_t lpr4 = 4LL << lpr_log2;
  S->lpr_log2 = lpr_log2;
  S->n_slices = 0;
  S->slots = 0;
  if (full) {
    S->base.assign(1, 0);
    S->width.clear();
    S->srow.clear();
    S->rslice.assign(n, -1);
  }
  std::vector<int64_t> idx;
  for (int64_t w0 = 0; w0 < n; w0 += kSortWindow) {
    const int64_t w1 = std::min(n, w0 + kSortWindow);
    idx.resize(w1 - w0);
    std::iota(idx.begin(), idx.end(), w0);
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return len(a) > len(b); });
    for (size_t s0 = 0; s0 < idx.size(); s0 += rpw) {
      const int64_t steps = (len(idx[s0]) + lpr4 - 1) / lpr4;  // longest row of the slice
      if (full) {
        for (int p = 0; p < rpw; ++p) {
          const size_t k = s0 + p;
          S->srow.push_back(k < idx.size() ? (int32_t)row_id(idx[k]) : -1);
          if (k < idx.size()) S->rslice[idx[k]] = (int32_t)(S->n_slices * rpw + p);
        }
        S->width.push_back((int32_t)steps);
        S->base.push_back(S->base.back() + steps * 256);
      }
      S->slots += steps * 256;
      S->n_slices += 1;
    }
  }
}

void build_sell(const int64_t* rp, int64_t R, int lpr_log2, bool full, Sell* S) {
  build_sell_list(R, [](int64_t i) { return i; },
                  [rp](int64_t i) { return rp[i + 1] - rp[i]; }, lpr_log2, full, S);
}

struct Layout {
  size_t table, state, ctr, sbase, swidth, srow, sci, sdv, slv, cp, ri, cdv, clv;
  size_t col_tslot0, col_nch, cscale, mom, d, l, dg, lg, coef, g;
  size_t gri, gcdv, gclv, gcol_tslot0, gcol_nch, ocp, ocount, gtr_items;
  size_t y, osbase, oswidth, osrow, osci, osdv, oslv, ogroups, pk_src, pk_dst, pk_len;
  size_t spart_a, spart_b, rpart, gpart, tpart, groups, row_items, tr_items, col_blocks;
  size_t bc, colcount, colmax, flags, rslice, rsum, goff, alist, spart, smask, sc_items,
      ss_items, pkind, pf, okind, of, ovec, gcoef, coef_row, rptr, plen, rci, rdv, rlv, btable,
      bgroups, total;
  int64_t NP;                 // positions of the all-row view
  int64_t sell_slots, n_slices, csc_slots, obj_slots, max_rows, max_tr, n_groups, n_col_blocks;
  int64_t row_slots;          // row-contiguous copy: every row padded to 4 slots
  int64_t max_blocks;         // blocks of a block-sequential sweep (one per sort window)
  int64_t obj_sell_slots, max_obj_slices, max_obj_groups, max_obj_srow;
  int64_t rows_per_block, nb;
};

constexpr int kDefaultGradientReservePct = 25;

int reserve_pct_of(int32_t v) { return v == 0 ? kDefaultGradientReservePct : (v < 0 ? 0 : std::min(v, 100)); }

// Layout for given SELL sizes; CSC and work lists use pattern-free bounds.
bool make_layout(int64_t R, int64_t C, int64_t nnz, int storage, int lpr_log2,
                 int64_t sell_slots, int64_t n_slices, int reserve_pct, Layout* L) {
  if (R < 0 || C < 1 || nnz < 0 || R >= (int64_t(1) << 31) || C >= (int64_t(1) << 31))
    return false;
  if (storage < FREDOPT_F32 || storage > FREDOPT_BF16_IDX16) return false;
  if (index16(storage) && C > 65536) return false;
  const int64_t csc = nnz + 3 * C;
  if (csc >= (int64_t(1) << 32) - 4) return false;
  const int rpw = kWave >> lpr_log2;
  const int vb = value_bytes(storage);
  L->sell_slots = sell_slots;
  L->n_slices = n_slices;
  L->csc_slots = csc;
  L->obj_slots = ((csc * reserve_pct) / 100 + 3) & ~int64_t(3);
  L->obj_sell_slots = reserve_pct > 0 ? (((sell_slots * reserve_pct) / 100 + 255) & ~int64_t(255)) : 0;
  // the objective-row view may use up to 16 lanes per row (4 rows per slice)
  L->max_obj_slices = reserve_pct > 0 ? R / 4 + R / kSortWindow + 2 : 0;
  L->max_obj_groups = (L->max_obj_slices + kFwdWaves - 1) / kFwdWaves + 1;
  L->max_obj_srow = reserve_pct > 0 ? R + (R / kSortWindow + 2) * kWave + 1 : 1;
  L->max_rows = R / kRowItemRows + 2;
  L->max_tr = C + csc / kTrChunkMin + 2;
  L->n_groups = (n_slices + kFwdWaves - 1) / kFwdWaves + 1;
  L->n_col_blocks = (C + kBlock - 1) / kBlock;
  int64_t rpb = 1024;
  if (R > 0 && R * C / rpb > kBlockCountCap) rpb = (R * C + kBlockCountCap - 1) / kBlockCountCap;
  L->rows_per_block = rpb;
  L->nb = R > 0 ? (R + rpb - 1) / rpb : 1;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t Rm = (size_t)std::max<int64_t>(R, 1);
  L->NP = n_slices * rpw;     // per-row data of the all-row view, in position order
  const size_t Pm = (size_t)std::max<int64_t>(L->NP, 1);
  const size_t Om = (size_t)std::max<int64_t>(L->max_obj_srow, 1);
  L->table = take(sizeof(DevPlan));
  L->state = take(sizeof(DevState));
  L->ctr = take(sizeof(uint32_t) * kCounters);
  L->sbase = take(sizeof(int64_t) * (n_slices + 1));
  L->swidth = take(sizeof(int32_t) * (n_slices + 1));
  L->srow = take(sizeof(int32_t) * (n_slices * rpw + 1));
  L->sci = take((size_t)index_bytes(storage) * sell_slots);
  L->sdv = take((size_t)vb * sell_slots);
  L->slv = take((size_t)vb * sell_slots);
  L->cp = take(sizeof(int64_t) * (C + 1));
  L->ri = take(sizeof(int32_t) * csc);
  L->cdv = take((size_t)vb * csc);
  L->clv = take((size_t)vb * csc);
  L->col_tslot0 = take(sizeof(int32_t) * C);
  L->col_nch = take(sizeof(int32_t) * C);
  L->gri = take(sizeof(int32_t) * L->obj_slots);
  L->gcdv = take((size_t)vb * L->obj_slots);
  L->gclv = take((size_t)vb * L->obj_slots);
  L->gcol_tslot0 = take(sizeof(int32_t) * C);
  L->gcol_nch = take(sizeof(int32_t) * C);
  L->ocp = take(sizeof(int64_t) * (C + 1));
  L->ocount = take(sizeof(uint32_t) * C);
  L->gtr_items = take(sizeof(TrItem) * L->max_tr);
  L->y = take(sizeof(float) * C);
  L->osbase = take(sizeof(int64_t) * (L->max_obj_slices + 1));
  L->oswidth = take(sizeof(int32_t) * (L->max_obj_slices + 1));
  L->osrow = take(sizeof(int32_t) * L->max_obj_srow);
  L->osci = take((size_t)index_bytes(storage) * L->obj_sell_slots);
  L->osdv = take((size_t)vb * L->obj_sell_slots);
  L->oslv = take((size_t)vb * L->obj_sell_slots);
  L->ogroups = take(sizeof(FwdGroup) * L->max_obj_groups);
  L->pk_src = take(sizeof(int32_t) * (reserve_pct > 0 ? Rm : 1));
  L->pk_dst = take(sizeof(int32_t) * (reserve_pct > 0 ? Rm : 1));
  L->pk_len = take(sizeof(int32_t) * (reserve_pct > 0 ? Rm : 1));
  L->cscale = take(sizeof(float) * C);
  L->mom = take(sizeof(double) * 3 * Pm);
  L->d = take(sizeof(float) * Pm);
  L->l = take(sizeof(float) * Pm);
  L->dg = take(sizeof(float) * Pm);
  L->lg = take(sizeof(float) * Pm);
  L->coef = take(sizeof(float2) * Pm);
  L->pkind = take(sizeof(uint16_t) * Pm);
  L->pf = take(sizeof(float) * 9 * Pm);          // dlo dhi clo chi tmax wf wo dt ct
  L->okind = take(sizeof(uint16_t) * Om);
  L->of = take(sizeof(float) * 3 * Om);          // wo dt ct of the objective-row view
  L->ovec = take(sizeof(float) * 4 * Om);        // its d, l, D g, L g (step search)
  L->gcoef = take(sizeof(float2) * Rm);          // gradient coefficients by row
  L->coef_row = take(sizeof(float2) * Rm);       // projection coefficients by row
  L->g = take(sizeof(float) * C);
  L->spart_a = take(sizeof(double) * kNPart * std::max(L->n_groups, L->max_obj_groups));
  L->spart_b = take(sizeof(double) * kNPart * std::max(L->n_groups, L->max_obj_groups));
  L->rpart = take(sizeof(double) * kNPart * L->max_rows);
  L->gpart = take(sizeof(double) * L->n_col_blocks);
  L->tpart = take(sizeof(float) * L->max_tr);
  L->groups = take(sizeof(FwdGroup) * L->n_groups);
  L->row_items = take(sizeof(RowItem) * L->max_rows);
  L->tr_items = take(sizeof(TrItem) * L->max_tr);
  L->col_blocks = take(sizeof(ColBlock) * L->n_col_blocks);
  L->bc = take(sizeof(uint32_t) * L->nb * C);
  L->colcount = take(sizeof(uint32_t) * C);
  L->colmax = take(sizeof(uint32_t) * C);
  L->flags = take(sizeof(uint32_t) * 4);
  L->rslice = take(sizeof(int32_t) * Rm);
  L->rsum = take(sizeof(float) * 2 * Pm);
  L->goff = take(sizeof(int32_t) * L->n_groups);
  L->alist = take(sizeof(ActRow) * Pm);
  // per-workgroup shares, or C sums in global memory when they do not fit in LDS
  L->spart = take(scatter_fits(C) ? sizeof(int64_t) * kScatterMaxWGs * C : sizeof(int64_t) * C);
  L->smask = take(scatter_fits(C) ? sizeof(uint64_t) * kScatterMaxWGs * ((C + 63) / 64)
                                  : sizeof(uint64_t));
  L->sc_items = take(sizeof(ScItem) * kScatterMaxWGs);
  L->ss_items = take(sizeof(ScItem) * ((C + 63) / 64));
  L->row_slots = nnz + 3 * R;
  L->rptr = take(sizeof(int64_t) * (Pm + 1));
  L->plen = take(sizeof(int32_t) * Pm);
  L->rci = take((size_t)index_bytes(storage) * std::max<int64_t>(L->row_slots, 1));
  L->rdv = take((size_t)vb * std::max<int64_t>(L->row_slots, 1));
  L->rlv = take((size_t)vb * std::max<int64_t>(L->row_slots, 1));
  L->max_blocks = R / kSortWindow + 2;
  L->btable = take(sizeof(DevPlan) * L->max_blocks);
  L->bgroups = take(sizeof(FwdGroup) * (L->n_groups + L->max_blocks));
  L->total = o;
  return true;
}

// Pattern-free bound of the SELL size (rows sorted by length inside a window: the
// slice widths telescope, so a window wastes at most rpw * n_cols slots plus the
// per-slice rounding).
bool bound_layout(int64_t R, int64_t C, int64_t nnz, int storage, int lpr_log2, int reserve_pct,
                  Layout* L) {
  if (R < 0 || C < 1 || nnz < 0) return false;
  const int64_t rpw = kWave >> lpr_log2;
  const int64_t nwin = (R + kSortWindow - 1) / kSortWindow;
  const int64_t n_slices = R / rpw + nwin + 1;
  const int64_t sell = nnz + nwin * rpw * C + n_slices * rpw * ((4LL << lpr_log2) - 1);
  return make_layout(R, C, nnz, storage, lpr_log2, sell, n_slices, reserve_pct, L);
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct fredopt_plan {
  int64_t R = 0, C = 0, nnz = 0;
  int storage = 0, device = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Layout L{};
  Sell sell;
  std::vector<int64_t> cp;
  int tr_chunk = (int)kTrChunkDefault;
  int n_cu = 256, wgs_per_cu = 2, max_wgs_per_cu = 2, lds_floats = 0;
  size_t smem_block = 0;              // LDS bytes a workgroup may use
  int n_scatter = 0;                  // active-row scatter workgroups (0: off)
  bool scatter_global = false;        // its column sums in global memory (C too wide)
  int64_t scatter_max_rows = 0;       // largest active-row count that uses it
  std::vector<FwdGroup> groups;
  std::vector<RowItem> rows;
  std::vector<TrItem> tr, gtr;
  std::vector<int32_t> col_ts0, col_nch, gcol_ts0, gcol_nch;
  std::vector<int32_t> row_len;       // real row lengths
  std::vector<int64_t> rptr;          // row-contiguous copy: first slot per position
  int64_t blk_rows = 0;               // block-sequential sweep: rows per block (cached lists)
  std::vector<int32_t> blk_g0, blk_ng;  // its blocks' first group and group count
  Sell osell;                         // objective-row view (host tables)
  std::vector<FwdGroup> ogroups;
  bool sched_obj = false;             // iterations use the objective-row view
  bool grad_valid = false;            // gradient CSC matches (grad_kind, grad_fp)
  bool grad_sub = false;              // gradient uses the objective-row CSC
  const uint16_t* grad_kind = nullptr;
  uint64_t grad_fp = 0, last_fp = 0;
  int64_t grad_entries = 0;
  std::vector<ColBlock> cblocks;
  DevPlan hp{};
  DevPlan* d_table = nullptr;
  DevState* d_state = nullptr;
  uint32_t* d_ctr = nullptr;
  FwdGroup* d_groups = nullptr;
  FwdGroup* d_ogroups = nullptr;
  RowItem* d_rows = nullptr;
  TrItem* d_tr = nullptr;
  TrItem* d_gtr = nullptr;
  ColBlock* d_cblocks = nullptr;
  std::vector<ScItem> sc_items, ss_items;  // active-row scatter and share-sum workgroups
  ScItem* d_sc = nullptr;
  ScItem* d_ss = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t graph = nullptr;
  int graph_r = -1;
  bool fwd_dynamic = true;            // all-row forward: groups from a counter
};

namespace {

template <typename T>
T* at(fredopt_plan* p, size_t off) {
  return reinterpret_cast<T*>(p->ws + off);
}

void build_groups(int64_t n_slices, std::vector<FwdGroup>* groups) {
  groups->clear();
  for (int64_t s0 = 0; s0 < n_slices; s0 += kFwdWaves)
    groups->push_back(FwdGroup{0, (int32_t)s0,
                               (int32_t)std::min<int64_t>(kFwdWaves, n_slices - s0),
                               (int32_t)groups->size()});
}

// Groups of the objective-row view: consecutive slices, at most kFwdWaves of them, a
// group closed before it would exceed `target` steps (a slice's weight is its steps,
// the quads each of its lanes streams).  The view's passes run their groups all at
// once, one per workgroup slot, and last as long as the heaviest group; with groups of
// 8 slices the heaviest holds 1.5x the mean on the clinical plan.  target is the
// smallest weight that leaves at most `slots` groups, but not below the mean weight of
// 8-slice groups (small views are not cut into groups of single slices).
int64_t count_groups(const std::vector<int32_t>& w, int64_t target) {
  int64_t n = 0, cur = 0, in = 0;
  for (int32_t x : w) {
    if (in > 0 && (in == kFwdWaves || cur + x > target)) {
      ++n;
      cur = 0;
      in = 0;
    }
    cur += x;
    ++in;
  }
  return n + (in > 0 ? 1 : 0);
}

void build_groups_balanced(const std::vector<int32_t>& w, int64_t slots,
                           std::vector<FwdGroup>* groups) {
  groups->clear();
  const int64_t n = (int64_t)w.size();
  if (n == 0) return;
  int64_t tot = 0, wmax = 0;
  for (int32_t x : w) {
    tot += x;
    wmax = std::max<int64_t>(wmax, x);
  }
  const int64_t n8 = (n + kFwdWaves - 1) / kFwdWaves;
  int64_t lo = std::max<int64_t>(wmax, 1), hi = std::max(tot, lo);  // count(hi) = n8
  if (n8 <= slots) {
    while (lo < hi) {  // smallest target with at most `slots` groups
      const int64_t mid = lo + (hi - lo) / 2;
      if (count_groups(w, mid) <= slots) hi = mid;
      else lo = mid + 1;
    }
  }
  const int64_t target = std::max(hi, (tot + n8 - 1) / n8);
  int32_t s0 = 0, in = 0;
  int64_t cur = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (in > 0 && (in == kFwdWaves || cur + w[i] > target)) {
      groups->push_back(FwdGroup{0, s0, in, (int32_t)groups->size()});
      s0 = (int32_t)i;
      in = 0;
      cur = 0;
    }
    cur += w[i];
    ++in;
  }
  groups->push_back(FwdGroup{0, s0, in, (int32_t)groups->size()});
}

// Ranges of positions of the all-row view (per-row data are in position order).
void build_row_items(fredopt_plan* p) {
  p->rows.clear();
  const int64_t np = p->L.NP;
  for (int64_t r0 = 0; r0 < np; r0 += kRowItemRows)
    p->rows.push_back(RowItem{0, (int32_t)p->rows.size(), (int32_t)r0,
                              (int32_t)std::min(np, r0 + kRowItemRows)});
  if (p->rows.empty()) p->rows.push_back(RowItem{0, 0, 0, 0});
}

// Columns cut into chunks of about `chunk` slots (on 4-slot boundaries), kept in
// column order so that consecutive blocks cover neighbouring beamlets.  Columns
// with no entries get no chunk (their sum is 0).
void chunk_columns(const std::vector<int64_t>& cp, int64_t C, int64_t chunk,
                   std::vector<TrItem>* items, std::vector<int32_t>* ts0,
                   std::vector<int32_t>* nch) {
  items->clear();
  ts0->assign(C, 0);
  nch->assign(C, 0);
  int32_t tslot = 0;
  for (int64_t j = 0; j < C; ++j) {
    const int64_t a = cp[j], b = cp[j + 1];
    const int64_t quads = (b - a) / 4;
    const int64_t n = (b - a + chunk - 1) / chunk;
    (*ts0)[j] = tslot;
    (*nch)[j] = (int32_t)n;
    for (int64_t c = 0; c < n; ++c) {
      TrItem t{};
      t.plan = 0;
      t.col = (int32_t)j;
      t.tslot = tslot + (int32_t)c;
      t.q0 = a + 4 * (c * quads / n);
      t.q1 = a + 4 * ((c + 1) * quads / n);
      items->push_back(t);
    }
    tslot += (int32_t)n;
  }
}

void build_tr_items(fredopt_plan* p) {
  chunk_columns(p->cp, p->C, p->tr_chunk, &p->tr, &p->col_ts0, &p->col_nch);
  p->cblocks.clear();
  for (int64_t c0 = 0; c0 < p->C; c0 += kBlock)
    p->cblocks.push_back(ColBlock{0, (int32_t)p->cblocks.size(), (int32_t)c0,
                                  (int32_t)std::min<int64_t>(p->C, c0 + kBlock)});
  p->grad_valid = false;
}

fredopt_status upload_tr(fredopt_plan* p, hipStream_t s) {
  if ((int64_t)p->tr.size() > p->L.max_tr) return fail(FREDOPT_E_WORKSPACE, "chunk list too long");
  if (!p->tr.empty())
    HIPCHK(hipMemcpyAsync(p->d_tr, p->tr.data(), sizeof(TrItem) * p->tr.size(),
                          hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(at<int32_t>(p, p->L.col_tslot0), p->col_ts0.data(),
                        sizeof(int32_t) * p->C, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(at<int32_t>(p, p->L.col_nch), p->col_nch.data(), sizeof(int32_t) * p->C,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->d_cblocks, p->cblocks.data(), sizeof(ColBlock) * p->cblocks.size(),
                        hipMemcpyHostToDevice, s));
  return FREDOPT_OK;
}

// Workgroups of the active-row scatter of a plan (n shares, share w -> {plan, w})
// and of its share sum (one per 64 columns).
// n scatter workgroups, and the column update's blocks of 64 columns (every plan has
// them: the update also finishes the column-major path)
void scatter_items(int32_t plan, int n, int64_t C, std::vector<ScItem>* sc,
                   std::vector<ScItem>* ss) {
  for (int w = 0; w < n; ++w) sc->push_back(ScItem{plan, w});
  for (int64_t j = 0; j < (C + 63) / 64; ++j) ss->push_back(ScItem{plan, (int32_t)j});
}

fredopt_status upload_scatter_items(fredopt_plan* p, hipStream_t s) {
  p->sc_items.clear();
  p->ss_items.clear();
  scatter_items(0, p->n_scatter, p->C, &p->sc_items, &p->ss_items);
  if (!p->sc_items.empty())
    HIPCHK(hipMemcpyAsync(p->d_sc, p->sc_items.data(), sizeof(ScItem) * p->sc_items.size(),
                          hipMemcpyHostToDevice, s));
  // the column update runs on both projection paths: its items always exist
  if (!p->ss_items.empty())
    HIPCHK(hipMemcpyAsync(p->d_ss, p->ss_items.data(), sizeof(ScItem) * p->ss_items.size(),
                          hipMemcpyHostToDevice, s));
  return FREDOPT_OK;
}

void drop_graph(fredopt_plan* p) {
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  p->graph = nullptr;
  p->graph_r = -1;
}

fredopt_status check_params(const fredopt_params* q, bool need_iter) {
  if (!q) return fail(FREDOPT_E_ARG, "params is NULL");
  if (!(q->lambda > 0.0 && q->lambda <= 2.0))
    return fail(FREDOPT_E_ARG, "lambda must lie in (0, 2], got %g", q->lambda);
  if (!(q->alpha > 0.0 && q->alpha < 1.0))
    return fail(FREDOPT_E_ARG, "alpha must lie in (0, 1), got %g", q->alpha);
  if (!(q->eta > 0.0 && q->eta <= 1.0))
    return fail(FREDOPT_E_ARG, "eta must lie in (0, 1], got %g", q->eta);
  if (q->reductions_n < 0 || q->reductions_n > 64)
    return fail(FREDOPT_E_ARG, "reductions_n must lie in [0, 64], got %d", q->reductions_n);
  if (need_iter && q->iter_max < 0) return fail(FREDOPT_E_ARG, "iter_max must be >= 0");
  if (q->normalization < 0 || q->normalization > 2)
    return fail(FREDOPT_E_ARG, "unknown normalization %d", q->normalization);
  if (q->objective != FREDOPT_OBJECTIVE_PRINTED && q->objective != FREDOPT_OBJECTIVE_ONE_SIDED)
    return fail(FREDOPT_E_ARG, "unknown objective %d", q->objective);
  if (q->unit_direction != 0 && q->unit_direction != 1)
    return fail(FREDOPT_E_ARG, "unit_direction must be 0 or 1, got %d", q->unit_direction);
  if (q->reserved != 0) return fail(FREDOPT_E_ARG, "reserved field must be 0");
  return FREDOPT_OK;
}

// R: the plan's rows (a plan without rows takes arrays of length 0, NULL allowed)
fredopt_status check_problem_ptrs(const fredopt_problem* pr, int64_t R) {
  if (!pr) return fail(FREDOPT_E_ARG, "problem is NULL");
  if (R > 0 && (!pr->kind || !pr->dose_lo || !pr->dose_hi || !pr->cdl_lo || !pr->cdl_hi ||
                !pr->letd_max || !pr->w_feas || !pr->w_obj || !pr->dose_target ||
                !pr->cdl_target))
    return fail(FREDOPT_E_ARG, "a problem array is NULL");
  if (!(pr->c > 0.0) || !std::isfinite(pr->c))
    return fail(FREDOPT_E_ARG, "c must be positive and finite, got %g", pr->c);
  return FREDOPT_OK;
}

void set_problem(fredopt_plan* p, const fredopt_problem* pr, const fredopt_params* q,
                 double ws_fixed, float* x) {
  DevPlan& h = p->hp;
  (void)pr;  // the kernels read the gathered copies (gather_problem)
  h.prm.lambda = q->lambda;
  h.prm.alpha = q->alpha;
  h.prm.eta = q->eta;
  h.prm.c = pr->c;
  h.prm.ws_fixed = ws_fixed;
  h.prm.normalization = q->normalization;
  h.prm.reductions_n = q->reductions_n;
  h.prm.objective = q->objective;
  h.prm.unit_dir = q->unit_direction;
  h.x = x;
  h.out_dose = h.out_letd = h.out_cdl = nullptr;
}

fredopt_status upload_table(fredopt_plan* p, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(p->d_table, &p->hp, sizeof(DevPlan), hipMemcpyHostToDevice, s));
  return FREDOPT_OK;
}

fredopt_status run_problem_check(fredopt_plan* p, const fredopt_problem* pr, hipStream_t s) {
  uint32_t* flags = at<uint32_t>(p, p->L.flags);
  HIPCHK(hipMemsetAsync(flags, 0, sizeof(uint32_t) * 4, s));
  launch_check_problem(p->R, pr->kind, pr->dose_lo, pr->dose_hi, pr->cdl_lo, pr->cdl_hi,
                       pr->letd_max, pr->w_feas, pr->w_obj, pr->dose_target, pr->cdl_target,
                       flags, s);
  HIPCHK(hipGetLastError());
  uint32_t fl[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(fl, flags, sizeof fl, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const uint32_t f = fl[0];
  p->last_fp = (uint64_t)fl[2] | ((uint64_t)fl[3] << 32);
  if (f & 8u) return fail(FREDOPT_E_ARG, "problem: unknown kind bits");
  if (f & 1u) return fail(FREDOPT_E_NONFINITE, "problem: non-finite bound, target or weight");
  if (f & 2u) return fail(FREDOPT_E_ARG, "problem: lower bound above upper bound");
  if (f & 4u) return fail(FREDOPT_E_ARG, "problem: AMS weight <= 0 or objective weight < 0");
  return FREDOPT_OK;
}

// Gradient CSC for this problem: the entries of rows with objective terms (Eq. 2
// has no other non-zero coefficients), compacted column by column in row order.
// Rebuilt only when the kind array (address or fingerprint) changes; falls back to
// the full CSC when it does not fit the reserved space.
fredopt_status prepare_gradient(fredopt_plan* p, const fredopt_problem* pr, hipStream_t s) {
  DevPlan& h = p->hp;
  const Layout& L = p->L;
  uint32_t* ocount = at<uint32_t>(p, L.ocount);
  const int64_t* d_cp = at<int64_t>(p, L.cp);
  launch_obj_count(p->C, d_cp, at<uint32_t>(p, L.colcount), h.ri, pr->kind, ocount, s);
  HIPCHK(hipGetLastError());
  std::vector<uint32_t> cnt(p->C);
  HIPCHK(hipMemcpyAsync(cnt.data(), ocount, sizeof(uint32_t) * p->C, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<int64_t> ocp(p->C + 1, 0);
  int64_t real = 0;
  for (int64_t j = 0; j < p->C; ++j) {
    ocp[j + 1] = ocp[j] + (((int64_t)cnt[j] + 3) & ~int64_t(3));
    real += cnt[j];
  }
  if (ocp[p->C] <= L.obj_slots) {
    const int vb = value_bytes(p->storage);
    HIPCHK(hipMemcpyAsync(at<int64_t>(p, L.ocp), ocp.data(), sizeof(int64_t) * (p->C + 1),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(p->ws + L.gri, 0, sizeof(int32_t) * ocp[p->C], s));
    HIPCHK(hipMemsetAsync(p->ws + L.gcdv, 0, (size_t)vb * ocp[p->C], s));
    HIPCHK(hipMemsetAsync(p->ws + L.gclv, 0, (size_t)vb * ocp[p->C], s));
    launch_obj_fill(value_of(p->storage), p->C, d_cp, at<uint32_t>(p, L.colcount), h.ri, h.cdv,
                    h.clv, pr->kind, at<int64_t>(p, L.ocp), at<int32_t>(p, L.gri),
                    p->ws + L.gcdv, p->ws + L.gclv, s);
    HIPCHK(hipGetLastError());
    chunk_columns(ocp, p->C, std::min<int64_t>(p->tr_chunk, kGradChunk), &p->gtr, &p->gcol_ts0,
                  &p->gcol_nch);
    h.gri = at<int32_t>(p, L.gri);
    h.gcdv = p->ws + L.gcdv;
    h.gclv = p->ws + L.gclv;
    p->grad_sub = true;
    p->grad_entries = real;
  } else {
    p->gtr = p->tr;
    p->gcol_ts0 = p->col_ts0;
    p->gcol_nch = p->col_nch;
    h.gri = h.ri;
    h.gcdv = h.cdv;
    h.gclv = h.clv;
    p->grad_sub = false;
    p->grad_entries = p->nnz;
  }
  if ((int64_t)p->gtr.size() > L.max_tr) return fail(FREDOPT_E_WORKSPACE, "gradient chunks");
  if (!p->gtr.empty())
    HIPCHK(hipMemcpyAsync(p->d_gtr, p->gtr.data(), sizeof(TrItem) * p->gtr.size(),
                          hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(at<int32_t>(p, L.gcol_tslot0), p->gcol_ts0.data(), sizeof(int32_t) * p->C,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(at<int32_t>(p, L.gcol_nch), p->gcol_nch.data(), sizeof(int32_t) * p->C,
                        hipMemcpyHostToDevice, s));
  h.gcol_tslot0 = at<int32_t>(p, L.gcol_tslot0);
  h.gcol_nch = at<int32_t>(p, L.gcol_nch);
  HIPCHK(hipStreamSynchronize(s));
  p->grad_valid = true;
  p->grad_kind = pr->kind;
  p->grad_fp = p->last_fp;
  drop_graph(p);
  return FREDOPT_OK;
}

// Objective-row sliced-ELL view for this problem: the rows with objective terms,
// copied from the all-row view.  With it an outer iteration needs the all-row
// forward product only once (at the perturbed point); without room for it the
// iteration keeps the two all-row forward products.
fredopt_status prepare_objective_view(fredopt_plan* p, const fredopt_problem* pr, hipStream_t s) {
  DevPlan& h = p->hp;
  const Layout& L = p->L;
  p->sched_obj = false;
  h.osell = h.sell;
  drop_graph(p);
  if (L.obj_sell_slots == 0) return FREDOPT_OK;
  std::vector<uint16_t> kind(p->R);
  if (p->R > 0) {
    HIPCHK(hipMemcpyAsync(kind.data(), pr->kind, sizeof(uint16_t) * p->R, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  std::vector<int32_t> rows;
  for (int64_t i = 0; i < p->R; ++i)
    if (kind[i] & (FREDOPT_OBJ_DOSE | FREDOPT_OBJ_CDL)) rows.push_back((int32_t)i);
  const int64_t n = (int64_t)rows.size();
  Sell& O = p->osell;
  // more lanes per row than the all-row view when that leaves too few workgroups,
  // as long as every lane still gets 4 quads of an average row
  int64_t obj_nnz = 0;
  for (int64_t i = 0; i < n; ++i) obj_nnz += p->row_len[rows[i]];
  int olg = p->sell.lpr_log2;
  while (olg < 4 && n / ((kWave >> olg) * kFwdWaves) < 2 * (int64_t)p->n_cu &&
         (int64_t(16) << (olg + 1)) * n <= obj_nnz)
    ++olg;
  auto fits = [&]() {
    return O.slots <= L.obj_sell_slots && O.n_slices <= L.max_obj_slices &&
           (int64_t)O.srow.size() <= L.max_obj_srow;
  };
  for (;; --olg) {
    build_sell_list(n, [&](int64_t i) { return (int64_t)rows[i]; },
                    [&](int64_t i) { return (int64_t)p->row_len[rows[i]]; }, olg, true, &O);
    if (fits()) break;
    if (olg == p->sell.lpr_log2) return FREDOPT_OK;  // the all-row view serves instead
  }
  build_groups_balanced(O.width, std::min<int64_t>((int64_t)p->n_cu * kObjWgsPerCu,
                                                  L.max_obj_groups),
                        &p->ogroups);
  if ((int64_t)p->ogroups.size() > L.max_obj_groups) return FREDOPT_OK;
  std::vector<int32_t> src(n), len(n);
  for (int64_t i = 0; i < n; ++i) {
    src[i] = p->sell.rslice[rows[i]];
    len[i] = p->row_len[rows[i]];
  }
  const int vb = value_bytes(p->storage);
  HIPCHK(hipMemcpyAsync(p->ws + L.osbase, O.base.data(), sizeof(int64_t) * (O.n_slices + 1),
                        hipMemcpyHostToDevice, s));
  if (O.n_slices > 0) {
    HIPCHK(hipMemcpyAsync(p->ws + L.oswidth, O.width.data(), sizeof(int32_t) * O.n_slices,
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->ws + L.osrow, O.srow.data(), sizeof(int32_t) * O.srow.size(),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->d_ogroups, p->ogroups.data(), sizeof(FwdGroup) * p->ogroups.size(),
                          hipMemcpyHostToDevice, s));
  }
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(p->ws + L.pk_src, src.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->ws + L.pk_dst, O.rslice.data(), sizeof(int32_t) * n,
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->ws + L.pk_len, len.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipMemsetAsync(p->ws + L.osci, 0, (size_t)index_bytes(p->storage) * O.slots, s));
  HIPCHK(hipMemsetAsync(p->ws + L.osdv, 0, (size_t)vb * O.slots, s));
  HIPCHK(hipMemsetAsync(p->ws + L.oslv, 0, (size_t)vb * O.slots, s));
  launch_pack_sub(value_of(p->storage), p->sell.lpr_log2, olg, n, at<int32_t>(p, L.pk_src),
                  at<int32_t>(p, L.pk_dst), at<int32_t>(p, L.pk_len), h.sell.sbase, h.sell.sci,
                  h.sell.sdv, h.sell.slv, at<int64_t>(p, L.osbase), p->ws + L.osci,
                  index16(p->storage) ? 1 : 0, p->ws + L.osdv, p->ws + L.oslv, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  h.osell.sbase = at<int64_t>(p, L.osbase);
  h.osell.swidth = at<int32_t>(p, L.oswidth);
  h.osell.srow = at<int32_t>(p, L.osrow);
  h.osell.sci = p->ws + L.osci;
  h.osell.sdv = p->ws + L.osdv;
  h.osell.slv = p->ws + L.oslv;
  h.osell.n_slices = (int32_t)O.n_slices;
  h.osell.n_groups = (int32_t)p->ogroups.size();
  h.osell.lpr_log2 = olg;

  p->sched_obj = true;
  drop_graph(p);
  return FREDOPT_OK;
}

// Per-problem preprocessing (gradient CSC and objective-row view), reused while the
// kind array keeps its address and fingerprint.
fredopt_status prepare_problem(fredopt_plan* p, const fredopt_problem* pr, hipStream_t s) {
  if (p->grad_valid && p->grad_kind == pr->kind && p->grad_fp == p->last_fp) return FREDOPT_OK;
  // the objective-row view first: the gradient copy then stores that view's positions
  fredopt_status st = prepare_objective_view(p, pr, s);
  if (st != FREDOPT_OK) return st;
  if ((st = prepare_gradient(p, pr, s)) != FREDOPT_OK) return st;
  // the objective-row pass writes the gradient coefficients of objective rows only;
  // every other row's stays zero (the column-major copies' padding slots gather
  // row 0's, with value 0)
  HIPCHK(hipMemsetAsync(p->hp.gcoef, 0, sizeof(float2) * (size_t)p->hp.R, s));
  if (p->sched_obj && !p->grad_sub) {  // the view needs the objective-row gradient copy
    p->sched_obj = false;
    p->hp.osell = p->hp.sell;
  }
  drop_graph(p);
  return FREDOPT_OK;
}

// The caller's problem (row order) in the views' position orders, for one call: the
// all-row view, and (obj) the objective-row view's objective terms.
fredopt_status gather_problem(fredopt_plan* p, const fredopt_problem* pr, bool obj,
                              hipStream_t s) {
  DevPlan& h = p->hp;
  GatherArrays src{}, dst{};
  src.kind = const_cast<uint16_t*>(pr->kind);
  const float* in[9] = {pr->dose_lo, pr->dose_hi, pr->cdl_lo, pr->cdl_hi, pr->letd_max,
                        pr->w_feas, pr->w_obj, pr->dose_target, pr->cdl_target};
  const float* out[9] = {h.dlo, h.dhi, h.clo, h.chi, h.tmax, h.wf, h.wo, h.dt, h.ct};
  for (int k = 0; k < 9; ++k) {
    src.f[k] = const_cast<float*>(in[k]);
    dst.f[k] = const_cast<float*>(out[k]);
  }
  dst.kind = const_cast<uint16_t*>(h.kind);
  if (!obj) launch_gather_problem(p->L.NP, h.sell.srow, src, dst, 9, s);
  if (obj && p->sched_obj) {
    GatherArrays osrc{}, odst{};
    osrc.kind = src.kind;
    osrc.f[0] = src.f[6];  // wo, dt, ct
    osrc.f[1] = src.f[7];
    osrc.f[2] = src.f[8];
    odst.kind = const_cast<uint16_t*>(h.okind);
    odst.f[0] = const_cast<float*>(h.owo);
    odst.f[1] = const_cast<float*>(h.odt);
    odst.f[2] = const_cast<float*>(h.oct);
    launch_gather_problem((int64_t)p->osell.srow.size(), h.osell.srow, osrc, odst, 3, s);
  }
  HIPCHK(hipGetLastError());
  return FREDOPT_OK;
}

// Checks the problem, gathers it into position order and prepares the per-problem
// copies (r > 0) for one call.
fredopt_status bind_problem(fredopt_plan* p, const fredopt_problem* pr, bool prepare,
                            hipStream_t s) {
  fredopt_status st = run_problem_check(p, pr, s);
  if (st != FREDOPT_OK) return st;
  // the gradient copy's preparation reads the kinds in position order
  if ((st = gather_problem(p, pr, false, s)) != FREDOPT_OK) return st;
  if (!prepare) return FREDOPT_OK;
  if ((st = prepare_problem(p, pr, s)) != FREDOPT_OK) return st;
  return gather_problem(p, pr, true, s);
}

fredopt_status upload_state(fredopt_plan* p, const fredopt_state* st, hipStream_t s) {
  DevState d{};
  d.k = st ? st->k : 0;
  d.s = st ? st->s : -1;
  HIPCHK(hipMemcpyAsync(p->d_state, &d, sizeof d, hipMemcpyHostToDevice, s));
  return FREDOPT_OK;
}

fredopt_status download_state(fredopt_plan* p, DevState* out, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(out, p->d_state, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return FREDOPT_OK;
}

void export_state(const DevState& d, fredopt_state* st) {
  st->k = d.k;
  st->s = d.s;
  st->n_violated = d.n_violated;
  st->beta = d.beta;
  st->cost = d.cost;
  st->cost_perturbed = d.cost_y;
  st->proximity = d.proximity;
  st->grad_sq = d.G;
  st->q = d.Q;
  st->n_active = d.n_active;
  st->projection_path = d.proj_scatter;
  st->reserved = 0;
  st->active_entries = d.active_entries;
}

enum Kind {
  kKindFwd, kKindRows, kKindChunks, kKindCol, kKindFin, kKindList, kKindScatter, kKindScatterSum,
  kKindSearch, kKindProject, kKindSearchPart
};

struct Launch {
  int id;        // FREDOPT_KERNEL_*
  int kind;      // Kind
  int mode;
  int sub = 0;   // forward / finalize: objective-row view
  int vsel = kVecX;
};

// One outer iteration of Fig. 3 (reductions_n = r perturbations, then the sweep).
// With the objective-row view (obj): Eq. (2), its gradient and the direction
// products touch only rows with objective terms; the all-row forward product is
// taken once, at the perturbed point y, and feeds the constraint residuals.
// Without it: the all-row forward products at x and along g, d and l moved by the
// accepted step.  The caller sets y = x before the first iteration; the
// projection writes x and y.  fold (every plan stages its vector in LDS): the last
// perturbation's move y = y - beta g is not stored; the residual pass stages
// y - beta g and the projection update recomputes it.
// The sweep's transposed product and update.  The device picks the path per plan
// and iteration (proj_scatter); one launch runs the transposed product by the path
// each plan took.  The last launch updates every column: from the scatter shares, or
// from the chunk partials of the column-major path.
void add_projection(std::vector<Launch>* seq, int col_mode) {
  seq->push_back({FREDOPT_KERNEL_ACTIVE_LIST, kKindList, 0});
  seq->push_back({FREDOPT_KERNEL_SCATTER, kKindProject, 0});  // either path, one launch
  seq->push_back({FREDOPT_KERNEL_SCATTER_SUM, kKindScatterSum, col_mode});
}

std::vector<Launch> iteration_sequence(int r, bool obj, bool fold, bool onesided) {
  std::vector<Launch> seq;
  if (r == 0) {
    seq.push_back({FREDOPT_KERNEL_FWD_RESID, kKindFwd, kFwdResid, 0, kVecX});
    seq.push_back({FREDOPT_KERNEL_FINALIZE, kKindFin, kFinResidFwd});
    add_projection(&seq, kColProj);
    return seq;
  }
  if (obj) {
    for (int t = 0; t < r; ++t) {
      seq.push_back({FREDOPT_KERNEL_FWD_OBJ, kKindFwd, kFwdObj, 1, kVecY});
      seq.push_back({FREDOPT_KERNEL_TR_GRAD, kKindChunks, 0});
      seq.push_back({FREDOPT_KERNEL_COL, kKindCol, kColGrad});
      seq.push_back({FREDOPT_KERNEL_FWD_DIR, kKindFwd, kFwdDir, 1, kVecG});
      seq.push_back({FREDOPT_KERNEL_FINALIZE, kKindFin, t == 0 ? kFinDir0 : kFinDir, 1});
      if (onesided) {
        seq.push_back({FREDOPT_KERNEL_LINE_SEARCH, kKindSearchPart, 0, 1});
        seq.push_back({FREDOPT_KERNEL_LINE_SEARCH, kKindSearch, 0, 1});
      }
      if (!(fold && t + 1 == r)) seq.push_back({FREDOPT_KERNEL_COL, kKindCol, kColYMove});
    }
    seq.push_back({FREDOPT_KERNEL_FWD_RESID, kKindFwd, kFwdResid, 0, fold ? kVecYMove : kVecY});
    seq.push_back({FREDOPT_KERNEL_FINALIZE, kKindFin, kFinResidFwd});
    add_projection(&seq, fold ? kColProjYMove : kColProjY);
    return seq;
  }
  seq.push_back({FREDOPT_KERNEL_FWD_OBJ, kKindFwd, kFwdObj, 0, kVecX});
  for (int t = 0; t < r; ++t) {
    const bool last = t + 1 == r;
    seq.push_back({FREDOPT_KERNEL_TR_GRAD, kKindChunks, 0});
    seq.push_back({FREDOPT_KERNEL_COL, kKindCol, t == 0 ? kColGrad : kColGradMove});
    seq.push_back({FREDOPT_KERNEL_FWD_DIR, kKindFwd, kFwdDir, 0, kVecG});
    seq.push_back({FREDOPT_KERNEL_FINALIZE, kKindFin, t == 0 ? kFinDir0 : kFinDir, 0});
    if (onesided) {
      seq.push_back({FREDOPT_KERNEL_LINE_SEARCH, kKindSearchPart, 0, 0});
      seq.push_back({FREDOPT_KERNEL_LINE_SEARCH, kKindSearch, 0, 0});
    }
    seq.push_back({FREDOPT_KERNEL_ROWS, kKindRows, last ? kRowsMoveResid : kRowsMoveObj});
    seq.push_back({FREDOPT_KERNEL_FINALIZE, kKindFin, last ? kFinResidRows : kFinMoveObj});
  }
  seq.push_back({FREDOPT_KERNEL_ACTIVE_LIST, kKindList, 0});  // coefficients by row
  seq.push_back({FREDOPT_KERNEL_TR_PROJ, kKindChunks, 1});
  seq.push_back({FREDOPT_KERNEL_COL, kKindCol, kColProjMove});
  return seq;
}

// What a launch sequence needs: the plan table and the work lists of one plan or
// of a batch of plans (every work item names its plan).
struct Exec {
  int storage = 0, n_cu = 256, wgs_per_cu = 2, lds_floats = 0, n_plans = 1;
  int list_block = kFwdBlock;  // threads of the list kernel: the most rows of a group
  bool fwd_dynamic = true;
  DevPlan* table = nullptr;
  const FwdGroup* groups = nullptr;
  int n_groups = 0;
  const FwdGroup* ogroups = nullptr;
  int n_ogroups = 0;
  const RowItem* rows = nullptr;
  int n_rows = 0;
  const TrItem* tr = nullptr;
  int n_tr = 0;
  const TrItem* gtr = nullptr;
  int n_gtr = 0;
  const ColBlock* cblocks = nullptr;
  int n_cblocks = 0;
  uint32_t* ctr = nullptr;
  const ScItem* sc = nullptr;  // active-row scatter workgroups (0: off)
  int n_sc = 0;
  const ScItem* ss = nullptr;  // their share sums, 64 columns each
  int n_ss = 0;
  size_t sc_lds = 0;           // LDS bytes of a scatter workgroup (widest plan)
};

// Rows a group of the all-row view holds: kFwdWaves slices of 64 / lanes-per-row.
int group_rows(const fredopt_plan* p) { return kFwdWaves << (6 - p->sell.lpr_log2); }

Exec exec_of(const fredopt_plan* p) {
  Exec e;
  e.storage = p->storage;
  e.n_cu = p->n_cu;
  e.wgs_per_cu = p->wgs_per_cu;
  e.lds_floats = p->lds_floats;
  e.list_block = group_rows(p);
  e.fwd_dynamic = p->fwd_dynamic;
  e.table = p->d_table;
  e.groups = p->d_groups;
  e.n_groups = (int)p->groups.size();
  e.ogroups = p->d_ogroups;
  e.n_ogroups = (int)p->ogroups.size();
  e.rows = p->d_rows;
  e.n_rows = (int)p->rows.size();
  e.tr = p->d_tr;
  e.n_tr = (int)p->tr.size();
  e.gtr = p->d_gtr;
  e.n_gtr = (int)p->gtr.size();
  e.cblocks = p->d_cblocks;
  e.n_cblocks = (int)p->cblocks.size();
  e.ctr = p->d_ctr;
  e.sc = p->d_sc;
  e.n_sc = (int)p->sc_items.size();
  e.ss = p->d_ss;
  e.n_ss = (int)p->ss_items.size();
  e.sc_lds = p->scatter_global ? 0 : (size_t)p->C * sizeof(int64_t);
  return e;
}

void enqueue(const Exec& e, const Launch& l, hipStream_t s) {
  switch (l.kind) {
    case kKindFwd: {
      // the small objective-row passes take their groups round robin (no counter)
      const int n = l.sub ? e.n_ogroups : e.n_groups;
      const bool dyn = !l.sub && e.fwd_dynamic;
      // the all-row pass streams best with one workgroup per CU; the objective-row
      // passes, one group per workgroup, want more of them in flight
      const int wgs = l.sub ? kObjWgsPerCu : e.wgs_per_cu;
      const int grid = (int)std::min<int64_t>((int64_t)n, (int64_t)e.n_cu * wgs);
      launch_forward(e.storage, l.mode, l.sub, e.table, l.sub ? e.ogroups : e.groups, n,
                     std::max(grid, 1), e.lds_floats, dyn ? e.ctr : nullptr, l.vsel, s);
      break;
    }
    case kKindRows:
      launch_rows(l.mode, e.table, e.rows, e.n_rows, s);
      break;
    case kKindChunks:
      if (l.mode == 0) {
        if (e.n_gtr > 0)
          launch_tr_chunks(e.storage, 0, e.table, e.gtr, e.n_gtr, e.n_cu * kTrWgsPerCu,
                           e.n_plans == 1, s);
      } else if (e.n_tr > 0) {
        launch_tr_chunks(e.storage, 1, e.table, e.tr, e.n_tr, e.n_cu * kTrWgsPerCu,
                         e.n_plans == 1, s);
      }
      break;
    case kKindCol:
      launch_tcol(l.mode, e.table, e.cblocks, e.n_cblocks, s);
      break;
    case kKindList:  // active-row list, or the coefficients by row for the CSC path
      launch_active_list(e.table, e.groups, e.n_groups, e.list_block, s);
      break;
    case kKindScatter:
      launch_scatter(e.storage, e.table, e.sc, e.n_sc, e.sc_lds, s);
      break;
    case kKindProject: {
      // the chunk walk's workgroups per CU: two unless the scatter's LDS sums leave
      // room for one (the same waves per CU as the separate chunk kernel when two fit)
      const int per_cu = e.sc_lds <= kProjectTwoPerCuLds ? 2 : 1;
      launch_project(e.storage, e.table, e.sc, e.n_sc, e.sc_lds, e.tr, e.n_tr, e.n_cu * per_cu,
                     e.n_plans == 1, s);
      break;
    }
    case kKindScatterSum:
      if (e.n_ss > 0) launch_scatter_sum(l.mode, e.table, e.ss, e.n_ss, s);
      break;
    case kKindSearchPart:
      launch_search_part(l.sub, e.table, e.n_plans, s);
      break;
    case kKindSearch:
      launch_linesearch(l.sub, e.table, e.n_plans, s);
      break;
    default:
      launch_finalize(l.mode, l.sub, e.table, e.n_plans, s);
      break;
  }
}

void enqueue(fredopt_plan* p, const Launch& l, hipStream_t s) { enqueue(exec_of(p), l, s); }

// The iteration for an exec: the last move folded when every plan stages its vector
// in LDS; the step search kernel with the one-sided objective.
std::vector<Launch> sequence_of(const Exec& e, int r, bool obj, bool onesided) {
  return iteration_sequence(r, obj, e.lds_floats > 0, onesided);
}

// Graphs are captured per (reductions_n, objective): the one-sided objective adds
// the step search to the sequence.
int graph_key(int r, int objective) { return 2 * r + (objective ? 1 : 0); }

fredopt_status enqueue_iteration(fredopt_plan* p, int r, hipStream_t s) {
  const Exec e = exec_of(p);
  for (const Launch& l : sequence_of(e, r, p->sched_obj, p->hp.prm.objective != 0))
    enqueue(e, l, s);
  HIPCHK(hipGetLastError());
  return FREDOPT_OK;
}

// One outer iteration captured on `cap` (a stream of its own) into *graph.
fredopt_status capture_iteration(const Exec& e, int r, bool obj, bool onesided, hipStream_t cap,
                                 hipGraphExec_t* graph) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  for (const Launch& l : sequence_of(e, r, obj, onesided)) enqueue(e, l, cap);
  const hipError_t le = hipGetLastError();
  const hipError_t ce = hipStreamEndCapture(cap, &g);
  if (le != hipSuccess || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(FREDOPT_E_DEVICE, "graph capture failed: %s",
                hipGetErrorString(le != hipSuccess ? le : ce));
  }
  const hipError_t ie = hipGraphInstantiate(graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    *graph = nullptr;
    return fail(FREDOPT_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(ie));
  }
  return FREDOPT_OK;
}

fredopt_status ensure_graph(fredopt_plan* p, int r) {
  const int key = graph_key(r, p->hp.prm.objective);
  if (p->graph && p->graph_r == key) return FREDOPT_OK;
  drop_graph(p);
  // a plan loaded without allocation gets its capture stream here
  if (!p->cap) HIPCHK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
  const fredopt_status st = capture_iteration(exec_of(p), r, p->sched_obj,
                                              p->hp.prm.objective != 0, p->cap, &p->graph);
  if (st != FREDOPT_OK) return st;
  p->graph_r = key;
  return FREDOPT_OK;
}

// Lanes per active row of the scatter: enough 4-entry quads for a mean row in one
// step, from 4 to 64 (a wave takes 64 / lanes rows at once).
int scatter_lanes_log2(int64_t R, int64_t nnz) {
  const int64_t quads = R > 0 ? (nnz / R + 3) / 4 : 1;
  int lg = 2;
  while (lg < 6 && (int64_t(1) << lg) < quads) ++lg;
  return lg;
}

// Default workgroups of the active-row scatter: one per 64k stored entries (each
// zeroes and writes C column sums, so a small plan wants few), at most one per CU.
int default_scatter_wgs(const fredopt_plan* p) {
  return (int)std::min<int64_t>(std::min<int64_t>(p->n_cu, kScatterMaxWGs),
                                1 + p->nnz / (int64_t(1) << 16));
}

fredopt_status device_limits(fredopt_plan* p) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  p->device = dev;
  int ncu = 0, smem_block = 0, smem_sm = 0;
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipDeviceGetAttribute(&smem_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (hipDeviceGetAttribute(&smem_sm, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
          hipSuccess ||
      smem_sm <= 0)
    smem_sm = smem_block;
  p->n_cu = ncu > 0 ? ncu : 256;
  p->smem_block = (size_t)std::max(smem_block, 0);
  // dynamic LDS limit of the kernels that stage vectors: what the device allows
  // next to their static LDS (plans of every size share the kernels)
  const size_t static_lds = 2048;
  const size_t dyn_max = p->smem_block > static_lds ? p->smem_block - static_lds : 0;
  for (int vt = FREDOPT_F32; vt <= FREDOPT_BF16_IDX16; ++vt)
    HIPCHK(set_forward_lds_limit(vt, dyn_max));
  HIPCHK(set_scatter_lds_limit(dyn_max));
  HIPCHK(set_project_lds_limit(dyn_max));
  const size_t need = (size_t)p->C * sizeof(float);
  if (need <= dyn_max) {
    p->lds_floats = (int)p->C;
    const int fit = (int)std::max<size_t>(1, (size_t)std::max(smem_sm, 1) / (need + static_lds));
    p->max_wgs_per_cu = std::min(4, fit);  // 4 x 512 threads = 32 waves per CU
  } else {
    p->lds_floats = 0;
    p->max_wgs_per_cu = 4;
  }
  // the scatter's C column sums: in LDS when they fit, else in global memory
  const size_t sneed = (size_t)p->C * sizeof(int64_t);
  p->scatter_global = !(scatter_fits(p->C) && sneed <= dyn_max);
  p->n_scatter = default_scatter_wgs(p);
  p->scatter_max_rows = p->R / 4;
  // workgroups per CU of the all-row streaming pass, as measured on the clinical
  // plan: one 8-wave workgroup for FP32; two for 16-bit values, whose steps carry
  // half the bytes, so a CU needs more waves in flight to keep HBM busy
  p->wgs_per_cu = std::min(p->storage == FREDOPT_F32 ? 1 : 2, p->max_wgs_per_cu);
  return FREDOPT_OK;
}

size_t exact_bytes(int64_t R, int64_t C, const int64_t* rp, int storage, int lpr_log2,
                   int reserve_pct) {
  Sell S;
  build_sell(rp, R, lpr_log2, false, &S);
  Layout L;
  if (!make_layout(R, C, rp[R], storage, lpr_log2, S.slots, S.n_slices, reserve_pct, &L))
    return 0;
  return L.total;
}

// Staging area of fredopt_load_matrices_noalloc: host matrices are copied here
// instead of into a buffer the library allocates.  Each device holds its own copy
// of this array from module load until the process ends.  In host code the name is
// a host-side stand-in, never a device address: the address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
constexpr size_t kNoallocStagingBytes = size_t(128) << 20;
__device__ __align__(256) unsigned char scratch[kNoallocStagingBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];    // held for the whole call that uses the area
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

// The device address of `scratch` on device dev (the current device); looked up on
// the first call on that device.  The caller holds g_scratch_mu[dev].
fredopt_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(FREDOPT_E_DEVICE, "device %d beyond the %d the staging table covers", dev,
                kMaxDevices);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FREDOPT_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FREDOPT_OK;
}

}  // namespace

// =============================================================================== ABI

extern "C" {

const char* fredopt_last_error(void) { return g_err.c_str(); }

size_t fredopt_workspace_bytes(int64_t n_rows, int64_t n_cols, int64_t nnz, int32_t storage) {
  Layout L;
  if (!bound_layout(n_rows, n_cols, nnz, storage, auto_lpr_log2(n_rows, nnz),
                    kDefaultGradientReservePct, &L))
    return 0;
  return L.total;
}

size_t fredopt_workspace_bytes_csr(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr,
                                   int32_t storage, int32_t lanes_per_row,
                                   int32_t gradient_reserve_pct) {
  if (!row_ptr || n_rows < 0 || n_cols < 1) return 0;
  int lg = 0;
  if (!lpr_log2_of(lanes_per_row, n_rows, row_ptr[n_rows], &lg)) return 0;
  for (int64_t i = 0; i < n_rows; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return 0;
  if (row_ptr[0] != 0) return 0;
  return exact_bytes(n_rows, n_cols, row_ptr, storage, lg, reserve_pct_of(gradient_reserve_pct));
}

// The load of Table 2 step (iii).  noalloc: host matrices are staged in `scratch`
// (at most kNoallocStagingBytes, one call per device at a time) instead of a buffer
// allocated here, and the plan's capture stream is created by its first solve.
static fredopt_status load_impl(const fredopt_matrices* m, void* workspace,
                                size_t workspace_bytes, void* stream, fredopt_plan** out,
                                bool noalloc) {
  if (!m || !out) return fail(FREDOPT_E_ARG, "matrices and out must be non-NULL");
  *out = nullptr;
  const int64_t R = m->n_rows, C = m->n_cols, nnz = m->nnz;
  int lg = 0;
  Layout Lb;
  const int pct = reserve_pct_of(m->gradient_reserve_pct);
  if (!lpr_log2_of(m->lanes_per_row, R, nnz, &lg) ||
      !bound_layout(R, C, nnz, m->storage, lg, pct, &Lb))
    return fail(FREDOPT_E_SHAPE, "invalid sizes, storage or layout (rows %lld cols %lld nnz %lld)",
                (long long)R, (long long)C, (long long)nnz);
  if (!m->row_ptr || (nnz > 0 && (!m->col_idx || !m->d_val || !m->l_val)))
    return fail(FREDOPT_E_ARG, "matrix array is NULL");
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
    return fail(FREDOPT_E_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);

  // host copy of the row pointers: validation, slicing, work lists
  std::vector<int64_t> h_rp(R + 1);
  if (m->on_device) {
    HIPCHK(hipMemcpyAsync(h_rp.data(), m->row_ptr, sizeof(int64_t) * (R + 1),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  } else {
    std::memcpy(h_rp.data(), m->row_ptr, sizeof(int64_t) * (R + 1));
  }
  if (h_rp[0] != 0 || h_rp[R] != nnz)
    return fail(FREDOPT_E_SHAPE, "row_ptr[0] != 0 or row_ptr[n] != nnz");
  for (int64_t i = 0; i < R; ++i)
    if (h_rp[i + 1] < h_rp[i]) return fail(FREDOPT_E_SHAPE, "row_ptr decreases at row %lld", (long long)i);
  for (int64_t i = 0; i < R; ++i)
    if (h_rp[i + 1] - h_rp[i] > C)
      return fail(FREDOPT_E_INDEX, "row %lld has more entries than columns", (long long)i);

  fredopt_plan* p = new fredopt_plan();
  p->R = R;
  p->C = C;
  p->nnz = nnz;
  p->storage = m->storage;
  p->ws = static_cast<char*>(workspace);
  p->ws_bytes = workspace_bytes;
  build_sell(h_rp.data(), R, lg, true, &p->sell);
  p->row_len.resize(R);
  for (int64_t i = 0; i < R; ++i) p->row_len[i] = (int32_t)(h_rp[i + 1] - h_rp[i]);
  if (!make_layout(R, C, nnz, m->storage, lg, p->sell.slots, p->sell.n_slices, pct, &p->L)) {
    delete p;
    return fail(FREDOPT_E_SHAPE, "layout failed");
  }
  const Layout& L = p->L;
  if (workspace_bytes < L.total) {
    const size_t need = L.total;
    delete p;
    return fail(FREDOPT_E_WORKSPACE, "workspace too small: %zu < %zu", workspace_bytes, need);
  }
  fredopt_status st = device_limits(p);
  if (st != FREDOPT_OK) {
    delete p;
    return st;
  }
  DeviceGuard guard(p->device);

  // device view of the input CSR (staged for host input)
  void* staging = nullptr;
  bool own_staging = false;                // allocated by this call, freed at its end
  std::unique_lock<std::mutex> staging_lock;  // noalloc: the device's staging area
  const int64_t* in_rp = m->row_ptr;
  const int32_t* in_col = m->col_idx;
  const float* in_dv = m->d_val;
  const float* in_lv = m->l_val;
  auto cleanup = [&](fredopt_status code) {
    if (staging) {
      if (own_staging)
        (void)hipFree(staging);
      else  // no kernel may still read the shared staging area once the lock is released
        (void)hipStreamSynchronize(s);
    }
    if (code != FREDOPT_OK) {
      if (p->cap) (void)hipStreamDestroy(p->cap);
      delete p;
    }
    return code;
  };
#define LCHK(expr)                                                                           \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return cleanup(fail(FREDOPT_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_))); \
  } while (0)
  if (!m->on_device) {
    const size_t bytes = align_up(sizeof(int64_t) * (R + 1)) + align_up(sizeof(int32_t) * nnz) +
                         2 * align_up(sizeof(float) * nnz);
    if (noalloc) {
      if (bytes > kNoallocStagingBytes)
        return cleanup(fail(FREDOPT_E_WORKSPACE,
                            "host matrices need %zu staging bytes; the no-allocation load "
                            "stages at most %zu (load device-resident matrices instead)",
                            bytes, kNoallocStagingBytes));
      if (p->device < 0 || p->device >= kMaxDevices)
        return cleanup(fail(FREDOPT_E_DEVICE, "device %d beyond the staging table", p->device));
      staging_lock = std::unique_lock<std::mutex>(g_scratch_mu[p->device]);
      const fredopt_status se = scratch_address(p->device, &staging);
      if (se != FREDOPT_OK) return cleanup(se);
    } else {
      LCHK(hipMalloc(&staging, bytes));
      own_staging = true;
    }
    char* b = static_cast<char*>(staging);
    int64_t* srp = reinterpret_cast<int64_t*>(b);
    b += align_up(sizeof(int64_t) * (R + 1));
    int32_t* scol = reinterpret_cast<int32_t*>(b);
    b += align_up(sizeof(int32_t) * nnz);
    float* sdv = reinterpret_cast<float*>(b);
    b += align_up(sizeof(float) * nnz);
    float* slv = reinterpret_cast<float*>(b);
    LCHK(hipMemcpyAsync(srp, m->row_ptr, sizeof(int64_t) * (R + 1), hipMemcpyHostToDevice, s));
    if (nnz > 0) {
      LCHK(hipMemcpyAsync(scol, m->col_idx, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
      LCHK(hipMemcpyAsync(sdv, m->d_val, sizeof(float) * nnz, hipMemcpyHostToDevice, s));
      LCHK(hipMemcpyAsync(slv, m->l_val, sizeof(float) * nnz, hipMemcpyHostToDevice, s));
    }
    in_rp = srp;
    in_col = scol;
    in_dv = sdv;
    in_lv = slv;
  }

  char* ws = p->ws;
  uint32_t* flags = reinterpret_cast<uint32_t*>(ws + L.flags);
  uint32_t* colcount = reinterpret_cast<uint32_t*>(ws + L.colcount);
  uint32_t* colmax = reinterpret_cast<uint32_t*>(ws + L.colmax);
  float* cscale = reinterpret_cast<float*>(ws + L.cscale);
  const bool q16 = m->storage != FREDOPT_F32;
  const int vb = value_bytes(m->storage);

  LCHK(hipMemsetAsync(ws + L.flags, 0, sizeof(uint32_t) * 4, s));
  LCHK(hipMemsetAsync(ws + L.ctr, 0, sizeof(uint32_t) * kCounters, s));
  LCHK(hipMemsetAsync(ws + L.colcount, 0, sizeof(uint32_t) * C, s));
  LCHK(hipMemsetAsync(ws + L.colmax, 0, sizeof(uint32_t) * C, s));
  LCHK(hipMemsetAsync(ws + L.state, 0, sizeof(DevState), s));
  launch_validate(R, C, in_rp, in_col, in_dv, in_lv, flags, s);
  LCHK(hipGetLastError());
  uint32_t f = 0;
  LCHK(hipMemcpyAsync(&f, flags, sizeof f, hipMemcpyDeviceToHost, s));
  LCHK(hipStreamSynchronize(s));
  if (f & 1u) return cleanup(fail(FREDOPT_E_INDEX, "column index out of range"));
  if (f & 2u) return cleanup(fail(FREDOPT_E_INDEX, "column indices not strictly increasing in a row"));
  if (f & 4u) return cleanup(fail(FREDOPT_E_NONFINITE, "non-finite or negative influence value"));

  launch_col_stats(nnz, in_rp, in_col, in_dv, in_lv, colcount, q16 ? colmax : nullptr, s);
  if (q16) launch_col_scale(C, colmax, cscale, s);
  LCHK(hipGetLastError());
  std::vector<uint32_t> h_cc(C);
  LCHK(hipMemcpyAsync(h_cc.data(), colcount, sizeof(uint32_t) * C, hipMemcpyDeviceToHost, s));
  LCHK(hipStreamSynchronize(s));
  p->cp.assign(C + 1, 0);
  for (int64_t j = 0; j < C; ++j) p->cp[j + 1] = p->cp[j] + (((int64_t)h_cc[j] + 3) & ~int64_t(3));
  if (p->cp[C] > L.csc_slots)
    return cleanup(fail(FREDOPT_E_WORKSPACE, "padded CSC exceeds the workspace bound"));

  // sliced-ELL copy
  const Sell& S = p->sell;
  int64_t* d_sbase = reinterpret_cast<int64_t*>(ws + L.sbase);
  int32_t* d_rslice = reinterpret_cast<int32_t*>(ws + L.rslice);
  void* sci = ws + L.sci;
  const int vt = value_of(m->storage);  // value conversion of the load kernels
  LCHK(hipMemcpyAsync(d_sbase, S.base.data(), sizeof(int64_t) * (S.n_slices + 1),
                      hipMemcpyHostToDevice, s));
  if (S.n_slices > 0) {
    LCHK(hipMemcpyAsync(ws + L.swidth, S.width.data(), sizeof(int32_t) * S.n_slices,
                        hipMemcpyHostToDevice, s));
    LCHK(hipMemcpyAsync(ws + L.srow, S.srow.data(), sizeof(int32_t) * S.srow.size(),
                        hipMemcpyHostToDevice, s));
  }
  if (R > 0)
    LCHK(hipMemcpyAsync(d_rslice, S.rslice.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice, s));
  LCHK(hipMemsetAsync(sci, 0, (size_t)index_bytes(m->storage) * S.slots, s));
  LCHK(hipMemsetAsync(ws + L.sdv, 0, (size_t)vb * S.slots, s));
  LCHK(hipMemsetAsync(ws + L.slv, 0, (size_t)vb * S.slots, s));
  const float* scale = q16 ? cscale : nullptr;
  launch_pack_sell(vt, R, S.lpr_log2, in_rp, in_col, in_dv, in_lv, scale, d_rslice, d_sbase,
                   sci, index16(m->storage) ? 1 : 0, ws + L.sdv, ws + L.slv, s);

  // row-contiguous copy (active-row scatter), rows at their positions, each padded to
  // a multiple of 4 slots
  {
    const int64_t NP = (int64_t)S.srow.size();
    p->rptr.assign(NP + 1, 0);
    for (int64_t sp = 0; sp < NP; ++sp) {
      const int32_t row = S.srow[sp];
      const int64_t len = row >= 0 ? h_rp[row + 1] - h_rp[row] : 0;
      p->rptr[sp + 1] = p->rptr[sp] + ((len + 3) & ~int64_t(3));
    }
    if (p->rptr[NP] > L.row_slots)
      return cleanup(fail(FREDOPT_E_WORKSPACE, "row copy exceeds the workspace bound"));
    const size_t Pm1 = (size_t)std::max<int64_t>(L.NP, 1);
    LCHK(hipMemsetAsync(ws + L.rptr, 0, sizeof(int64_t) * (Pm1 + 1), s));
    LCHK(hipMemcpyAsync(ws + L.rptr, p->rptr.data(), sizeof(int64_t) * (NP + 1),
                        hipMemcpyHostToDevice, s));
    LCHK(hipMemsetAsync(ws + L.plen, 0, sizeof(int32_t) * Pm1, s));
    const size_t rs = (size_t)std::max<int64_t>(p->rptr[NP], 1);
    LCHK(hipMemsetAsync(ws + L.rci, 0, (size_t)index_bytes(m->storage) * rs, s));
    LCHK(hipMemsetAsync(ws + L.rdv, 0, (size_t)vb * rs, s));
    LCHK(hipMemsetAsync(ws + L.rlv, 0, (size_t)vb * rs, s));
    launch_pack_rows(vt, R, in_rp, in_col, in_dv, in_lv, scale, d_rslice,
                     reinterpret_cast<const int64_t*>(ws + L.rptr), ws + L.rci,
                     index16(m->storage) ? 1 : 0, ws + L.rdv, ws + L.rlv,
                     reinterpret_cast<int32_t*>(ws + L.plen), s);
  }

  // CSC: zero (padding slots keep row 0, value 0), per-block counts, offsets, fill
  int64_t* d_cp = reinterpret_cast<int64_t*>(ws + L.cp);
  int32_t* ri = reinterpret_cast<int32_t*>(ws + L.ri);
  LCHK(hipMemcpyAsync(d_cp, p->cp.data(), sizeof(int64_t) * (C + 1), hipMemcpyHostToDevice, s));
  LCHK(hipMemsetAsync(ri, 0, sizeof(int32_t) * p->cp[C], s));
  LCHK(hipMemsetAsync(ws + L.cdv, 0, (size_t)vb * p->cp[C], s));
  LCHK(hipMemsetAsync(ws + L.clv, 0, (size_t)vb * p->cp[C], s));
  uint32_t* bc = reinterpret_cast<uint32_t*>(ws + L.bc);
  LCHK(hipMemsetAsync(bc, 0, sizeof(uint32_t) * L.nb * C, s));
  launch_block_count(R, C, (int)L.rows_per_block, in_rp, in_col, bc, s);
  launch_block_offsets(C, (int)L.nb, d_cp, bc, s);
  launch_fill_csc(vt, R, C, (int)L.rows_per_block, in_rp, in_col, in_dv, in_lv, scale, bc, ri,
                  ws + L.cdv, ws + L.clv, s);
  // per-row data in position order; padding positions stay zero
  const size_t Pm = (size_t)std::max<int64_t>(L.NP, 1);
  LCHK(hipMemsetAsync(ws + L.mom, 0, sizeof(double) * 3 * Pm, s));
  LCHK(hipMemsetAsync(ws + L.rsum, 0, sizeof(float) * 2 * Pm, s));
  launch_moments(vt, R, in_rp, in_col, in_dv, in_lv, scale, d_rslice,
                 reinterpret_cast<double*>(ws + L.mom), reinterpret_cast<float*>(ws + L.rsum), s);
  LCHK(hipGetLastError());

  // plan descriptor and work lists
  p->d_table = reinterpret_cast<DevPlan*>(ws + L.table);
  p->d_state = reinterpret_cast<DevState*>(ws + L.state);
  p->d_ctr = reinterpret_cast<uint32_t*>(ws + L.ctr);
  p->d_groups = reinterpret_cast<FwdGroup*>(ws + L.groups);
  p->d_ogroups = reinterpret_cast<FwdGroup*>(ws + L.ogroups);
  p->d_rows = reinterpret_cast<RowItem*>(ws + L.row_items);
  p->d_tr = reinterpret_cast<TrItem*>(ws + L.tr_items);
  p->d_gtr = reinterpret_cast<TrItem*>(ws + L.gtr_items);
  p->d_cblocks = reinterpret_cast<ColBlock*>(ws + L.col_blocks);
  build_groups(S.n_slices, &p->groups);
  build_row_items(p);
  build_tr_items(p);
  DevPlan& h = p->hp;
  std::memset(&h, 0, sizeof h);
  h.R = R;
  h.C = C;
  h.vtype = m->storage;
  h.lpr_log2 = S.lpr_log2;
  h.sell.lpr_log2 = S.lpr_log2;
  h.n_row_items = (int32_t)p->rows.size();
  h.n_col_blocks = (int32_t)p->cblocks.size();
  h.sell.n_slices = (int32_t)S.n_slices;
  h.sell.n_groups = (int32_t)p->groups.size();
  h.sell.sbase = d_sbase;
  h.sell.swidth = reinterpret_cast<const int32_t*>(ws + L.swidth);
  h.sell.srow = reinterpret_cast<const int32_t*>(ws + L.srow);
  h.sell.sci = sci;
  h.sell.sdv = ws + L.sdv;
  h.sell.slv = ws + L.slv;
  h.osell = h.sell;
  h.y = reinterpret_cast<float*>(ws + L.y);
  h.ri = ri;
  h.cdv = ws + L.cdv;
  h.clv = ws + L.clv;
  h.col_tslot0 = reinterpret_cast<const int32_t*>(ws + L.col_tslot0);
  h.col_nch = reinterpret_cast<const int32_t*>(ws + L.col_nch);
  h.gri = ri;  // until a problem is prepared
  h.gcdv = h.cdv;
  h.gclv = h.clv;
  h.gcol_tslot0 = h.col_tslot0;
  h.gcol_nch = h.col_nch;
  h.cscale = scale;
  h.mom = reinterpret_cast<const double*>(ws + L.mom);
  h.d = reinterpret_cast<float*>(ws + L.d);
  h.l = reinterpret_cast<float*>(ws + L.l);
  h.dg = reinterpret_cast<float*>(ws + L.dg);
  h.lg = reinterpret_cast<float*>(ws + L.lg);
  h.coef = reinterpret_cast<float2*>(ws + L.coef);
  h.NP = L.NP;
  {
    float* pf = reinterpret_cast<float*>(ws + L.pf);
    h.kind = reinterpret_cast<const uint16_t*>(ws + L.pkind);
    const float** fp[9] = {&h.dlo, &h.dhi, &h.clo, &h.chi, &h.tmax, &h.wf, &h.wo, &h.dt, &h.ct};
    for (int k = 0; k < 9; ++k) *fp[k] = pf + (size_t)k * Pm;
    const size_t Om = (size_t)std::max<int64_t>(L.max_obj_srow, 1);
    float* of = reinterpret_cast<float*>(ws + L.of);
    h.okind = reinterpret_cast<const uint16_t*>(ws + L.okind);
    h.owo = of;
    h.odt = of + Om;
    h.oct = of + 2 * Om;
    float* ov = reinterpret_cast<float*>(ws + L.ovec);
    h.od = ov;
    h.ol = ov + Om;
    h.odg = ov + 2 * Om;
    h.olg = ov + 3 * Om;
    h.gcoef = reinterpret_cast<float2*>(ws + L.gcoef);
    h.coef_row = reinterpret_cast<float2*>(ws + L.coef_row);
  }
  h.g = reinterpret_cast<float*>(ws + L.g);
  h.spart_a = reinterpret_cast<double*>(ws + L.spart_a);
  h.spart_b = reinterpret_cast<double*>(ws + L.spart_b);
  // the step search's first-window sums (kSearchWindow doubles per workgroup) reuse it
  h.search_cap = (int32_t)std::min<int64_t>(
      (int64_t)kNPart * std::max(L.n_groups, L.max_obj_groups) / kSearchWindow, 1 << 30);
  h.search_pad = 0;
  h.rpart = reinterpret_cast<double*>(ws + L.rpart);
  h.gpart = reinterpret_cast<double*>(ws + L.gpart);
  h.tpart = reinterpret_cast<float*>(ws + L.tpart);
  h.rsum = reinterpret_cast<const float*>(ws + L.rsum);
  h.goff = reinterpret_cast<int32_t*>(ws + L.goff);
  h.alist = reinterpret_cast<ActRow*>(ws + L.alist);
  h.spart = reinterpret_cast<int64_t*>(ws + L.spart);
  h.smask = reinterpret_cast<uint64_t*>(ws + L.smask);
  h.n_scatter = p->n_scatter;
  h.scatter_global = p->scatter_global ? 1 : 0;
  h.rptr = reinterpret_cast<const int64_t*>(ws + L.rptr);
  h.plen = reinterpret_cast<const int32_t*>(ws + L.plen);
  h.rci = ws + L.rci;
  h.rdv = ws + L.rdv;
  h.rlv = ws + L.rlv;
  h.sc_lg2 = scatter_lanes_log2(R, nnz);
  h.scatter_max_rows = (int32_t)std::min<int64_t>(p->scatter_max_rows, INT32_MAX);
  h.st = p->d_state;
  p->d_sc = reinterpret_cast<ScItem*>(ws + L.sc_items);
  p->d_ss = reinterpret_cast<ScItem*>(ws + L.ss_items);
  st = upload_scatter_items(p, s);
  if (st != FREDOPT_OK) return cleanup(st);
  h.prm.ws_fixed = -1.0;
  if ((int64_t)p->groups.size() > L.n_groups || (int64_t)p->rows.size() > L.max_rows)
    return cleanup(fail(FREDOPT_E_WORKSPACE, "work lists exceed the workspace bound"));
  if (!p->groups.empty())
    LCHK(hipMemcpyAsync(p->d_groups, p->groups.data(), sizeof(FwdGroup) * p->groups.size(),
                        hipMemcpyHostToDevice, s));
  LCHK(hipMemcpyAsync(p->d_rows, p->rows.data(), sizeof(RowItem) * p->rows.size(),
                      hipMemcpyHostToDevice, s));
  st = upload_tr(p, s);
  if (st != FREDOPT_OK) return cleanup(st);
  LCHK(hipMemsetAsync(h.g, 0, sizeof(float) * C, s));
  LCHK(hipMemsetAsync(h.coef, 0, sizeof(float2) * Pm, s));
  LCHK(hipMemsetAsync(ws + L.pkind, 0, sizeof(uint16_t) * Pm, s));
  LCHK(hipMemsetAsync(ws + L.pf, 0, sizeof(float) * 9 * Pm, s));
  LCHK(hipMemsetAsync(h.spart_a, 0, sizeof(double) * kNPart * L.n_groups, s));
  LCHK(hipMemsetAsync(h.spart_b, 0, sizeof(double) * kNPart * L.n_groups, s));
  // global column sums of the scatter start at zero (the column update re-zeroes them)
  if (p->scatter_global) LCHK(hipMemsetAsync(h.spart, 0, sizeof(int64_t) * C, s));
  st = upload_table(p, s);
  if (st != FREDOPT_OK) return cleanup(st);
  if (!noalloc) LCHK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
  LCHK(hipStreamSynchronize(s));
#undef LCHK
  *out = p;
  return cleanup(FREDOPT_OK);
}

fredopt_status fredopt_load_matrices(const fredopt_matrices* m, void* workspace,
                                     size_t workspace_bytes, void* stream, fredopt_plan** out) {
  return load_impl(m, workspace, workspace_bytes, stream, out, false);
}

fredopt_status fredopt_load_matrices_noalloc(const fredopt_matrices* m, void* workspace,
                                             size_t workspace_bytes, void* stream,
                                             fredopt_plan** out) {
  return load_impl(m, workspace, workspace_bytes, stream, out, true);
}

fredopt_status fredopt_free_plan(fredopt_plan* p) {
  if (!p) return fail(FREDOPT_E_ARG, "plan is NULL");
  {
    DeviceGuard guard(p->device);
    drop_graph(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
  }
  delete p;
  return FREDOPT_OK;
}

fredopt_status fredopt_get_plan_info(const fredopt_plan* p, fredopt_plan_info* info) {
  if (!p || !info) return fail(FREDOPT_E_ARG, "plan and info must be non-NULL");
  std::memset(info, 0, sizeof *info);
  info->n_rows = p->R;
  info->n_cols = p->C;
  info->nnz = p->nnz;
  info->sell_slots = p->sell.slots;
  info->csc_slots = p->cp.empty() ? 0 : p->cp[p->C];
  info->bytes_per_sell_slot = index_bytes(p->storage) + 2 * value_bytes(p->storage);
  info->bytes_per_csc_slot = 4 + 2 * value_bytes(p->storage);
  info->n_slices = p->sell.n_slices;
  info->tr_items = (int64_t)p->tr.size();
  info->row_items = (int64_t)p->rows.size();
  info->workspace_bytes = (int64_t)p->L.total;
  info->grad_entries = p->grad_valid ? p->grad_entries : 0;
  int64_t oe = 0;
  if (p->grad_valid && p->sched_obj)
    for (int32_t row : p->osell.srow)
      if (row >= 0) oe += p->row_len[row];
  info->obj_entries = oe;
  info->schedule = p->sched_obj ? 1 : 0;
  info->storage = p->storage;
  info->lanes_per_row = 1 << p->sell.lpr_log2;
  info->fwd_grid = (int32_t)std::min<int64_t>((int64_t)p->groups.size(),
                                              (int64_t)p->n_cu * p->wgs_per_cu);
  info->tr_chunk = p->tr_chunk;
  info->lds_x = p->lds_floats > 0 ? 1 : 0;
  info->scatter_wgs = p->n_scatter;
  info->scatter_max_rows = p->scatter_max_rows;
  info->obj_lanes_per_row = p->sched_obj ? 1 << p->hp.osell.lpr_log2 : 0;
  info->fwd_schedule = p->fwd_dynamic ? 1 : 2;
  info->scatter_lanes = 1 << p->hp.sc_lg2;
  info->row_copy_slots = p->rptr.empty() ? 0 : p->rptr.back();
  return FREDOPT_OK;
}

fredopt_status fredopt_dose_let(fredopt_plan* p, const float* x, double c, float* dose,
                                float* letd, float* cdl, void* stream) {
  if (!p || !x) return fail(FREDOPT_E_ARG, "plan and x must be non-NULL");
  if (!(c > 0.0) || !std::isfinite(c)) return fail(FREDOPT_E_ARG, "c must be positive and finite");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevPlan& h = p->hp;
  h.x = const_cast<float*>(x);
  h.prm.c = c;
  h.out_dose = dose;
  h.out_letd = letd;
  h.out_cdl = cdl;
  fredopt_status st = upload_table(p, s);
  h.out_dose = h.out_letd = h.out_cdl = nullptr;
  if (st != FREDOPT_OK) return st;
  if (dose || letd || cdl) enqueue(p, Launch{0, kKindFwd, kFwdDoseLet, 0, kVecX}, s);
  HIPCHK(hipGetLastError());
  return FREDOPT_OK;
}

fredopt_status fredopt_project_sweep(fredopt_plan* p, const fredopt_problem* pr,
                                     const fredopt_params* q, double weight_scale,
                                     float* x_inout, double* proximity_out, void* stream) {
  if (!p || !x_inout) return fail(FREDOPT_E_ARG, "plan and x must be non-NULL");
  fredopt_status st = check_problem_ptrs(pr, p->R);
  if (st != FREDOPT_OK) return st;
  if ((st = check_params(q, false)) != FREDOPT_OK) return st;
  if (!(weight_scale > 0.0) || !std::isfinite(weight_scale))
    return fail(FREDOPT_E_ARG, "weight_scale must be positive and finite");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = bind_problem(p, pr, false, s)) != FREDOPT_OK) return st;
  set_problem(p, pr, q, weight_scale, x_inout);
  if ((st = upload_table(p, s)) != FREDOPT_OK) return st;
  fredopt_state zero{};
  zero.s = -1;
  if ((st = upload_state(p, &zero, s)) != FREDOPT_OK) return st;
  if ((st = enqueue_iteration(p, 0, s)) != FREDOPT_OK) return st;
  DevState d;
  if ((st = download_state(p, &d, s)) != FREDOPT_OK) return st;
  if (proximity_out) *proximity_out = d.proximity;
  if (d.nonfinite) return fail(FREDOPT_E_NONFINITE, "non-finite value during the sweep");
  return FREDOPT_OK;
}

static fredopt_status step_common(fredopt_plan* p, const fredopt_problem* pr,
                                  const fredopt_params* q, fredopt_state* stt, float* x,
                                  void* stream, int iters, bool use_graph) {
  if (!p || !x || !stt) return fail(FREDOPT_E_ARG, "plan, state and x must be non-NULL");
  fredopt_status st = check_problem_ptrs(pr, p->R);
  if (st != FREDOPT_OK) return st;
  if ((st = check_params(q, true)) != FREDOPT_OK) return st;
  if (stt->k < 0 || stt->s < -1) return fail(FREDOPT_E_STATE, "state needs k >= 0 and s >= -1");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int r = q->reductions_n;
  if ((st = bind_problem(p, pr, r > 0, s)) != FREDOPT_OK) return st;
  set_problem(p, pr, q, -1.0, x);
  if ((st = upload_table(p, s)) != FREDOPT_OK) return st;
  if ((st = upload_state(p, stt, s)) != FREDOPT_OK) return st;
  if (iters > 0) enqueue(p, Launch{FREDOPT_KERNEL_COL, kKindCol, kColYCopy}, s);
  if (use_graph && iters > 0) {
    if ((st = ensure_graph(p, r)) != FREDOPT_OK) return st;
    for (int i = 0; i < iters; ++i) HIPCHK(hipGraphLaunch(p->graph, s));
  } else {
    for (int i = 0; i < iters; ++i)
      if ((st = enqueue_iteration(p, r, s)) != FREDOPT_OK) return st;
  }
  DevState d;
  if ((st = download_state(p, &d, s)) != FREDOPT_OK) return st;
  if (iters > 0) export_state(d, stt);
  if (d.nonfinite) return fail(FREDOPT_E_NONFINITE, "non-finite value during an iteration");
  return FREDOPT_OK;
}

fredopt_status fredopt_superiorize_step(fredopt_plan* p, const fredopt_problem* pr,
                                        const fredopt_params* q, fredopt_state* st,
                                        float* x_inout, void* stream) {
  return step_common(p, pr, q, st, x_inout, stream, 1, false);
}

fredopt_status fredopt_solve(fredopt_plan* p, const fredopt_problem* pr, const fredopt_params* q,
                             fredopt_state* st, float* x_inout, void* stream) {
  if (!q) return fail(FREDOPT_E_ARG, "params is NULL");
  return step_common(p, pr, q, st, x_inout, stream, q->iter_max, true);
}

fredopt_status fredopt_profile_kernels(fredopt_plan* p, const fredopt_problem* pr,
                                       const fredopt_params* q, fredopt_state* stt,
                                       float* x, int32_t n_iters, void* stream, double* ms_out,
                                       int64_t* count_out) {
  if (!p || !x || !stt || !ms_out) return fail(FREDOPT_E_ARG, "NULL argument");
  if (n_iters < 1) return fail(FREDOPT_E_ARG, "n_iters must be >= 1");
  fredopt_status st = check_problem_ptrs(pr, p->R);
  if (st != FREDOPT_OK) return st;
  if ((st = check_params(q, false)) != FREDOPT_OK) return st;
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = bind_problem(p, pr, q->reductions_n > 0, s)) != FREDOPT_OK) return st;
  set_problem(p, pr, q, -1.0, x);
  if ((st = upload_table(p, s)) != FREDOPT_OK) return st;
  if ((st = upload_state(p, stt, s)) != FREDOPT_OK) return st;
  enqueue(p, Launch{FREDOPT_KERNEL_COL, kKindCol, kColYCopy}, s);
  const std::vector<Launch> seq =
      sequence_of(exec_of(p), q->reductions_n, p->sched_obj, q->objective != 0);
  const size_t n = seq.size() * (size_t)n_iters;
  std::vector<hipEvent_t> ev(2 * n, nullptr);
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  size_t t = 0;
  for (int it = 0; it < n_iters; ++it)
    for (const Launch& l : seq) {
      HIPCHK(hipEventRecord(ev[2 * t], s));
      enqueue(p, l, s);
      HIPCHK(hipEventRecord(ev[2 * t + 1], s));
      ++t;
    }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  double sum[FREDOPT_NUM_KERNELS] = {0};
  int64_t cnt[FREDOPT_NUM_KERNELS] = {0};
  t = 0;
  for (int it = 0; it < n_iters; ++it)
    for (const Launch& l : seq) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev[2 * t], ev[2 * t + 1]));
      sum[l.id] += ms;
      cnt[l.id] += 1;
      ++t;
    }
  for (auto& e : ev) (void)hipEventDestroy(e);
  for (int k = 0; k < FREDOPT_NUM_KERNELS; ++k) {
    ms_out[k] = cnt[k] ? sum[k] / (double)cnt[k] : 0.0;
    if (count_out) count_out[k] = cnt[k];
  }
  DevState d;
  if ((st = download_state(p, &d, s)) != FREDOPT_OK) return st;
  export_state(d, stt);
  if (d.nonfinite) return fail(FREDOPT_E_NONFINITE, "non-finite value during an iteration");
  return FREDOPT_OK;
}

fredopt_status fredopt_set_tuning(fredopt_plan* p, int32_t fwd_wgs_per_cu, int32_t tr_chunk,
                                  int32_t fwd_schedule) {
  if (!p) return fail(FREDOPT_E_ARG, "plan is NULL");
  if (fwd_schedule < 0 || fwd_schedule > 2)
    return fail(FREDOPT_E_ARG, "fwd_schedule must be 0, 1 or 2");
  if (fwd_wgs_per_cu < 0 || fwd_wgs_per_cu > 8)
    return fail(FREDOPT_E_ARG, "fwd_wgs_per_cu must lie in [0, 8]");
  if (tr_chunk != 0 && (tr_chunk < kTrChunkMin || tr_chunk % 256 != 0))
    return fail(FREDOPT_E_ARG, "tr_chunk must be a multiple of 256");
  DeviceGuard guard(p->device);
  if (fwd_wgs_per_cu) p->wgs_per_cu = std::min(fwd_wgs_per_cu, p->max_wgs_per_cu);
  if (fwd_schedule) p->fwd_dynamic = fwd_schedule == 1;
  if (tr_chunk) {
    p->tr_chunk = tr_chunk;
    build_tr_items(p);
    fredopt_status st = upload_tr(p, nullptr);
    if (st != FREDOPT_OK) return st;
  }
  drop_graph(p);
  HIPCHK(hipStreamSynchronize(nullptr));
  return FREDOPT_OK;
}

fredopt_status fredopt_set_scatter(fredopt_plan* p, int32_t n_workgroups,
                                   int64_t max_active_rows) {
  if (!p) return fail(FREDOPT_E_ARG, "plan is NULL");
  if (n_workgroups < -1 || n_workgroups > kScatterMaxWGs)
    return fail(FREDOPT_E_ARG, "n_workgroups must lie in [-1, %d]", (int)kScatterMaxWGs);
  if (max_active_rows < -1) return fail(FREDOPT_E_ARG, "max_active_rows must be >= -1");
  DeviceGuard guard(p->device);
  if (n_workgroups == -1)
    p->n_scatter = 0;
  else if (n_workgroups > 0)
    p->n_scatter = n_workgroups;
  else
    p->n_scatter = default_scatter_wgs(p);
  p->scatter_max_rows = max_active_rows >= 0 ? max_active_rows : p->R / 4;
  p->hp.n_scatter = p->n_scatter;
  p->hp.scatter_max_rows = (int32_t)std::min<int64_t>(p->scatter_max_rows, INT32_MAX);
  fredopt_status st = upload_scatter_items(p, nullptr);
  if (st == FREDOPT_OK) st = upload_table(p, nullptr);
  if (st != FREDOPT_OK) return st;
  drop_graph(p);
  HIPCHK(hipStreamSynchronize(nullptr));
  return FREDOPT_OK;
}

fredopt_status fredopt_autotune(fredopt_plan* p, const float* x, void* stream) {
  if (!p || !x) return fail(FREDOPT_E_ARG, "plan and x must be non-NULL");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto timeit = [&](const Launch& l, int reps) -> double {
    enqueue(p, l, s);  // warm
    (void)hipEventRecord(e0, s);
    for (int i = 0; i < reps; ++i) enqueue(p, l, s);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms / reps;
  };
  const DevPlan saved = p->hp;
  // forward: dose / LETd outputs into the plan's own d and l buffers
  p->hp.x = const_cast<float*>(x);
  p->hp.prm.c = 0.04;
  p->hp.out_dose = p->hp.d;
  p->hp.out_letd = p->hp.l;
  p->hp.out_cdl = nullptr;
  fredopt_status st = upload_table(p, s);
  int best_w = p->wgs_per_cu;
  double best = 1e30;
  for (int w = 1; st == FREDOPT_OK && w <= p->max_wgs_per_cu; ++w) {
    p->wgs_per_cu = w;
    const double t = timeit(Launch{0, kKindFwd, kFwdDoseLet, 0, kVecX}, 5);
    if (t < best) {
      best = t;
      best_w = w;
    }
  }
  p->wgs_per_cu = best_w;
  // transposed chunks (coefficients zero: the timing does not depend on them)
  HIPCHK(hipMemsetAsync(p->hp.coef, 0, sizeof(float2) * std::max<int64_t>(p->L.NP, 1), s));
  int best_chunk = p->tr_chunk;
  best = 1e30;
  for (int ch : {1024, 2048, 4096, 8192, 16384}) {
    if (st != FREDOPT_OK) break;
    p->tr_chunk = ch;
    build_tr_items(p);
    if ((st = upload_tr(p, s)) != FREDOPT_OK) break;
    const double t = timeit(Launch{0, kKindChunks, 1}, 5);
    if (t < best) {
      best = t;
      best_chunk = ch;
    }
  }
  p->tr_chunk = best_chunk;
  build_tr_items(p);
  p->hp = saved;
  if (st == FREDOPT_OK) st = upload_tr(p, s);
  if (st == FREDOPT_OK) st = upload_table(p, s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  drop_graph(p);
  HIPCHK(hipStreamSynchronize(s));
  return st;
}

}  // extern "C"

// ------------------------------------------------------------------- batches ----
//
// Several plans iterated by the same launches: one table of plan descriptors and
// the concatenation of the plans' work lists (each item names its plan).  Every
// plan keeps its own workspace, state and partial sums, and a plan's items are the
// ones it has alone, so its arithmetic (and result) does not depend on the batch
// (the active-row scatter of a plan may get fewer workgroups than alone: its exact
// integer sums do not depend on how the rows are shared out).
// Plans with and without the objective-row view follow different iteration
// schedules: they form two sub-batches whose launch sequences are captured one
// after the other into the same graph.

struct SubBatch {
  std::vector<int32_t> idx;   // caller's plan indices, in table order
  bool obj = false;
  Exec ex;
};

struct fredopt_batch {
  std::vector<fredopt_plan*> plans;        // caller's order
  std::vector<fredopt_problem> problems;   // copies; the arrays stay the caller's
  std::vector<int32_t> pos;                // table position of the caller's plan i
  std::vector<int32_t> nsc;                // active-row scatter workgroups of plan i
  std::vector<SubBatch> subs;
  int device = 0, storage = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  DevPlan* d_table = nullptr;
  std::vector<DevPlan> table;
  hipStream_t cap = nullptr;
  hipGraphExec_t graph = nullptr;
  int graph_r = -1;
};

namespace {

struct BatchLayout {
  size_t table, ctr, groups, ogroups, rows, tr, gtr, cblocks, sc, ss, total;
};

// Bounds from each plan's own layout, so the size is known before the problems
// are prepared.
BatchLayout batch_layout(fredopt_plan* const* plans, int32_t n) {
  int64_t g = 0, og = 0, rw = 0, t = 0, gt = 0, cb = 0, sc = 0, ss = 0;
  for (int32_t i = 0; i < n; ++i) {
    const Layout& L = plans[i]->L;
    sc += kScatterMaxWGs;
    ss += (plans[i]->C + 63) / 64;
    g += L.n_groups;
    og += L.max_obj_groups;
    rw += L.max_rows;
    t += L.max_tr;
    gt += L.max_tr;
    cb += L.n_col_blocks;
  }
  BatchLayout B{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at_ = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return at_;
  };
  B.table = take(sizeof(DevPlan) * (size_t)n);
  B.ctr = take(sizeof(uint32_t) * kCounters * 2);  // one set per sub-batch
  B.groups = take(sizeof(FwdGroup) * g);
  B.ogroups = take(sizeof(FwdGroup) * og);
  B.rows = take(sizeof(RowItem) * rw);
  B.tr = take(sizeof(TrItem) * t);
  B.gtr = take(sizeof(TrItem) * gt);
  B.cblocks = take(sizeof(ColBlock) * cb);
  B.sc = take(sizeof(ScItem) * sc);
  B.ss = take(sizeof(ScItem) * ss);
  B.total = o;
  return B;
}

void drop_batch_graph(fredopt_batch* b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  b->graph_r = -1;
}

template <typename T>
void append(std::vector<T>* dst, const std::vector<T>& src, int32_t plan) {
  for (T v : src) {
    v.plan = plan;
    dst->push_back(v);
  }
}

// Copies v to ws + *off (advancing *off) and returns the device address.
template <typename T>
const T* place(char* ws, size_t* off, const std::vector<T>& v, hipStream_t s, bool* ok) {
  const T* at_ = reinterpret_cast<const T*>(ws + *off);
  if (!v.empty() &&
      hipMemcpyAsync(ws + *off, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s) !=
          hipSuccess)
    *ok = false;
  *off += sizeof(T) * v.size();
  return at_;
}

}  // namespace

extern "C" {

size_t fredopt_batch_workspace_bytes(fredopt_plan* const* plans, int32_t n) {
  if (!plans || n < 1) return 0;
  for (int32_t i = 0; i < n; ++i)
    if (!plans[i]) return 0;
  return batch_layout(plans, n).total;
}

fredopt_status fredopt_batch_create(fredopt_plan* const* plans, int32_t n,
                                    const fredopt_problem* problems, void* workspace,
                                    size_t workspace_bytes, void* stream, fredopt_batch** out) {
  if (!plans || !problems || !workspace || !out || n < 1)
    return fail(FREDOPT_E_ARG, "plans, problems, workspace and out must be non-NULL, n >= 1");
  *out = nullptr;
  for (int32_t i = 0; i < n; ++i) {
    if (!plans[i]) return fail(FREDOPT_E_ARG, "plan %d is NULL", i);
    for (int32_t j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return fail(FREDOPT_E_ARG, "plan %d appears twice", i);
    if (plans[i]->storage != plans[0]->storage)
      return fail(FREDOPT_E_ARG, "all plans of a batch need the same value storage");
    if (plans[i]->device != plans[0]->device)
      return fail(FREDOPT_E_ARG, "all plans of a batch need the same device");
    fredopt_status st = check_problem_ptrs(&problems[i], plans[i]->R);
    if (st != FREDOPT_OK) return st;
  }
  const BatchLayout B = batch_layout(plans, n);
  if (workspace_bytes < B.total)
    return fail(FREDOPT_E_WORKSPACE, "batch workspace too small: %zu < %zu", workspace_bytes,
                B.total);
  DeviceGuard guard(plans[0]->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int32_t i = 0; i < n; ++i) {
    fredopt_status st = bind_problem(plans[i], &problems[i], true, s);
    if (st != FREDOPT_OK) return st;
  }
  fredopt_batch* b = new fredopt_batch;
  b->device = plans[0]->device;
  b->storage = plans[0]->storage;
  b->ws = static_cast<char*>(workspace);
  b->ws_bytes = workspace_bytes;
  b->d_table = reinterpret_cast<DevPlan*>(b->ws + B.table);
  b->pos.assign(n, 0);
  b->nsc.assign(n, 0);
  for (int32_t i = 0; i < n; ++i) {
    b->plans.push_back(plans[i]);
    b->problems.push_back(problems[i]);
  }
  // sub-batches by schedule: objective-row view first
  for (int obj = 1; obj >= 0; --obj) {
    SubBatch sb;
    sb.obj = obj == 1;
    for (int32_t i = 0; i < n; ++i)
      if (plans[i]->sched_obj == sb.obj) sb.idx.push_back(i);
    if (!sb.idx.empty()) b->subs.push_back(sb);
  }
  size_t off_g = B.groups, off_og = B.ogroups, off_r = B.rows, off_t = B.tr, off_gt = B.gtr,
         off_c = B.cblocks, off_sc = B.sc, off_ss = B.ss;
  int32_t base = 0;
  bool ok = true;
  for (size_t k = 0; k < b->subs.size(); ++k) {
    SubBatch& sb = b->subs[k];
    std::vector<FwdGroup> groups, ogroups;
    std::vector<RowItem> rows;
    std::vector<TrItem> tr, gtr;
    std::vector<ColBlock> cblocks;
    std::vector<ScItem> sc, ss;
    int lds = 0, wgs = 4, list_block = kWave;
    size_t sc_lds = 0;
    bool all_lds = true;
    for (size_t j = 0; j < sb.idx.size(); ++j) {
      fredopt_plan* p = plans[sb.idx[j]];
      b->pos[sb.idx[j]] = base + (int32_t)j;
      append(&groups, p->groups, (int32_t)j);
      if (sb.obj) append(&ogroups, p->ogroups, (int32_t)j);
      append(&rows, p->rows, (int32_t)j);
      append(&tr, p->tr, (int32_t)j);
      append(&gtr, p->gtr, (int32_t)j);
      append(&cblocks, p->cblocks, (int32_t)j);
      // the active-row path, one workgroup per 64k entries of the plan (measured on
      // 48 plans of 0.2-4M entries: one per 2M 82,800 plan-iterations/s, per 256k
      // 91,000, per 64k 95,800, per 16k 92,200); its integer sums do not depend on
      // how its rows are shared out
      const int nsc = p->n_scatter > 0
                          ? (int)std::min<int64_t>(p->n_scatter, 1 + p->nnz / (int64_t(1) << 16))
                          : 0;
      b->nsc[sb.idx[j]] = nsc;
      scatter_items((int32_t)j, nsc, p->C, &sc, &ss);
      if (nsc > 0 && !p->scatter_global) sc_lds = std::max(sc_lds, (size_t)p->C * sizeof(int64_t));
      lds = std::max(lds, p->lds_floats);
      all_lds = all_lds && p->lds_floats > 0;
      list_block = std::max(list_block, group_rows(p));
      wgs = std::min(wgs, p->wgs_per_cu);
    }
    Exec& e = sb.ex;
    e.storage = b->storage;
    e.n_cu = plans[0]->n_cu;
    e.wgs_per_cu = std::max(1, wgs);
    e.lds_floats = all_lds ? lds : 0;
    e.list_block = list_block;
    e.n_plans = (int)sb.idx.size();
    e.fwd_dynamic = true;
    e.table = b->d_table + base;
    e.groups = place(b->ws, &off_g, groups, s, &ok);
    e.n_groups = (int)groups.size();
    e.ogroups = place(b->ws, &off_og, ogroups, s, &ok);
    e.n_ogroups = (int)ogroups.size();
    e.rows = place(b->ws, &off_r, rows, s, &ok);
    e.n_rows = (int)rows.size();
    e.tr = place(b->ws, &off_t, tr, s, &ok);
    e.n_tr = (int)tr.size();
    e.gtr = place(b->ws, &off_gt, gtr, s, &ok);
    e.n_gtr = (int)gtr.size();
    e.cblocks = place(b->ws, &off_c, cblocks, s, &ok);
    e.n_cblocks = (int)cblocks.size();
    e.ctr = reinterpret_cast<uint32_t*>(b->ws + B.ctr) + kCounters * k;
    e.sc = place(b->ws, &off_sc, sc, s, &ok);
    e.n_sc = (int)sc.size();
    e.ss = place(b->ws, &off_ss, ss, s, &ok);
    e.n_ss = (int)ss.size();
    e.sc_lds = sc_lds;
    base += (int32_t)sb.idx.size();
  }
  fredopt_status st = FREDOPT_OK;
  if (!ok) st = fail(FREDOPT_E_DEVICE, "batch upload failed");
  if (st == FREDOPT_OK &&
      hipMemsetAsync(b->ws + B.ctr, 0, sizeof(uint32_t) * kCounters * 2, s) != hipSuccess)
    st = fail(FREDOPT_E_DEVICE, "counter reset failed");
  if (st == FREDOPT_OK && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
    st = fail(FREDOPT_E_DEVICE, "stream creation failed");
  if (st == FREDOPT_OK && hipStreamSynchronize(s) != hipSuccess)
    st = fail(FREDOPT_E_DEVICE, "batch upload failed");
  if (st != FREDOPT_OK) {
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return st;
  }
  *out = b;
  return FREDOPT_OK;
}

fredopt_status fredopt_batch_free(fredopt_batch* b) {
  if (!b) return fail(FREDOPT_E_ARG, "batch is NULL");
  {
    DeviceGuard guard(b->device);
    drop_batch_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
  }
  delete b;
  return FREDOPT_OK;
}

fredopt_status fredopt_batch_solve(fredopt_batch* b, const fredopt_params* q,
                                   fredopt_state* states, float* const* x, int32_t n_iters,
                                   void* stream) {
  if (!b || !states || !x) return fail(FREDOPT_E_ARG, "batch, states and x must be non-NULL");
  fredopt_status st = check_params(q, false);
  if (st != FREDOPT_OK) return st;
  if (n_iters < 0) return fail(FREDOPT_E_ARG, "n_iters must be >= 0");
  const int32_t n = (int32_t)b->plans.size();
  for (int32_t i = 0; i < n; ++i) {
    if (!x[i]) return fail(FREDOPT_E_ARG, "x[%d] is NULL", i);
    if (states[i].k < 0 || states[i].s < -1)
      return fail(FREDOPT_E_STATE, "state %d needs k >= 0 and s >= -1", i);
  }
  DeviceGuard guard(b->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  b->table.resize(n);
  for (int32_t i = 0; i < n; ++i) {
    fredopt_plan* p = b->plans[i];
    // the problem values may have changed since the last call (the kinds may not)
    if ((st = gather_problem(p, &b->problems[i], false, s)) != FREDOPT_OK) return st;
    if ((st = gather_problem(p, &b->problems[i], true, s)) != FREDOPT_OK) return st;
    set_problem(p, &b->problems[i], q, -1.0, x[i]);
    b->table[b->pos[i]] = p->hp;
    b->table[b->pos[i]].n_scatter = b->nsc[i];
    if ((st = upload_state(p, &states[i], s)) != FREDOPT_OK) return st;
  }
  HIPCHK(hipMemcpyAsync(b->d_table, b->table.data(), sizeof(DevPlan) * n, hipMemcpyHostToDevice,
                        s));
  if (n_iters > 0) {
    for (const SubBatch& sb : b->subs)
      enqueue(sb.ex, Launch{FREDOPT_KERNEL_COL, kKindCol, kColYCopy}, s);
    const int r = q->reductions_n;
    const int key = graph_key(r, q->objective);
    if (!(b->graph && b->graph_r == key)) {
      drop_batch_graph(b);
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
      for (const SubBatch& sb : b->subs)
        for (const Launch& l : sequence_of(sb.ex, r, sb.obj, q->objective != 0))
          enqueue(sb.ex, l, b->cap);
      const hipError_t le = hipGetLastError();
      const hipError_t ce = hipStreamEndCapture(b->cap, &g);
      if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(FREDOPT_E_DEVICE, "graph capture failed: %s",
                    hipGetErrorString(le != hipSuccess ? le : ce));
      }
      const hipError_t ie = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        b->graph = nullptr;
        return fail(FREDOPT_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(ie));
      }
      b->graph_r = key;
    }
    for (int32_t i = 0; i < n_iters; ++i) HIPCHK(hipGraphLaunch(b->graph, s));
  }
  HIPCHK(hipGetLastError());
  bool nonfinite = false;
  for (int32_t i = 0; i < n; ++i) {
    DevState d;
    if ((st = download_state(b->plans[i], &d, s)) != FREDOPT_OK) return st;
    if (n_iters > 0) export_state(d, &states[i]);
    nonfinite = nonfinite || d.nonfinite;
  }
  if (nonfinite) return fail(FREDOPT_E_NONFINITE, "non-finite value during an iteration");
  return FREDOPT_OK;
}

// ------------------------------------------------------ robustness evaluation ----

size_t fredopt_scenario_workspace_bytes(fredopt_plan* const* plans, int32_t n) {
  if (!plans || n < 1) return 0;
  size_t groups = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (!plans[i]) return 0;
    groups += plans[i]->groups.size();
  }
  return align_up(sizeof(uint32_t) * kCounters) + align_up(sizeof(DevPlan) * (size_t)n) +
         align_up(sizeof(FwdGroup) * std::max<size_t>(groups, 1));
}

fredopt_status fredopt_scenario_dose_let(fredopt_plan* const* plans, int32_t n, const float* x,
                                         double c, float* dose, float* letd, float* cdl,
                                         float* dose_min, float* dose_max, float* letd_min,
                                         float* letd_max, void* workspace,
                                         size_t workspace_bytes, void* stream) {
  if (!plans || n < 1 || !x) return fail(FREDOPT_E_ARG, "plans (n >= 1) and x must be non-NULL");
  if (!(c > 0.0) || !std::isfinite(c)) return fail(FREDOPT_E_ARG, "c must be positive and finite");
  if ((dose_min == nullptr) != (dose_max == nullptr) ||
      (letd_min == nullptr) != (letd_max == nullptr))
    return fail(FREDOPT_E_ARG, "band arrays come in pairs (min and max)");
  for (int32_t i = 0; i < n; ++i) {
    if (!plans[i]) return fail(FREDOPT_E_ARG, "plan %d is NULL", i);
    const fredopt_plan* p = plans[i];
    if (p->R != plans[0]->R || p->C != plans[0]->C)
      return fail(FREDOPT_E_SHAPE, "scenario %d is %lld x %lld, scenario 0 %lld x %lld: every "
                  "scenario must have the nominal plan's voxels and beamlets", i,
                  (long long)p->R, (long long)p->C, (long long)plans[0]->R,
                  (long long)plans[0]->C);
    if (p->storage != plans[0]->storage || p->device != plans[0]->device)
      return fail(FREDOPT_E_ARG, "scenario %d has another storage or device than scenario 0", i);
  }
  const size_t need = fredopt_scenario_workspace_bytes(plans, n);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0 ||
      workspace_bytes < need)
    return fail(FREDOPT_E_WORKSPACE, "workspace must be 256-byte aligned and hold %zu bytes",
                need);
  const fredopt_plan* p0 = plans[0];
  const int64_t R = p0->R;
  DeviceGuard guard(p0->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the scenarios' descriptors and the concatenation of their work lists
  std::vector<DevPlan> table((size_t)n);
  std::vector<FwdGroup> groups;
  int lds = p0->lds_floats;
  for (int32_t i = 0; i < n; ++i) {
    DevPlan h = plans[i]->hp;
    h.x = const_cast<float*>(x);
    h.prm.c = c;
    h.out_dose = dose ? dose + (int64_t)i * R : nullptr;
    h.out_letd = letd ? letd + (int64_t)i * R : nullptr;
    h.out_cdl = cdl ? cdl + (int64_t)i * R : nullptr;
    h.band[0] = reinterpret_cast<uint32_t*>(dose_min);
    h.band[1] = reinterpret_cast<uint32_t*>(dose_max);
    h.band[2] = reinterpret_cast<uint32_t*>(letd_min);
    h.band[3] = reinterpret_cast<uint32_t*>(letd_max);
    table[(size_t)i] = h;
    append(&groups, plans[i]->groups, i);
    lds = std::min(lds, plans[i]->lds_floats);
  }
  char* ws = static_cast<char*>(workspace);
  uint32_t* ctr = reinterpret_cast<uint32_t*>(ws);
  DevPlan* d_table = reinterpret_cast<DevPlan*>(ws + align_up(sizeof(uint32_t) * kCounters));
  FwdGroup* d_groups = reinterpret_cast<FwdGroup*>(reinterpret_cast<char*>(d_table) +
                                                   align_up(sizeof(DevPlan) * (size_t)n));
  HIPCHK(hipMemsetAsync(ctr, 0, sizeof(uint32_t) * kCounters, s));
  HIPCHK(hipMemcpyAsync(d_table, table.data(), sizeof(DevPlan) * table.size(),
                        hipMemcpyHostToDevice, s));
  if (!groups.empty())
    HIPCHK(hipMemcpyAsync(d_groups, groups.data(), sizeof(FwdGroup) * groups.size(),
                          hipMemcpyHostToDevice, s));
  launch_band(0, R, reinterpret_cast<uint32_t*>(dose_min), reinterpret_cast<uint32_t*>(dose_max),
              s);
  launch_band(0, R, reinterpret_cast<uint32_t*>(letd_min), reinterpret_cast<uint32_t*>(letd_max),
              s);
  Exec e;
  e.storage = p0->storage;
  e.n_cu = p0->n_cu;
  e.wgs_per_cu = p0->wgs_per_cu;
  e.lds_floats = lds;
  e.n_plans = n;
  e.fwd_dynamic = true;
  e.table = d_table;
  e.groups = d_groups;
  e.n_groups = (int)groups.size();
  e.ctr = ctr;
  if (e.n_groups > 0 && (dose || letd || cdl || dose_min || letd_min))
    enqueue(e, Launch{0, kKindFwd, kFwdDoseLet, 0, kVecX}, s);
  launch_band(1, R, reinterpret_cast<uint32_t*>(dose_min), reinterpret_cast<uint32_t*>(dose_max),
              s);
  launch_band(1, R, reinterpret_cast<uint32_t*>(letd_min), reinterpret_cast<uint32_t*>(letd_max),
              s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));  // the host tables above are read until here
  return FREDOPT_OK;
}

// ---------------------------------------------------------------- evaluation ----

fredopt_status fredopt_volume_histogram(const float* values, int64_t n_rows, const int32_t* rows,
                                        int64_t n, double vmax, int32_t n_bins, uint32_t* cum,
                                        void* stream) {
  if (!cum || (n > 0 && (!values || !rows)))
    return fail(FREDOPT_E_ARG, "values, rows and cum must be non-NULL");
  if (n_rows < 0 || n < 0) return fail(FREDOPT_E_SHAPE, "n_rows and n must be >= 0");
  if (!(vmax > 0.0) || !std::isfinite(vmax)) return fail(FREDOPT_E_ARG, "vmax must be positive");
  if (n_bins < 1 || n_bins > kMaxHistBins)
    return fail(FREDOPT_E_ARG, "n_bins must lie in [1, %d], got %d", kMaxHistBins, n_bins);
  int dev = 0, ncu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(set_histogram_lds_limit(sizeof(uint32_t) * (kMaxHistBins + 1)));
  launch_volume_histogram(values, n_rows, rows, n, vmax, n_bins, cum, ncu,
                          static_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return FREDOPT_OK;
}

fredopt_status fredopt_roi_quantiles(const float* values, int64_t n_rows, const int32_t* rows,
                                     int64_t n, const double* q, int32_t n_q, float* out,
                                     void* stream) {
  if (!q || !out || (n > 0 && (!values || !rows)))
    return fail(FREDOPT_E_ARG, "values, rows, q and out must be non-NULL");
  if (n_rows < 0 || n < 0) return fail(FREDOPT_E_SHAPE, "n_rows and n must be >= 0");
  if (n_q < 1 || n_q > kMaxQuantiles)
    return fail(FREDOPT_E_ARG, "n_q must lie in [1, %d], got %d", kMaxQuantiles, n_q);
  for (int32_t k = 0; k < n_q; ++k)
    if (!(q[k] > 0.0 && q[k] <= 1.0)) return fail(FREDOPT_E_ARG, "q[%d] must lie in (0, 1]", k);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) {  // an empty region: every quantile is 0
    HIPCHK(hipMemsetAsync(out, 0, sizeof(float) * (size_t)n_q, s));
    return FREDOPT_OK;
  }
  int64_t ranks[kMaxQuantiles];
  for (int32_t k = 0; k < n_q; ++k) {
    // nearest rank: ceil(q n), at least 1 (a guard of 1e-12 keeps q n = 95.0000000001
    // from rounding up a representation error)
    int64_t r = (int64_t)std::ceil(q[k] * (double)n - 1e-12);
    ranks[k] = std::min<int64_t>(std::max<int64_t>(r, 1), n);
  }
  launch_quantiles(values, n_rows, rows, n, ranks, n_q, out, s);
  HIPCHK(hipGetLastError());
  return FREDOPT_OK;
}

// ----------------------------------------------------- block-sequential sweep ----

fredopt_status fredopt_project_sweep_blocks(fredopt_plan* p, const fredopt_problem* pr,
                                            const fredopt_params* q, double weight_scale,
                                            int64_t block_rows, float* x_inout, void* stream) {
  if (!p || !x_inout) return fail(FREDOPT_E_ARG, "plan and x must be non-NULL");
  fredopt_status st = check_problem_ptrs(pr, p->R);
  if (st != FREDOPT_OK) return st;
  if ((st = check_params(q, false)) != FREDOPT_OK) return st;
  if (!(weight_scale > 0.0) || !std::isfinite(weight_scale))
    return fail(FREDOPT_E_ARG, "weight_scale must be positive and finite");
  if (block_rows < 1 || (block_rows < p->R && block_rows % kSortWindow != 0))
    return fail(FREDOPT_E_ARG, "block_rows must be a multiple of %lld rows (or cover every "
                "row), got %lld", (long long)kSortWindow, (long long)block_rows);
  if (p->n_scatter <= 0)
    return fail(FREDOPT_E_STATE, "block sweeps use the active-row projection, which is off "
                "for this plan (fredopt_set_scatter)");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = bind_problem(p, pr, false, s)) != FREDOPT_OK) return st;
  set_problem(p, pr, q, weight_scale, x_inout);
  if ((st = upload_table(p, s)) != FREDOPT_OK) return st;
  fredopt_state zero{};
  zero.s = -1;
  if ((st = upload_state(p, &zero, s)) != FREDOPT_OK) return st;
  const Layout& L = p->L;
  const int64_t R = p->R;
  const int64_t rows_b = std::min<int64_t>(block_rows, std::max<int64_t>(R, 1));
  // blocks of whole sort windows: their rows own a contiguous range of slices
  const int rpw = kWave >> p->sell.lpr_log2;
  std::vector<FwdGroup> bg;
  if (p->blk_rows != rows_b) {
    p->blk_g0.clear();
    p->blk_ng.clear();
    int64_t slice = 0;
    for (int64_t r0 = 0; r0 < R; r0 += rows_b) {
      const int64_t r1 = std::min(R, r0 + rows_b);
      int64_t n_sl = 0;  // slices of the windows [r0, r1): each window's own count
      for (int64_t w0 = r0; w0 < r1; w0 += kSortWindow)
        n_sl += (std::min(r1, w0 + kSortWindow) - w0 + rpw - 1) / rpw;
      p->blk_g0.push_back((int32_t)bg.size());
      int32_t slot = 0;
      for (int64_t s0 = slice; s0 < slice + n_sl; s0 += kFwdWaves)
        bg.push_back(FwdGroup{0, (int32_t)s0, (int32_t)std::min<int64_t>(kFwdWaves, slice + n_sl - s0),
                              slot++});
      p->blk_ng.push_back(slot);
      slice += n_sl;
    }
    if (slice != p->sell.n_slices || (int64_t)p->blk_g0.size() > L.max_blocks ||
        (int64_t)bg.size() > L.n_groups + L.max_blocks)
      return fail(FREDOPT_E_STATE, "block layout does not match the plan's slices");
    HIPCHK(hipMemcpyAsync(p->ws + L.bgroups, bg.data(), sizeof(FwdGroup) * bg.size(),
                          hipMemcpyHostToDevice, s));
    p->blk_rows = rows_b;
  }
  const int nb = (int)p->blk_g0.size();
  // one descriptor per block: the plan's, with the block's group count (its partial
  // slots) and the active-row projection for every active count
  std::vector<DevPlan> tb((size_t)std::max(nb, 1), p->hp);
  for (int b = 0; b < nb; ++b) {
    tb[b].sell.n_groups = p->blk_ng[b];
    tb[b].scatter_max_rows = INT32_MAX;
  }
  DevPlan* d_tb = at<DevPlan>(p, L.btable);
  HIPCHK(hipMemcpyAsync(d_tb, tb.data(), sizeof(DevPlan) * (size_t)nb, hipMemcpyHostToDevice, s));
  const FwdGroup* d_bg = at<FwdGroup>(p, L.bgroups);
  for (int b = 0; b < nb; ++b) {
    if (p->blk_ng[b] == 0) continue;
    Exec e = exec_of(p);
    e.table = d_tb + b;
    e.groups = d_bg + p->blk_g0[b];
    e.n_groups = p->blk_ng[b];
    enqueue(e, Launch{FREDOPT_KERNEL_FWD_RESID, kKindFwd, kFwdResid, 0, kVecX}, s);
    enqueue(e, Launch{FREDOPT_KERNEL_FINALIZE, kKindFin, kFinResidFwd}, s);
    enqueue(e, Launch{FREDOPT_KERNEL_ACTIVE_LIST, kKindList, 0}, s);
    enqueue(e, Launch{FREDOPT_KERNEL_SCATTER, kKindScatter, 0}, s);
    enqueue(e, Launch{FREDOPT_KERNEL_SCATTER_SUM, kKindScatterSum, kColProjNoClamp}, s);
  }
  enqueue(p, Launch{FREDOPT_KERNEL_COL, kKindCol, kColClamp}, s);
  HIPCHK(hipGetLastError());
  DevState d;
  if ((st = download_state(p, &d, s)) != FREDOPT_OK) return st;  // synchronises
  if (d.nonfinite) return fail(FREDOPT_E_NONFINITE, "non-finite value during the sweep");
  return FREDOPT_OK;
}

}  // extern "C"
