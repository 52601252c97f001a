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
constexpr int64_t kFwdItemMinSlots = 1024;
constexpr int64_t kFwdItemMaxSlots = 65536;
constexpr int64_t kFwdItemMaxRows = 4096;
constexpr int64_t kRowItemRows = 2048;
constexpr int64_t kTrChunkMin = 1024;
constexpr int64_t kTrChunkDefault = 4096;
constexpr int64_t kBlockCountCap = int64_t(1) << 24;

inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int value_bytes(int storage) { return storage == FREDOPT_F32 ? 4 : 2; }

struct Layout {
  size_t table, state, cnt, rp, cp, ci, dv, lv, ri, cdv, clv, cscale, mom;
  size_t d, l, dg, lg, coef, g, colval, fpart, rpart, tpart;
  size_t fwd_items, row_items, tr_items, bc, colcount, colmax, flags, total;
  int64_t csr_slots, csc_slots, max_fwd, max_rows, max_tr;
  int64_t rows_per_block, nb;
};

// Upper-bound layout for every pattern with these sizes (row / column padding to a
// multiple of 4 slots adds at most 3 slots per row / column).
bool make_layout(int64_t R, int64_t C, int64_t nnz, int storage, Layout* L) {
  if (R < 0 || C < 1 || nnz < 0 || R >= (int64_t(1) << 31) || C >= (int64_t(1) << 31))
    return false;
  if (storage < FREDOPT_F32 || storage > FREDOPT_BF16) return false;
  const int64_t csr = nnz + 3 * R, csc = nnz + 3 * C;
  if (csc >= (int64_t(1) << 32) - 4) return false;
  const int vb = value_bytes(storage);
  L->csr_slots = csr;
  L->csc_slots = csc;
  L->max_fwd = csr / kFwdItemMinSlots + R / kFwdItemMaxRows + 2;
  L->max_rows = R / kRowItemRows + 2;
  L->max_tr = C + csc / kTrChunkMin + 2;
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
  L->table = take(sizeof(DevPlan));
  L->state = take(sizeof(DevState));
  L->cnt = take(sizeof(uint32_t) * (kPlanTickets + C));
  L->rp = take(sizeof(int64_t) * (R + 1));
  L->cp = take(sizeof(int64_t) * (C + 1));
  L->ci = take(sizeof(int32_t) * csr);
  L->dv = take((size_t)vb * csr);
  L->lv = take((size_t)vb * csr);
  L->ri = take(sizeof(int32_t) * csc);
  L->cdv = take((size_t)vb * csc);
  L->clv = take((size_t)vb * csc);
  L->cscale = take(sizeof(float) * C);
  L->mom = take(sizeof(double) * 3 * (R > 0 ? R : 1));
  L->d = take(sizeof(float) * R);
  L->l = take(sizeof(float) * R);
  L->dg = take(sizeof(float) * R);
  L->lg = take(sizeof(float) * R);
  L->coef = take(sizeof(float2) * R);
  L->g = take(sizeof(float) * C);
  L->colval = take(sizeof(double) * C);
  L->fpart = take(sizeof(double) * kNPart * L->max_fwd);
  L->rpart = take(sizeof(double) * kNPart * L->max_rows);
  L->tpart = take(sizeof(float) * L->max_tr);
  L->fwd_items = take(sizeof(FwdItem) * L->max_fwd);
  L->row_items = take(sizeof(RowItem) * L->max_rows);
  L->tr_items = take(sizeof(TrItem) * L->max_tr);
  L->bc = take(sizeof(uint32_t) * L->nb * C);
  L->colcount = take(sizeof(uint32_t) * C);
  L->colmax = take(sizeof(uint32_t) * C);
  L->flags = take(sizeof(uint32_t) * 4);
  L->total = o;
  return true;
}

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
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
  Layout L{};
  std::vector<int64_t> rp, cp;
  int lanes = 64, tr_chunk = (int)kTrChunkDefault, fwd_grid = 0, lds_floats = 0;
  int n_cu = 256, grid_mult = 3;
  size_t lds_cap = 65536;
  std::vector<FwdItem> fwd;
  std::vector<RowItem> rows;
  std::vector<TrItem> tr;
  DevPlan hp{};
  DevPlan* d_table = nullptr;
  DevState* d_state = nullptr;
  FwdItem* d_fwd = nullptr;
  RowItem* d_rows = nullptr;
  TrItem* d_tr = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t graph = nullptr;
  int graph_r = -1;
};

namespace {

template <typename T>
T* at(fredopt_plan* p, size_t off) {
  return reinterpret_cast<T*>(p->ws + off);
}

void build_fwd_items(fredopt_plan* p) {
  p->fwd.clear();
  const int64_t slots = p->rp[p->R];
  int64_t target = slots / (8 * (int64_t)std::max(1, p->fwd_grid));
  target = std::min(std::max(target, kFwdItemMinSlots), kFwdItemMaxSlots);
  int64_t r0 = 0;
  while (r0 < p->R) {
    int64_t r1 = r0;
    while (r1 < p->R && r1 - r0 < kFwdItemMaxRows && p->rp[r1] - p->rp[r0] < target) ++r1;
    p->fwd.push_back(FwdItem{0, (int32_t)p->fwd.size(), (int32_t)r0, (int32_t)r1});
    r0 = r1;
  }
  if (p->fwd.empty()) p->fwd.push_back(FwdItem{0, 0, 0, 0});
}

void build_row_items(fredopt_plan* p) {
  p->rows.clear();
  for (int64_t r0 = 0; r0 < p->R; r0 += kRowItemRows)
    p->rows.push_back(RowItem{0, (int32_t)p->rows.size(), (int32_t)r0,
                              (int32_t)std::min(p->R, r0 + kRowItemRows)});
  if (p->rows.empty()) p->rows.push_back(RowItem{0, 0, 0, 0});
}

// Columns split into chunks of about tr_chunk slots (boundaries on 4-slot quads),
// then ordered longest first so the hardware dispatcher balances the grid.
void build_tr_items(fredopt_plan* p) {
  p->tr.clear();
  int32_t tslot = 0;
  const int64_t ch = p->tr_chunk;
  for (int64_t j = 0; j < p->C; ++j) {
    const int64_t a = p->cp[j], b = p->cp[j + 1];
    const int64_t quads = (b - a) / 4;
    const int64_t n = std::max<int64_t>(1, (b - a + ch - 1) / ch);
    for (int64_t c = 0; c < n; ++c) {
      TrItem t{};
      t.plan = 0;
      t.col = (int32_t)j;
      t.chunk = (int32_t)c;
      t.nchunks = (int32_t)n;
      t.q0 = a + 4 * (c * quads / n);
      t.q1 = a + 4 * ((c + 1) * quads / n);
      t.tslot0 = tslot;
      p->tr.push_back(t);
    }
    tslot += (int32_t)n;
  }
  std::stable_sort(p->tr.begin(), p->tr.end(), [](const TrItem& x, const TrItem& y) {
    return (x.q1 - x.q0) > (y.q1 - y.q0);
  });
}

int pick_lanes(const fredopt_plan* p) {
  if (p->R == 0) return 64;
  const double aq = (double)p->rp[p->R] / 4.0 / (double)p->R;
  int g = 4;
  while (g < 64 && g < aq / 2.0) g *= 2;
  return g;
}

fredopt_status upload_items(fredopt_plan* p, hipStream_t s) {
  if ((int64_t)p->fwd.size() > p->L.max_fwd || (int64_t)p->rows.size() > p->L.max_rows ||
      (int64_t)p->tr.size() > p->L.max_tr)
    return fail(FREDOPT_E_WORKSPACE, "work lists exceed the workspace bound");
  HIPCHK(hipMemcpyAsync(p->d_fwd, p->fwd.data(), sizeof(FwdItem) * p->fwd.size(),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->d_rows, p->rows.data(), sizeof(RowItem) * p->rows.size(),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->d_tr, p->tr.data(), sizeof(TrItem) * p->tr.size(),
                        hipMemcpyHostToDevice, s));
  p->hp.lanes = p->lanes;
  p->hp.n_fwd_items = (int32_t)p->fwd.size();
  p->hp.n_row_items = (int32_t)p->rows.size();
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
  if (q->reserved != 0) return fail(FREDOPT_E_ARG, "reserved field must be 0");
  return FREDOPT_OK;
}

fredopt_status check_problem_ptrs(const fredopt_problem* pr) {
  if (!pr) return fail(FREDOPT_E_ARG, "problem is NULL");
  if (!pr->kind || !pr->dose_lo || !pr->dose_hi || !pr->cdl_lo || !pr->cdl_hi || !pr->letd_max ||
      !pr->w_feas || !pr->w_obj || !pr->dose_target || !pr->cdl_target)
    return fail(FREDOPT_E_ARG, "a problem array is NULL");
  if (!(pr->c > 0.0) || !std::isfinite(pr->c))
    return fail(FREDOPT_E_ARG, "c must be positive and finite, got %g", pr->c);
  return FREDOPT_OK;
}

void set_problem(fredopt_plan* p, const fredopt_problem* pr, const fredopt_params* q,
                 double ws_fixed, float* x) {
  DevPlan& h = p->hp;
  h.kind = pr->kind;
  h.dlo = pr->dose_lo;
  h.dhi = pr->dose_hi;
  h.clo = pr->cdl_lo;
  h.chi = pr->cdl_hi;
  h.tmax = pr->letd_max;
  h.wf = pr->w_feas;
  h.wo = pr->w_obj;
  h.dt = pr->dose_target;
  h.ct = pr->cdl_target;
  h.prm.lambda = q->lambda;
  h.prm.alpha = q->alpha;
  h.prm.eta = q->eta;
  h.prm.c = pr->c;
  h.prm.ws_fixed = ws_fixed;
  h.prm.normalization = q->normalization;
  h.prm.reductions_n = q->reductions_n;
  h.x = x;
  h.out_dose = h.out_letd = h.out_cdl = nullptr;
}

fredopt_status upload_table(fredopt_plan* p, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(p->d_table, &p->hp, sizeof(DevPlan), hipMemcpyHostToDevice, s));
  return FREDOPT_OK;
}

fredopt_status run_problem_check(fredopt_plan* p, const fredopt_problem* pr, hipStream_t s) {
  uint32_t* flags = at<uint32_t>(p, p->L.flags);
  HIPCHK(hipMemsetAsync(flags, 0, sizeof(uint32_t), s));
  launch_check_problem(p->R, pr->kind, pr->dose_lo, pr->dose_hi, pr->cdl_lo, pr->cdl_hi,
                       pr->letd_max, pr->w_feas, pr->w_obj, pr->dose_target, pr->cdl_target,
                       flags, s);
  HIPCHK(hipGetLastError());
  uint32_t f = 0;
  HIPCHK(hipMemcpyAsync(&f, flags, sizeof f, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (f & 8u) return fail(FREDOPT_E_ARG, "problem: unknown kind bits");
  if (f & 1u) return fail(FREDOPT_E_NONFINITE, "problem: non-finite bound, target or weight");
  if (f & 2u) return fail(FREDOPT_E_ARG, "problem: lower bound above upper bound");
  if (f & 4u) return fail(FREDOPT_E_ARG, "problem: AMS weight <= 0 or objective weight < 0");
  return FREDOPT_OK;
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
}

struct Launch {
  int id;       // FREDOPT_KERNEL_*
  int kind;     // 0 forward, 1 rows, 2 transposed
  int mode;
};

std::vector<Launch> iteration_sequence(int r) {
  std::vector<Launch> seq;
  if (r == 0) {
    seq.push_back({FREDOPT_KERNEL_FWD_RESID, 0, kFwdResid});
    seq.push_back({FREDOPT_KERNEL_TR_PROJ, 2, kTrProj});
    return seq;
  }
  seq.push_back({FREDOPT_KERNEL_FWD_OBJ, 0, kFwdObj});
  for (int t = 0; t < r; ++t) {
    seq.push_back({FREDOPT_KERNEL_TR_GRAD, 2, t == 0 ? kTrGrad : kTrGradMove});
    seq.push_back({FREDOPT_KERNEL_FWD_DIR, 0, kFwdDir});
    seq.push_back({FREDOPT_KERNEL_ROWS, 1, t + 1 < r ? kRowsMoveObj : kRowsMoveResid});
  }
  seq.push_back({FREDOPT_KERNEL_TR_PROJ, 2, kTrProjMove});
  return seq;
}

void enqueue(fredopt_plan* p, const Launch& l, hipStream_t s) {
  if (l.kind == 0) {
    const int grid = std::min<int>((int)p->fwd.size(), p->fwd_grid);
    launch_forward(p->storage, l.mode, p->d_table, p->d_fwd, (int)p->fwd.size(), grid,
                   p->lds_floats, s);
  } else if (l.kind == 1) {
    launch_rows(l.mode, p->d_table, p->d_rows, (int)p->rows.size(), s);
  } else {
    launch_transposed(p->storage, l.mode, p->d_table, p->d_tr, (int)p->tr.size(), s);
  }
}

fredopt_status enqueue_iteration(fredopt_plan* p, int r, hipStream_t s) {
  for (const Launch& l : iteration_sequence(r)) enqueue(p, l, s);
  HIPCHK(hipGetLastError());
  return FREDOPT_OK;
}

fredopt_status ensure_graph(fredopt_plan* p, int r) {
  if (p->graph && p->graph_r == r) return FREDOPT_OK;
  drop_graph(p);
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
  for (const Launch& l : iteration_sequence(r)) enqueue(p, l, p->cap);
  const hipError_t le = hipGetLastError();
  const hipError_t ce = hipStreamEndCapture(p->cap, &g);
  if (le != hipSuccess || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(FREDOPT_E_DEVICE, "graph capture failed: %s",
                hipGetErrorString(le != hipSuccess ? le : ce));
  }
  const hipError_t ie = hipGraphInstantiate(&p->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    p->graph = nullptr;
    return fail(FREDOPT_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(ie));
  }
  p->graph_r = r;
  return FREDOPT_OK;
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
  p->lds_cap = (size_t)std::max(smem_block, 0);
  const size_t static_lds = 4096 + 64;  // reduction scratch of k_forward
  const size_t need = (size_t)p->C * sizeof(float);
  if (need + static_lds <= p->lds_cap) {
    p->lds_floats = (int)p->C;
    if (need > 0) HIPCHK(set_forward_lds_limit(p->storage, need));
    const size_t per_wg = need + static_lds;
    const int fit = (int)std::max<size_t>(1, (size_t)std::max(smem_sm, 1) / per_wg);
    p->grid_mult = std::min(4, std::max(1, fit));
  } else {
    p->lds_floats = 0;
    p->grid_mult = 4;
  }
  p->fwd_grid = p->n_cu * p->grid_mult;
  return FREDOPT_OK;
}

}  // namespace

// =============================================================================== ABI

extern "C" {

const char* fredopt_last_error(void) { return g_err.c_str(); }

size_t fredopt_workspace_bytes(int64_t n_rows, int64_t n_cols, int64_t nnz, int32_t storage) {
  Layout L;
  if (!make_layout(n_rows, n_cols, nnz, storage, &L)) return 0;
  return L.total;
}

fredopt_status fredopt_load_matrices(const fredopt_matrices* m, void* workspace,
                                     size_t workspace_bytes, void* stream, fredopt_plan** out) {
  if (!m || !out) return fail(FREDOPT_E_ARG, "matrices and out must be non-NULL");
  *out = nullptr;
  const int64_t R = m->n_rows, C = m->n_cols, nnz = m->nnz;
  Layout L;
  if (!make_layout(R, C, nnz, m->storage, &L))
    return fail(FREDOPT_E_SHAPE, "invalid sizes or storage (rows %lld cols %lld nnz %lld)",
                (long long)R, (long long)C, (long long)nnz);
  if (!m->row_ptr || (nnz > 0 && (!m->col_idx || !m->d_val || !m->l_val)))
    return fail(FREDOPT_E_ARG, "matrix array is NULL");
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
    return fail(FREDOPT_E_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
  if (workspace_bytes < L.total)
    return fail(FREDOPT_E_WORKSPACE, "workspace too small: %zu < %zu", workspace_bytes, L.total);
  hipStream_t s = static_cast<hipStream_t>(stream);

  // host copy of the row pointers: validation, padding, work lists
  std::vector<int64_t> h_rp(R + 1);
  if (m->on_device) {
    HIPCHK(hipMemcpyAsync(h_rp.data(), m->row_ptr, sizeof(int64_t) * (R + 1),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  } else {
    std::memcpy(h_rp.data(), m->row_ptr, sizeof(int64_t) * (R + 1));
  }
  if (h_rp[0] != 0 || h_rp[R] != nnz) return fail(FREDOPT_E_SHAPE, "row_ptr[0] != 0 or row_ptr[n] != nnz");
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
  p->L = L;
  fredopt_status st = device_limits(p);
  if (st != FREDOPT_OK) {
    delete p;
    return st;
  }
  DeviceGuard guard(p->device);

  // device view of the input CSR (staged for host input)
  void* staging = nullptr;
  const int64_t* in_rp = m->row_ptr;
  const int32_t* in_col = m->col_idx;
  const float* in_dv = m->d_val;
  const float* in_lv = m->l_val;
  auto cleanup = [&](fredopt_status code) {
    if (staging) (void)hipFree(staging);
    if (code != FREDOPT_OK) {
      if (p->cap) (void)hipStreamDestroy(p->cap);
      delete p;
    }
    return code;
  };
#define LCHK(expr)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return cleanup(fail(FREDOPT_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_))); \
  } while (0)
  if (!m->on_device) {
    const size_t bytes = align_up(sizeof(int64_t) * (R + 1)) + align_up(sizeof(int32_t) * nnz) +
                         2 * align_up(sizeof(float) * nnz);
    LCHK(hipMalloc(&staging, bytes));
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

  LCHK(hipMemsetAsync(ws + L.flags, 0, sizeof(uint32_t) * 4, s));
  LCHK(hipMemsetAsync(ws + L.cnt, 0, sizeof(uint32_t) * (kPlanTickets + C), s));
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

  // padded row / column pointers
  p->rp.assign(R + 1, 0);
  for (int64_t i = 0; i < R; ++i) p->rp[i + 1] = p->rp[i] + ((h_rp[i + 1] - h_rp[i] + 3) & ~int64_t(3));
  p->cp.assign(C + 1, 0);
  for (int64_t j = 0; j < C; ++j) p->cp[j + 1] = p->cp[j] + (((int64_t)h_cc[j] + 3) & ~int64_t(3));
  if (p->rp[R] > L.csr_slots || p->cp[C] > L.csc_slots)
    return cleanup(fail(FREDOPT_E_WORKSPACE, "padded matrix exceeds the workspace bound"));

  int64_t* d_rp = reinterpret_cast<int64_t*>(ws + L.rp);
  int64_t* d_cp = reinterpret_cast<int64_t*>(ws + L.cp);
  LCHK(hipMemcpyAsync(d_rp, p->rp.data(), sizeof(int64_t) * (R + 1), hipMemcpyHostToDevice, s));
  LCHK(hipMemcpyAsync(d_cp, p->cp.data(), sizeof(int64_t) * (C + 1), hipMemcpyHostToDevice, s));

  const int vb = value_bytes(m->storage);
  const float* scale = q16 ? cscale : nullptr;
  int32_t* ci = reinterpret_cast<int32_t*>(ws + L.ci);
  int32_t* ri = reinterpret_cast<int32_t*>(ws + L.ri);
  launch_pack_csr(m->storage, R, in_rp, in_col, in_dv, in_lv, scale, d_rp, ci, ws + L.dv,
                  ws + L.lv, s);
  // CSC: zero (padding slots keep row 0, value 0), per-block counts, offsets, fill
  LCHK(hipMemsetAsync(ri, 0, sizeof(int32_t) * p->cp[C], s));
  LCHK(hipMemsetAsync(ws + L.cdv, 0, (size_t)vb * p->cp[C], s));
  LCHK(hipMemsetAsync(ws + L.clv, 0, (size_t)vb * p->cp[C], s));
  uint32_t* bc = reinterpret_cast<uint32_t*>(ws + L.bc);
  LCHK(hipMemsetAsync(bc, 0, sizeof(uint32_t) * L.nb * C, s));
  launch_block_count(R, C, (int)L.rows_per_block, in_rp, in_col, bc, s);
  launch_block_offsets(C, (int)L.nb, d_cp, bc, s);
  launch_fill_csc(m->storage, R, C, (int)L.rows_per_block, in_rp, in_col, in_dv, in_lv, scale, bc,
                  ri, ws + L.cdv, ws + L.clv, s);
  launch_moments(m->storage, R, d_rp, ws + L.dv, ws + L.lv, ci, scale,
                 reinterpret_cast<double*>(ws + L.mom), s);
  LCHK(hipGetLastError());

  // plan descriptor
  p->d_table = reinterpret_cast<DevPlan*>(ws + L.table);
  p->d_state = reinterpret_cast<DevState*>(ws + L.state);
  p->d_fwd = reinterpret_cast<FwdItem*>(ws + L.fwd_items);
  p->d_rows = reinterpret_cast<RowItem*>(ws + L.row_items);
  p->d_tr = reinterpret_cast<TrItem*>(ws + L.tr_items);
  DevPlan& h = p->hp;
  std::memset(&h, 0, sizeof h);
  h.R = R;
  h.C = C;
  h.vtype = m->storage;
  h.rp = d_rp;
  h.ci = ci;
  h.dv = ws + L.dv;
  h.lv = ws + L.lv;
  h.cp = d_cp;
  h.ri = ri;
  h.cdv = ws + L.cdv;
  h.clv = ws + L.clv;
  h.cscale = scale;
  h.mom = reinterpret_cast<const double*>(ws + L.mom);
  h.d = reinterpret_cast<float*>(ws + L.d);
  h.l = reinterpret_cast<float*>(ws + L.l);
  h.dg = reinterpret_cast<float*>(ws + L.dg);
  h.lg = reinterpret_cast<float*>(ws + L.lg);
  h.coef = reinterpret_cast<float2*>(ws + L.coef);
  h.g = reinterpret_cast<float*>(ws + L.g);
  h.fpart = reinterpret_cast<double*>(ws + L.fpart);
  h.rpart = reinterpret_cast<double*>(ws + L.rpart);
  h.tpart = reinterpret_cast<float*>(ws + L.tpart);
  h.colval = reinterpret_cast<double*>(ws + L.colval);
  h.cnt = reinterpret_cast<uint32_t*>(ws + L.cnt);
  h.st = p->d_state;
  h.prm.ws_fixed = -1.0;
  p->lanes = pick_lanes(p);
  build_fwd_items(p);
  build_row_items(p);
  build_tr_items(p);
  st = upload_items(p, s);
  if (st != FREDOPT_OK) return cleanup(st);
  LCHK(hipMemsetAsync(h.g, 0, sizeof(float) * C, s));
  LCHK(hipMemsetAsync(h.coef, 0, sizeof(float2) * (R > 0 ? R : 1), s));
  st = upload_table(p, s);
  if (st != FREDOPT_OK) return cleanup(st);
  LCHK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
  LCHK(hipStreamSynchronize(s));
#undef LCHK
  *out = p;
  return cleanup(FREDOPT_OK);
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
  info->csr_slots = p->rp.empty() ? 0 : p->rp[p->R];
  info->csc_slots = p->cp.empty() ? 0 : p->cp[p->C];
  info->bytes_per_csr_slot = 4 + 2 * value_bytes(p->storage);
  info->bytes_per_csc_slot = 4 + 2 * value_bytes(p->storage);
  info->fwd_items = (int64_t)p->fwd.size();
  info->tr_items = (int64_t)p->tr.size();
  info->row_items = (int64_t)p->rows.size();
  info->storage = p->storage;
  info->lanes_per_row = p->lanes;
  info->fwd_grid = std::min<int>((int)p->fwd.size(), p->fwd_grid);
  info->tr_chunk = p->tr_chunk;
  info->lds_x = p->lds_floats > 0 ? 1 : 0;
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
  if (dose || letd || cdl) enqueue(p, Launch{0, 0, kFwdDoseLet}, s);
  HIPCHK(hipGetLastError());
  return FREDOPT_OK;
}

fredopt_status fredopt_project_sweep(fredopt_plan* p, const fredopt_problem* pr,
                                     const fredopt_params* q, double weight_scale,
                                     float* x_inout, double* proximity_out, void* stream) {
  if (!p || !x_inout) return fail(FREDOPT_E_ARG, "plan and x must be non-NULL");
  fredopt_status st = check_problem_ptrs(pr);
  if (st != FREDOPT_OK) return st;
  if ((st = check_params(q, false)) != FREDOPT_OK) return st;
  if (!(weight_scale > 0.0) || !std::isfinite(weight_scale))
    return fail(FREDOPT_E_ARG, "weight_scale must be positive and finite");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = run_problem_check(p, pr, s)) != FREDOPT_OK) return st;
  set_problem(p, pr, q, weight_scale, x_inout);
  if ((st = upload_table(p, s)) != FREDOPT_OK) return st;
  fredopt_state zero{};
  zero.s = -1;
  if ((st = upload_state(p, &zero, s)) != FREDOPT_OK) return st;
  enqueue(p, Launch{FREDOPT_KERNEL_FWD_RESID, 0, kFwdResid}, s);
  enqueue(p, Launch{FREDOPT_KERNEL_TR_PROJ, 2, kTrProj}, s);
  HIPCHK(hipGetLastError());
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
  fredopt_status st = check_problem_ptrs(pr);
  if (st != FREDOPT_OK) return st;
  if ((st = check_params(q, true)) != FREDOPT_OK) return st;
  if (stt->k < 0 || stt->s < -1) return fail(FREDOPT_E_STATE, "state needs k >= 0 and s >= -1");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = run_problem_check(p, pr, s)) != FREDOPT_OK) return st;
  set_problem(p, pr, q, -1.0, x);
  if ((st = upload_table(p, s)) != FREDOPT_OK) return st;
  if ((st = upload_state(p, stt, s)) != FREDOPT_OK) return st;
  const int r = q->reductions_n;
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
  fredopt_status st = check_problem_ptrs(pr);
  if (st != FREDOPT_OK) return st;
  if ((st = check_params(q, false)) != FREDOPT_OK) return st;
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = run_problem_check(p, pr, s)) != FREDOPT_OK) return st;
  set_problem(p, pr, q, -1.0, x);
  if ((st = upload_table(p, s)) != FREDOPT_OK) return st;
  if ((st = upload_state(p, stt, s)) != FREDOPT_OK) return st;
  const std::vector<Launch> seq = iteration_sequence(q->reductions_n);
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

fredopt_status fredopt_set_tuning(fredopt_plan* p, int32_t lanes_per_row, int32_t tr_chunk) {
  if (!p) return fail(FREDOPT_E_ARG, "plan is NULL");
  if (lanes_per_row != 0 && lanes_per_row != 4 && lanes_per_row != 8 && lanes_per_row != 16 &&
      lanes_per_row != 32 && lanes_per_row != 64)
    return fail(FREDOPT_E_ARG, "lanes_per_row must be 4, 8, 16, 32 or 64");
  if (tr_chunk != 0 && (tr_chunk < kTrChunkMin || tr_chunk % 1024 != 0))
    return fail(FREDOPT_E_ARG, "tr_chunk must be a multiple of 1024");
  DeviceGuard guard(p->device);
  if (lanes_per_row) p->lanes = lanes_per_row;
  if (tr_chunk) p->tr_chunk = tr_chunk;
  build_tr_items(p);
  drop_graph(p);
  fredopt_status st = upload_items(p, nullptr);
  if (st != FREDOPT_OK) return st;
  st = upload_table(p, nullptr);
  if (st != FREDOPT_OK) return st;
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
  DevPlan saved = p->hp;
  // forward width: dose / LETd outputs into the plan's own d and l buffers
  p->hp.x = const_cast<float*>(x);
  p->hp.prm.c = 0.04;
  p->hp.out_dose = p->hp.d;
  p->hp.out_letd = p->hp.l;
  p->hp.out_cdl = nullptr;
  fredopt_status st = FREDOPT_OK;
  int best_lanes = p->lanes;
  double best = 1e30;
  for (int g : {4, 8, 16, 32, 64}) {
    p->lanes = g;
    p->hp.lanes = g;
    if ((st = upload_table(p, s)) != FREDOPT_OK) break;
    const double t = timeit(Launch{0, 0, kFwdDoseLet}, 5);
    if (t < best) {
      best = t;
      best_lanes = g;
    }
  }
  p->lanes = best_lanes;
  p->hp.lanes = best_lanes;
  // transposed chunk: gradient mode on zero coefficients
  HIPCHK(hipMemsetAsync(p->hp.coef, 0, sizeof(float2) * (p->R > 0 ? p->R : 1), s));
  int best_chunk = p->tr_chunk;
  best = 1e30;
  if (st == FREDOPT_OK && (st = upload_table(p, s)) == FREDOPT_OK) {
    for (int ch : {1024, 2048, 4096, 8192, 16384}) {
      p->tr_chunk = ch;
      build_tr_items(p);
      if ((st = upload_items(p, s)) != FREDOPT_OK) break;
      const double t = timeit(Launch{0, 2, kTrGrad}, 5);
      if (t < best) {
        best = t;
        best_chunk = ch;
      }
    }
  }
  p->tr_chunk = best_chunk;
  build_tr_items(p);
  saved.lanes = p->lanes;
  p->hp = saved;
  if (st == FREDOPT_OK) st = upload_items(p, s);
  if (st == FREDOPT_OK) st = upload_table(p, s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  drop_graph(p);
  HIPCHK(hipStreamSynchronize(s));
  return st;
}

}  // extern "C"
