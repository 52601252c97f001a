// Iteration kernels of the superiorized dose / LETd feasibility-seeking loop
// (Borys et al., arXiv 2509.20012, Figs. 2-3, Eq. 2) for gfx950.
//
//  k_forward    d = D v and l = L v over a sliced-ELL copy (rows sorted by length
//               inside windows, lpr lanes per row, 16-byte loads per lane and step,
//               the vector staged in LDS), groups of 8 slices per 512-thread
//               workgroup, handed out by an atomic counter (all-row passes) or round
//               robin (objective-row passes, whose groups are balanced by weight);
//               scheduling only: every group writes its own partial, so results do
//               not depend on the schedule.  Epilogues: dose / LETd / cDL (Eq. 1, with
//               per-voxel scenario bands), Eq. (2) value and gradient coefficients,
//               the direction products with Q, or the Fig. 2 residuals folded into
//               projection coefficients.
//  k_rows       moves d and l along the accepted perturbation and evaluates the
//               constraint residuals (or the next gradient coefficients).
//  k_tr_chunks  D^T cD + L^T cL over the CSC copy, one wavefront per fixed-size chunk
//               of a column; chunk partials only (no floating-point atomics).
//  k_active_list  the rows with a non-zero projection coefficient, compacted in slice
//               order (or, on the column-major path, the coefficients in row order).
//  k_project    the sweep's transposed product by the path the device chose: the
//               active-row scatter (64-bit fixed-point sums in LDS, order free) and
//               the column-major chunk walk in one launch; k_scatter is the scatter
//               alone (block-sequential sweeps).
//  k_scatter_sum  per column: the scatter shares or the chunk partials, then the
//               projection update and the x >= 0 clamp (Fig. 2, last loop).
//  k_tcol       per column: gradient chunk sums, moves of y and x, the clamp.
//  k_finalize   one workgroup per plan: sums the partial slots in a fixed order (FP64)
//               and makes the plan-level decisions (step size of Fig. 3, weights,
//               list offsets, projection path).
//  k_search_part, k_linesearch  the one-sided objective's step search (Fig. 3's
//               trials, a window of candidate exponents at a time).
//  k_band_fill, k_band_finish  per-voxel min / max bands of a robustness evaluation.
//
// Partial slot layout (kNPart doubles):
//   objective pass  [0] chi^2                         [5] non-finite rows
//   direction pass  [0] Q                             [5] non-finite rows
//   residual pass   [0] sum w (enabled) [1] sum w (violated) [2] sum w v^2/||a||^2
//                   [3] violated  [4] degenerate  [5] non-finite  [6] chi^2
//                   [7] rows with a non-zero projection coefficient
//                   [8] sum over those rows of |cD| sum D + |cL| sum L (stored units)
//                   [9] stored entries of those rows
#include "fredopt_device.h"
#include "kernels.h"

#include <math.h>

namespace fo {

// Matrix entries are streamed once per pass and never re-read within it: the loads
// carry the non-temporal hint so they do not displace the vectors held in cache.
template <typename T>
__device__ __forceinline__ T stream_load(const FO_GLOBAL T* p) {
  return __builtin_nontemporal_load(p);
}

__device__ __forceinline__ v4i load_idx4(const FO_GLOBAL int32_t* p) {
  return stream_load((const FO_GLOBAL v4i*)p);
}

// Column indices of the sliced-ELL copy: the slice starting at element sb, and the
// four indices at element e of it.
template <int VT>
__device__ __forceinline__ const FO_GLOBAL void* sell_idx_ptr(const void* base, int64_t sb) {
  return (const FO_GLOBAL char*)(base) + sb * (index16(VT) ? 2 : 4);
}

template <int VT>
__device__ __forceinline__ v4i sell_idx4(const FO_GLOBAL void* ci, uint32_t e) {
  if constexpr (index16(VT)) {
    const v2u u = stream_load((const FO_GLOBAL v2u*)((const FO_GLOBAL uint16_t*)ci + e));
    return v4i{(int)(u.x & 0xffffu), (int)(u.x >> 16), (int)(u.y & 0xffffu), (int)(u.y >> 16)};
  } else {
    return load_idx4((const FO_GLOBAL int32_t*)ci + e);
  }
}

// Four consecutive stored values starting at element e of a global array, as floats.
template <int VT>
struct VLoad;

template <>
struct VLoad<kF32> {
  static __device__ __forceinline__ v4f q4(const FO_GLOBAL void* p, uint32_t e) {
    return stream_load((const FO_GLOBAL v4f*)((const FO_GLOBAL float*)p + e));
  }
};

template <>
struct VLoad<kF16> {
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4f q4(const FO_GLOBAL void* p, uint32_t e) {
    const h4 h = stream_load((const FO_GLOBAL h4*)((const FO_GLOBAL _Float16*)p + e));
    return v4f{(float)h.x, (float)h.y, (float)h.z, (float)h.w};
  }
};

template <>
struct VLoad<kBF16> {
  static __device__ __forceinline__ v4f q4(const FO_GLOBAL void* p, uint32_t e) {
    const v2u u = stream_load((const FO_GLOBAL v2u*)((const FO_GLOBAL uint16_t*)p + e));
    return v4f{__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
               __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u)};
  }
};

template <>
struct VLoad<kF16I> : VLoad<kF16> {};
template <>
struct VLoad<kBF16I> : VLoad<kBF16> {};

template <int VT>
__device__ __forceinline__ const FO_GLOBAL void* value_ptr(const void* base, int64_t e) {
  const int vb = VT == kF32 ? 4 : 2;
  return (const FO_GLOBAL char*)(base) + e * vb;
}

// ------------------------------------------------------------------ reductions --

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ float wave_sumf(float v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sum over a 256-thread block in a fixed order; every thread gets the result.
// Sum over a workgroup of NW waves (result in every thread; fixed order).
template <int NW = kBlock / kWave>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int tid = threadIdx.x;
  __syncthreads();
  if ((tid & (kWave - 1)) == 0) sh[tid / kWave] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) r += sh[w];
  __syncthreads();
  return r;
}

// Exclusive prefix sum over a workgroup of NW waves; *total gets the sum.
template <int NW>
__device__ __forceinline__ int block_scan(int v, int* sh, int* total) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  int x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == kWave - 1) sh[wave] = x;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    before += w < wave ? sh[w] : 0;
    all += sh[w];
  }
  *total = all;
  return before + x - v;
}

// ---------------------------------------------------------------- epilogues ----

// The Eq. (2) data of one view in its position order.
struct ObjArrays {
  const uint16_t* kind;
  const float *wo, *dt, *ct;
  float2* coef;
};

template <int SUB>
__device__ __forceinline__ ObjArrays obj_arrays(const DevPlan* P) {
  if constexpr (SUB) return ObjArrays{P->okind, P->owo, P->odt, P->oct, P->gcoef};
  else return ObjArrays{P->kind, P->wo, P->dt, P->ct, P->gcoef};
}

// A row's epilogue inputs, read at the start of its slice so that their latency
// overlaps the slice's matrix stream (read in the epilogue, each of the row's kinds
// cost a dependent memory round trip with no matrix loads in flight).  Every array
// holds a value at every position of its view; padding positions have kind 0 and
// their values are never used.
struct RowIn {
  float wo = 0.f, dt = 0.f, ct = 0.f;                          // Eq. (2)
  float wf = 0.f, dhi = 0.f, dlo = 0.f, chi = 0.f, clo = 0.f, tmax = 0.f;  // Fig. 2
  double sdd = 0.0, sll = 0.0, sdl = 0.0;                      // row moments
};

__device__ __forceinline__ void load_obj_in(const ObjArrays& A, int r, RowIn* in) {
  in->wo = gconst(A.wo)[r];
  in->dt = gconst(A.dt)[r];
  in->ct = gconst(A.ct)[r];
}

__device__ __forceinline__ void load_feas_in(const DevPlan* P, int r, RowIn* in) {
  in->wf = gconst(P->wf)[r];
  in->dhi = gconst(P->dhi)[r];
  in->dlo = gconst(P->dlo)[r];
  in->chi = gconst(P->chi)[r];
  in->clo = gconst(P->clo)[r];
  in->tmax = gconst(P->tmax)[r];
  const FO_GLOBAL double* m = gconst(P->mom) + 3 * (int64_t)r;
  in->sdd = m[0];
  in->sll = m[1];
  in->sdl = m[2];
}

// Whether the OAR term of Eq. (2) counts at residual f = cDLhat - c l: always as
// printed; only above the target (f < 0) with the one-sided objective.
__device__ __forceinline__ bool oar_on(const DevPlan* P, double f) {
  return P->prm.objective == 0 || f < 0.0;
}

// Eq. (2) terms of a row (kinds k, inputs in) at (d, l): adds the value to *chi and
// stores the gradient coefficients (-2 w (Dhat - d), -2 c w (cDLhat - c l)) at index
// rc (the row).
__device__ __forceinline__ void objective_row(const DevPlan* P, const ObjArrays& A,
                                              const RowIn& in, int rc, unsigned k, float d,
                                              float l, double* chi) {
  double uD = 0.0, uL = 0.0;
  if (k & (kObjDose | kObjCdl)) {
    const double w = in.wo, c = P->prm.c;
    if (k & kObjDose) {
      const double e = (double)in.dt - (double)d;
      *chi += w * e * e;
      uD = -2.0 * w * e;
    }
    if (k & kObjCdl) {
      const double f = (double)in.ct - c * (double)l;
      if (oar_on(P, f)) {
        *chi += w * f * f;
        uL = -2.0 * c * w * f;
      }
    }
  }
  ((FO_GLOBAL v2f*)(A.coef))[rc] = v2f{(float)uD, (float)uL};
}

__device__ __forceinline__ double objective_value(const DevPlan* P, const RowIn& in, unsigned k,
                                                  float d, float l) {
  double s = 0.0;
  if (k & (kObjDose | kObjCdl)) {
    const double w = in.wo, c = P->prm.c;
    if (k & kObjDose) {
      const double e = (double)in.dt - (double)d;
      s += w * e * e;
    }
    if (k & kObjCdl) {
      const double f = (double)in.ct - c * (double)l;
      if (oar_on(P, f)) s += w * f * f;
    }
  }
  return s;
}

// Fig. 2 at (d, l) for every enabled kind of row r: signed violation v (strict
// comparisons, equality is feasible), unscaled step lambda * w_i * v / ||a||^2
// folded into the (D, L) coefficient pair of the row.  ||a||^2 comes from the row
// moments: ||D_i||^2, c^2 ||L_i||^2, ||L_i - T D_i||^2 = sum L^2 - 2T sum DL +
// T^2 sum D^2.  Accumulates slots [0]..[4] of the residual layout.
__device__ __forceinline__ void residual_row(const DevPlan* P, const RowIn& in, int r,
                                             unsigned k, float d, float l, double* acc) {
  double kD = 0.0, kL = 0.0;
  if (k & kConstraintBits) {
    const double w = in.wf, lam = P->prm.lambda, c = P->prm.c;
    const double dd = d, ll = l;
    const double sdd = in.sdd, sll = in.sll, sdl = in.sdl;
    auto take = [&](double v, double n2, double scale, int which, double T) {
      if (!(n2 > kDegenerateRel * scale)) {
        acc[4] += 1.0;
        return;
      }
      const double kap = lam * w * v / n2;
      acc[1] += w;
      acc[2] += w * v * v / n2;
      acc[3] += 1.0;
      if (which == 0) {
        kD += kap;
      } else if (which == 1) {
        kL += c * kap;
      } else {
        kL += kap;
        kD -= T * kap;
      }
    };
    if (k & kDoseHi) {
      acc[0] += w;
      const double b = in.dhi;
      if (dd > b) take(dd - b, sdd, sdd, 0, 0.0);
    }
    if (k & kDoseLo) {
      acc[0] += w;
      const double b = in.dlo;
      if (dd < b) take(dd - b, sdd, sdd, 0, 0.0);
    }
    if (k & kCdlHi) {
      acc[0] += w;
      const double b = in.chi, ax = c * ll;
      if (ax > b) take(ax - b, c * c * sll, c * c * sll, 1, 0.0);
    }
    if (k & kCdlLo) {
      acc[0] += w;
      const double b = in.clo, ax = c * ll;
      if (ax < b) take(ax - b, c * c * sll, c * c * sll, 1, 0.0);
    }
    if (k & kLetdHi) {
      acc[0] += w;
      const double T = in.tmax, ax = ll - T * dd;
      if (ax > 0.0) take(ax, sll - 2.0 * T * sdl + T * T * sdd, sll + T * T * sdd, 2, T);
    }
  }
  const float fD = (float)kD, fL = (float)kL;
  ((FO_GLOBAL v2f*)(P->coef))[r] = v2f{fD, fL};
  if (fD != 0.f || fL != 0.f) {
    const v2f rs = ((const FO_GLOBAL v2f*)(P->rsum))[r];
    acc[7] += 1.0;
    acc[8] += fabs((double)fD) * (double)rs.x + fabs((double)fL) * (double)rs.y;
    acc[9] += (double)gconst(P->plen)[r];
  }
}

__device__ __forceinline__ bool finite2(float a, float b) { return isfinite(a) && isfinite(b); }

// A plan whose iteration produced a non-finite value is halted: every later kernel of
// the call skips it (the flag is set by a finalisation kernel and cleared when the
// host uploads a state), so x keeps the iterate reached when it was detected and a
// long solve does no further work on it.
__device__ __forceinline__ bool halted(const DevPlan* P) { return P->st->nonfinite != 0; }

// Plan-level completion of a residual pass: proximity, weights, the projection
// scale weight_scale / W, and the outer counter (Fig. 3: weights eta^k w).
__device__ __forceinline__ void finalize_residuals(const DevPlan* P, const double* s) {
  DevState* st = P->st;
  const double wall = s[0], wviol = s[1];
  st->w_all = wall;
  st->w_viol = wviol;
  st->proximity = wall > 0.0 ? 0.5 * s[2] / wall : 0.0;
  st->n_violated = (int64_t)s[3];
  st->n_degenerate = (int64_t)s[4];
  if (s[5] > 0.0) st->nonfinite = 1;
  st->cost_y = s[6];
  const int norm = P->prm.normalization;
  const double W = norm == 0 ? wall : (norm == 1 ? wviol : 1.0);
  const double ws = P->prm.ws_fixed >= 0.0 ? P->prm.ws_fixed : pow(P->prm.eta, (double)st->k);
  st->ws = ws;
  st->scale = W > 0.0 ? ws / W : 0.0;
  if (P->prm.ws_fixed < 0.0) st->k += 1;
}

// Step decision of Fig. 3 on the device.  Along the direction v (g, or g / ||g||
// with unit_dir) the cost is quadratic: chi^2(y - beta v) - chi^2(y) =
// -beta slope + beta^2 Qv with slope = <g, v> (G = ||g||^2, or sqrt(G)) and Qv = Q(v)
// (Q, or Q / G), so a trial beta = alpha^s strictly lowers it iff beta Qv < slope.  s is
// the smallest integer above the previous s with that property (the inner loop of
// Fig. 3 tries s+1, s+2, ...).  A search that would need alpha^s < 1e-300 skips the
// perturbation and leaves s unchanged.  The moves take step = beta times the factor
// that turns g into v.
__device__ __forceinline__ void decide_step(const DevPlan* P, double G, double Q) {
  DevState* st = P->st;
  st->G = G;
  st->Q = Q;
  if (!isfinite(G) || !isfinite(Q)) st->nonfinite = 1;
  if (st->pstop || !(G > 0.0) || !isfinite(G) || !isfinite(Q)) {
    st->beta = 0.0;
    st->step = 0.0;
    st->pstop = 1;
    return;
  }
  const bool unit = P->prm.unit_dir != 0;
  const double nrm = sqrt(G);
  const double slope = unit ? nrm : G, Qv = unit ? Q / G : Q;
  const double a = P->prm.alpha;
  const int64_t s0 = st->s;
  auto ok = [&](int64_t s) { return pow(a, (double)s) * Qv < slope; };
  int64_t s = s0 + 1;
  if (!ok(s)) {
    // here Qv > 0: a^s Qv < slope  <=>  s > log(slope / Qv) / log(a)
    const double est = log(slope / Qv) / log(a);
    if (!(est < 1e6)) {
      st->beta = 0.0;
      st->step = 0.0;
      st->pstop = 1;
      st->capped = 1;
      return;
    }
    int64_t s1 = (int64_t)floor(est) - 2;
    if (s1 < s0 + 1) s1 = s0 + 1;
    while (s1 > s0 + 1 && ok(s1 - 1)) --s1;
    while (!ok(s1)) ++s1;
    s = s1;
  }
  const double beta = pow(a, (double)s);
  if (beta < kBetaFloor) {
    st->beta = 0.0;
    st->step = 0.0;
    st->pstop = 1;
    st->capped = 1;
    return;
  }
  st->s = s;
  st->beta = beta;
  st->step = unit ? beta / nrm : beta;
}

// The same inputs when the one-sided objective leaves the decision to the search
// kernel: records G and Q and stops the perturbations if there is no descent.
__device__ __forceinline__ void prepare_search(const DevPlan* P, double G, double Q) {
  DevState* st = P->st;
  st->G = G;
  st->Q = Q;
  st->beta = 0.0;
  st->step = 0.0;
  if (!isfinite(G) || !isfinite(Q)) st->nonfinite = 1;
  if (st->pstop || !(G > 0.0) || !isfinite(G) || !isfinite(Q)) st->pstop = 1;
}

// -------------------------------------------------------------- forward pass ---

// Order-preserving map of a float's bits to an unsigned integer (negative values
// below positive ones, -inf lowest, +inf highest), so integer atomic min / max keep
// per-voxel bands over scenarios regardless of the order the scenarios arrive in.
__host__ __device__ __forceinline__ uint32_t band_enc(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ __forceinline__ float band_dec(uint32_t e) {
  return __uint_as_float((e & 0x80000000u) ? (e & 0x7FFFFFFFu) : ~e);
}

template <int MODE>
__device__ __forceinline__ constexpr unsigned fwd_slots() {
  return MODE == kFwdResid ? 0x3FFu : 0x21u;
}

// One slice of a sliced-ELL view: d = D v, l = L v for its rows, then the epilogue
// of MODE.  SUB selects the objective-row view, whose direction pass only needs Q.
// Without LDS staging the vector is read from global memory; gmv != null: the vector
// is vec - beta gmv (the pending perturbation step, kVecYMove).
template <int VT, int MODE, int SUB>
__device__ __forceinline__ void forward_slice(const DevPlan* __restrict__ P, int s,
                                              const float* __restrict__ xs, bool use_lds,
                                              const float* __restrict__ vec,
                                              const float* __restrict__ gmv, double beta,
                                              int lane, double* wpart) {
  const SellView& V = SUB ? P->osell : P->sell;
  const int lg2 = uniform(V.lpr_log2);
  const int lpr = 1 << lg2;
  const int rpw = kWave >> lg2;
  const int pos = lane >> lg2;
  const int64_t sb = gconst(V.sbase)[s];
  const int W = uniform(gconst(V.swidth)[s]);
  // the row's position: its data are indexed by it (padding positions have kind 0)
  const int sp = s * rpw + pos;
  const ObjArrays A = obj_arrays<SUB>(P);
  unsigned kind = 0;
  if constexpr (MODE != kFwdDoseLet) kind = gconst(A.kind)[sp];
  // the gradient coefficients are stored by row (the column-major gradient gathers them)
  int crow = 0;
  if constexpr (MODE == kFwdObj) crow = gconst(V.srow)[sp];
  // the epilogue's row inputs, requested before the matrix stream by every lane of
  // the row (the same addresses; loaded by the owner lane alone, the values become
  // a branch's results and the compiler converts them before the stream starts);
  // the direction pass needs the objective weight only
  RowIn in;
  if constexpr (MODE == kFwdDir) in.wo = gconst(A.wo)[sp];
  if constexpr (MODE == kFwdObj || MODE == kFwdResid) load_obj_in(A, sp, &in);
  if constexpr (MODE == kFwdResid) load_feas_in(P, sp, &in);
  // slice-relative element offsets fit 32 bits; the slice bases are wave-uniform

  const FO_GLOBAL void* ci = sell_idx_ptr<VT>(V.sci, sb);
  const FO_GLOBAL void* dv = value_ptr<VT>(V.sdv, sb);
  const FO_GLOBAL void* lv = value_ptr<VT>(V.slv, sb);
  float ad = 0.f, al = 0.f;
  if (use_lds) {
#pragma unroll 4
    for (int t = 0; t < W; ++t) {
      const uint32_t e = (uint32_t)t * 256u + 4u * (uint32_t)lane;
      const v4i c4 = sell_idx4<VT>(ci, e);
      const v4f d4 = VLoad<VT>::q4(dv, e);
      const v4f l4 = VLoad<VT>::q4(lv, e);
      const float x0 = xs[c4.x], x1 = xs[c4.y], x2 = xs[c4.z], x3 = xs[c4.w];
      ad = fmaf(d4.x, x0, ad);
      ad = fmaf(d4.y, x1, ad);
      ad = fmaf(d4.z, x2, ad);
      ad = fmaf(d4.w, x3, ad);
      al = fmaf(l4.x, x0, al);
      al = fmaf(l4.y, x1, al);
      al = fmaf(l4.z, x2, al);
      al = fmaf(l4.w, x3, al);
    }
  } else {
    const FO_GLOBAL float* cs = gconst(P->cscale);
    const FO_GLOBAL float* gv = gconst(vec);
    const FO_GLOBAL float* gg = gconst(gmv);
    const bool scaled = P->cscale != nullptr;
    auto val = [&](int c) {
      const float v = gmv ? (float)((double)gv[c] - beta * (double)gg[c]) : gv[c];
      return scaled ? v * cs[c] : v;
    };
    for (int t = 0; t < W; ++t) {
      const uint32_t e = (uint32_t)t * 256u + 4u * (uint32_t)lane;
      const v4i c4 = sell_idx4<VT>(ci, e);
      const v4f d4 = VLoad<VT>::q4(dv, e);
      const v4f l4 = VLoad<VT>::q4(lv, e);
      const float x0 = val(c4.x);
      const float x1 = val(c4.y);
      const float x2 = val(c4.z);
      const float x3 = val(c4.w);
      ad = fmaf(d4.x, x0, ad);
      ad = fmaf(d4.y, x1, ad);
      ad = fmaf(d4.z, x2, ad);
      ad = fmaf(d4.w, x3, ad);
      al = fmaf(l4.x, x0, al);
      al = fmaf(l4.y, x1, al);
      al = fmaf(l4.z, x2, al);
      al = fmaf(l4.w, x3, al);
    }
  }
  for (int o = lpr >> 1; o > 0; o >>= 1) {
    ad += __shfl_xor(ad, o);
    al += __shfl_xor(al, o);
  }
  double acc[kNPart];
#pragma unroll
  for (int k = 0; k < kNPart; ++k) acc[k] = 0.0;
  if ((lane & (lpr - 1)) == 0) {
    if constexpr (MODE == kFwdDoseLet) {
      // outputs in the caller's row order
      const int row = gconst(V.srow)[sp];
      if (row >= 0) {
        const float letd = ad > 0.f ? al / ad : 0.f;
        if (P->out_dose) gmut(P->out_dose)[row] = ad;
        if (P->out_letd) gmut(P->out_letd)[row] = letd;
        if (P->out_cdl) gmut(P->out_cdl)[row] = (float)(P->prm.c * (double)al);
        if (P->band[0]) {  // robustness evaluation: the scenario joins the voxel's bands
          atomicMin(P->band[0] + row, band_enc(ad));
          atomicMax(P->band[1] + row, band_enc(ad));
        }
        if (P->band[2]) {
          atomicMin(P->band[2] + row, band_enc(letd));
          atomicMax(P->band[3] + row, band_enc(letd));
        }
      }
    } else if constexpr (MODE == kFwdObj) {
      if constexpr (!SUB) {  // the all-row pass keeps d and l for the moves
        gmut(P->d)[sp] = ad;
        gmut(P->l)[sp] = al;
      } else {               // the objective-row view keeps them for the step search
        gmut(P->od)[sp] = ad;
        gmut(P->ol)[sp] = al;
      }
      if (crow >= 0) objective_row(P, A, in, crow, kind, ad, al, &acc[0]);
      if (!finite2(ad, al)) acc[5] += 1.0;
    } else if constexpr (MODE == kFwdDir) {
      if constexpr (!SUB) {
        gmut(P->dg)[sp] = ad;
        gmut(P->lg)[sp] = al;
      } else {
        gmut(P->odg)[sp] = ad;
        gmut(P->olg)[sp] = al;
      }
      if (kind & (kObjDose | kObjCdl)) {
        const double wo = in.wo, c = P->prm.c;
        if (kind & kObjDose) acc[0] += wo * (double)ad * (double)ad;
        if (kind & kObjCdl) acc[0] += wo * c * c * (double)al * (double)al;
      }
      if (!finite2(ad, al)) acc[5] += 1.0;
    } else {
      gmut(P->d)[sp] = ad;
      gmut(P->l)[sp] = al;
      residual_row(P, in, sp, kind, ad, al, acc);
      acc[6] += objective_value(P, in, kind, ad, al);
      if (!finite2(ad, al)) acc[5] += 1.0;
    }
  }
  if constexpr (MODE != kFwdDoseLet) {
    constexpr unsigned used = fwd_slots<MODE>();
#pragma unroll
    for (int k = 0; k < kNPart; ++k)
      if (used & (1u << k)) acc[k] = wave_sum(acc[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < kNPart; ++k) wpart[k] = acc[k];
    }
  }
}

// Copies v (times the per-column scales when SCALED) into LDS.  Each thread has
// kStage loads (kStageMix elements of two or three arrays) in flight before its first
// store, so the copy costs a few memory round trips instead of one per kFwdBlock
// elements.
constexpr int kStage = 16;
constexpr int kStageMix = 8;  // elements per round when two or three arrays are read

// One element of the staged vector: v, or v - beta g rounded to FP32 as the separate
// move would store it (MOVE), times the column scale (SCALED).
template <bool SCALED, bool MOVE>
__device__ __forceinline__ float staged(float v, float g, float cs, double beta) {
  float a = MOVE ? (float)((double)v - beta * (double)g) : v;
  if (SCALED) a *= cs;
  return a;
}

// MOVE: stages v - beta g, rounded to FP32 as the separate move would store it.
template <bool SCALED, bool MOVE>
__device__ __forceinline__ void stage_vector(const FO_GLOBAL float* v, const FO_GLOBAL float* cs,
                                             const FO_GLOBAL float* g, double beta, int C,
                                             float* xs, int tid) {
  if (C <= kFwdBlock) {  // one element per thread
    if (tid < C) xs[tid] = staged<SCALED, MOVE>(v[tid], MOVE ? g[tid] : 0.f,
                                                 SCALED ? cs[tid] : 0.f, beta);
    return;
  }
  if constexpr (!SCALED && !MOVE) {
    // a plain copy: the loads are issued together and only the stores are tested
    for (int j0 = tid; j0 < C; j0 += kStage * kFwdBlock) {
      float t[kStage];
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int j = j0 + u * kFwdBlock;
        t[u] = j < C ? v[j] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int j = j0 + u * kFwdBlock;
        if (j < C) xs[j] = t[u];
      }
    }
  } else {
    for (int j0 = tid; j0 < C; j0 += kStageMix * kFwdBlock) {
      // every load is issued before any value is used, and none sits behind a
      // branch: indices past the end take element C - 1 and store its own value
      // again.  With the arithmetic inside a bounds test, each element waited for its
      // own loads
      float tv[kStageMix], tg[kStageMix], ts[kStageMix];
#pragma unroll
      for (int u = 0; u < kStageMix; ++u) {
        const int j = min(j0 + u * kFwdBlock, C - 1);
        tv[u] = v[j];
        tg[u] = MOVE ? g[j] : 0.f;
        ts[u] = SCALED ? cs[j] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kStageMix; ++u)
        xs[min(j0 + u * kFwdBlock, C - 1)] = staged<SCALED, MOVE>(tv[u], tg[u], ts[u], beta);
    }
  }
}

template <int VT, int MODE, int SUB>
__global__ __launch_bounds__(kFwdBlock) void k_forward(const DevPlan* __restrict__ plans,
                                                       const FwdGroup* __restrict__ groups,
                                                       int n_groups, int lds_floats,
                                                       uint32_t* ctr, int vsel) {
  extern __shared__ float xs[];
  __shared__ int s_g;
  __shared__ double wpart[kFwdWaves][kNPart];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  int cur = -1;
  bool use_lds = false;
  const float* vec = nullptr;
  const float* gmv = nullptr;
  double beta = 0.0;
  int next = -1;  // thread 0: the next group, requested while this one finishes
  for (int it = 0;; ++it) {
    int gi;
    if (ctr) {  // dynamic: next group from a counter (taken only when this one is done,
                // so the last groups go to whichever workgroups are free)
      if (tid == 0) s_g = next >= 0 ? next : (int)atomicAdd(&ctr[0], 1u);
      __syncthreads();
      gi = s_g;
      if (gi >= n_groups) {
        // the last workgroup to run out of work re-arms the counters for the next launch
        if (tid == 0) {
          const unsigned e = atomicAdd(&ctr[1], 1u);
          if (e == gridDim.x - 1) {
            atomicExch(&ctr[0], 0u);
            atomicExch(&ctr[1], 0u);
          }
        }
        break;
      }
    } else {    // static: groups b, b + grid, b + 2 grid, ...
      __syncthreads();  // the previous group's partials are read before wpart is reused
      gi = blockIdx.x + it * gridDim.x;
      if (gi >= n_groups) break;
    }
    const FwdGroup G = groups[gi];
    const DevPlan* __restrict__ P = plans + G.plan;
    if (MODE != kFwdDoseLet && halted(P)) {  // uniform over the workgroup
      next = -1;
      continue;
    }
    if (G.plan != cur) {
      vec = vsel == kVecG ? P->g : (vsel == kVecX ? P->x : P->y);
      const bool move = vsel == kVecYMove;
      gmv = move ? P->g : nullptr;
      beta = move ? P->st->step : 0.0;
      use_lds = P->C <= (int64_t)lds_floats;
      if (use_lds) {
        const FO_GLOBAL float* gv = gconst(vec);
        const FO_GLOBAL float* cs = gconst(P->cscale);
        const FO_GLOBAL float* gg = gconst(gmv);
        const int C = (int)P->C;
        if (P->cscale) {
          if (move) stage_vector<true, true>(gv, cs, gg, beta, C, xs, tid);
          else stage_vector<true, false>(gv, cs, gg, beta, C, xs, tid);
        } else {
          if (move) stage_vector<false, true>(gv, cs, gg, beta, C, xs, tid);
          else stage_vector<false, false>(gv, cs, gg, beta, C, xs, tid);
        }
      }
      __syncthreads();
      cur = G.plan;
    }
    if (wave < G.n)
      forward_slice<VT, MODE, SUB>(P, G.slice0 + wave, xs, use_lds, vec, gmv, beta, lane,
                                   wpart[wave]);
    // the next group is requested once wave 0's slice is done, so that the counter's
    // round trip overlaps the other waves' work instead of following the group
    if (ctr && tid == 0) next = (int)atomicAdd(&ctr[0], 1u);
    __syncthreads();
    if constexpr (MODE != kFwdDoseLet) {
      // the group's partial: its slices' partials in wave order
      if (tid < kNPart) {
        double v = 0.0;
        for (int w = 0; w < G.n; ++w) v += wpart[w][tid];
        gmut(MODE == kFwdDir ? P->spart_b : P->spart_a)[(int64_t)G.slot * kNPart + tid] = v;
      }
    }
  }
}

// ------------------------------------------------------------------ rows pass --

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_rows(const DevPlan* __restrict__ plans,
                                                 const RowItem* __restrict__ items) {
  __shared__ double sh4[kBlock / kWave];
  const RowItem w = items[blockIdx.x];
  const DevPlan* __restrict__ P = plans + w.plan;
  if (halted(P)) return;
  const int tid = threadIdx.x;
  const double beta = P->st->step;  // the accepted move along g
  double acc[kNPart];
#pragma unroll
  for (int k = 0; k < kNPart; ++k) acc[k] = 0.0;
  for (int r = w.r0 + tid; r < w.r1; r += kBlock) {
    // the accepted perturbation y = x - beta g moves d and l by -beta (D g, L g)
    const float d = (float)((double)gmut(P->d)[r] - beta * (double)gmut(P->dg)[r]);
    const float l = (float)((double)gmut(P->l)[r] - beta * (double)gmut(P->lg)[r]);
    gmut(P->d)[r] = d;
    gmut(P->l)[r] = l;
    const ObjArrays A = obj_arrays<0>(P);
    RowIn in;
    load_obj_in(A, r, &in);
    if constexpr (MODE == kRowsMoveObj) {
      const int row = gconst(P->sell.srow)[r];
      if (row >= 0) objective_row(P, A, in, row, gconst(P->kind)[r], d, l, &acc[0]);
    } else {
      load_feas_in(P, r, &in);
      const unsigned kr = gconst(P->kind)[r];
      residual_row(P, in, r, kr, d, l, acc);
      acc[6] += objective_value(P, in, kr, d, l);
    }
    if (!finite2(d, l)) acc[5] += 1.0;
  }
  constexpr unsigned used = MODE == kRowsMoveObj ? 0x21u : 0x3FFu;
  double s[kNPart];
#pragma unroll
  for (int k = 0; k < kNPart; ++k) s[k] = (used & (1u << k)) ? block_sum(acc[k], sh4) : 0.0;
  if (tid == 0) {
    FO_GLOBAL double* dst = gmut(P->rpart) + (int64_t)w.slot * kNPart;
#pragma unroll
    for (int k = 0; k < kNPart; ++k) dst[k] = s[k];
  }
}

// ------------------------------------------------------------ transposed pass --

// Work items are laid out so that consecutive logical blocks cover consecutive
// columns; the hardware hands block b to XCD b % 8, so block b runs logical block
// (b % 8) * nb8 + b / 8 and each XCD's L2 sees a contiguous column range.
// TAG only separates the gradient (0) and projection (1) launches in profiles.
constexpr int kTrRound = 2;  // steps of a chunk whose loads are in flight together

template <int VT, int TAG>
__device__ __forceinline__ void tr_chunk(const DevPlan* __restrict__ plans, const TrItem& w,
                                         int lane);

// A persistent grid (a multiple of 8 workgroups) walks the virtual blocks
// vb = b, b + grid, ...; virtual block vb covers items of block
// (vb mod 8) nb8 + vb / 8, so each workgroup stays on one XCD's contiguous share of
// columns.  single: every item belongs to plans[0] (its projection path is checked
// once).
template <int VT, int TAG, int B>
__device__ __forceinline__ void chunk_walk(const DevPlan* __restrict__ plans,
                                           const TrItem* __restrict__ items, int n_items, int nb8,
                                           int single) {
  if (single && (halted(plans) || (TAG == 1 && plans[0].st->proj_scatter))) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int vb = blockIdx.x; vb < nb8 * 8; vb += gridDim.x) {
    const int lb = (vb & 7) * nb8 + (vb >> 3);
    const int it = lb * (B / kWave) + wave;
    if (it >= n_items) continue;
    const TrItem w = items[uniform(it)];
    if (!single && (halted(plans + w.plan) || (TAG == 1 && plans[w.plan].st->proj_scatter)))
      continue;
    tr_chunk<VT, TAG>(plans, w, lane);
  }
}

template <int VT, int TAG>
__global__ __launch_bounds__(kBlock) void k_tr_chunks(const DevPlan* __restrict__ plans,
                                                      const TrItem* __restrict__ items,
                                                      int n_items, int nb8, int single) {
  chunk_walk<VT, TAG, kBlock>(plans, items, n_items, nb8, single);
}

template <int VT, int TAG>
__device__ __forceinline__ void tr_chunk(const DevPlan* __restrict__ plans, const TrItem& w,
                                         int lane) {
  const DevPlan* __restrict__ P = plans + w.plan;
  // chunk-relative element offsets fit 32 bits; the chunk base is wave-uniform
  const FO_GLOBAL int32_t* ri = gconst(TAG == 0 ? P->gri : P->ri) + w.q0;
  const FO_GLOBAL void* cdv = value_ptr<VT>(TAG == 0 ? P->gcdv : P->cdv, w.q0);
  const FO_GLOBAL void* clv = value_ptr<VT>(TAG == 0 ? P->gclv : P->clv, w.q0);
  const FO_GLOBAL v2f* cf = (const FO_GLOBAL v2f*)(TAG == 0 ? P->gcoef : P->coef_row);
  const uint32_t n = (uint32_t)(w.q1 - w.q0);
  float acc = 0.f;
  // rounds of kTrRound steps of 4 kWave slots: the round's stream loads are issued
  // together, then its coefficient gathers, so a short chunk costs two memory round
  // trips per round (lanes past the chunk end are masked off)
  for (uint32_t t0 = 0; t0 < n; t0 += kTrRound * 4u * kWave) {
    v4i r4[kTrRound];
    v4f d4[kTrRound], l4[kTrRound];
#pragma unroll
    for (int u = 0; u < kTrRound; ++u) {
      const uint32_t e = t0 + (uint32_t)u * 4u * kWave + 4u * (uint32_t)lane;
      if (e < n) {
        r4[u] = load_idx4(ri + e);
        d4[u] = VLoad<VT>::q4(cdv, e);
        l4[u] = VLoad<VT>::q4(clv, e);
      }
    }
    v2f c[kTrRound][4];
#pragma unroll
    for (int u = 0; u < kTrRound; ++u) {
      const uint32_t e = t0 + (uint32_t)u * 4u * kWave + 4u * (uint32_t)lane;
      if (e < n) {
        c[u][0] = cf[(uint32_t)r4[u].x];
        c[u][1] = cf[(uint32_t)r4[u].y];
        c[u][2] = cf[(uint32_t)r4[u].z];
        c[u][3] = cf[(uint32_t)r4[u].w];
      }
    }
#pragma unroll
    for (int u = 0; u < kTrRound; ++u) {
      const uint32_t e = t0 + (uint32_t)u * 4u * kWave + 4u * (uint32_t)lane;
      if (e < n) {
        acc = fmaf(d4[u].x, c[u][0].x, acc);
        acc = fmaf(l4[u].x, c[u][0].y, acc);
        acc = fmaf(d4[u].y, c[u][1].x, acc);
        acc = fmaf(l4[u].y, c[u][1].y, acc);
        acc = fmaf(d4[u].z, c[u][2].x, acc);
        acc = fmaf(l4[u].z, c[u][2].y, acc);
        acc = fmaf(d4[u].w, c[u][3].x, acc);
        acc = fmaf(l4[u].w, c[u][3].y, acc);
      }
    }
  }
  acc = wave_sumf(acc);
  if (lane == 0) gmut(P->tpart)[w.tslot] = acc;
}

// ---------------------------------------------- projection over active rows ----

// The rows with a non-zero projection coefficient, group by group in slice order
// (list offsets from the residual finalisation), with what the scatter needs; when
// the sweep takes the column-major path instead, the coefficients in row order.  One
// workgroup per group, one thread per row position: the launch's block is the most
// rows a group of any of its plans holds (8 slices of 64 / lanes-per-row rows).
__global__ __launch_bounds__(kFwdBlock) void k_active_list(const DevPlan* __restrict__ plans,
                                                           const FwdGroup* __restrict__ groups,
                                                           int n_groups) {
  __shared__ int wsum[kFwdWaves];
  const FwdGroup G = groups[blockIdx.x];
  const DevPlan* __restrict__ P = plans + G.plan;
  if (halted(P)) return;
  const int rpw_log2 = 6 - P->lpr_log2;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int n = G.n << rpw_log2;
  const int sp = (G.slice0 << rpw_log2) + tid;
  if (!P->st->proj_scatter) {
    // the column-major path gathers the coefficients by row
    if (tid < n) {
      const int row = gconst(P->sell.srow)[sp];
      if (row >= 0)
        ((FO_GLOBAL v2f*)(P->coef_row))[row] = ((const FO_GLOBAL v2f*)(P->coef))[sp];
    }
    return;
  }
  // the residual pass counted the group's active rows
  if (gconst(P->spart_a)[(int64_t)G.slot * kNPart + 7] == 0.0) return;
  bool act = false;
  v2f c = v2f{0.f, 0.f};
  if (tid < n) {
    c = ((const FO_GLOBAL v2f*)(P->coef))[sp];
    act = c.x != 0.f || c.y != 0.f;
  }
  const uint64_t m = __ballot(act);
  if (lane == 0) wsum[wave] = __popcll(m);
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  before += __popcll(m & ((1ull << lane) - 1ull));
  if (act) {
    const int64_t off = gconst(P->rptr)[sp];
    const int nq = (int)((gconst(P->rptr)[sp + 1] - off) >> 2);
    // ActRow as two 16-byte stores
    FO_GLOBAL v4i* dst = (FO_GLOBAL v4i*)(P->alist + gconst(P->goff)[G.slot] + before);
    dst[0] = v4i{(int)(uint32_t)off, (int)(off >> 32), nq, gconst(P->plen)[sp]};
    dst[1] = v4i{__float_as_int(c.x), __float_as_int(c.y), 0, 0};
  }
}

__device__ __forceinline__ void fx_add(unsigned long long* acc, int col, double v, double fs) {
  if (v != 0.0) atomicAdd(&acc[col], (unsigned long long)__double2ll_rn(v * fs));
}

// The same fixed-point sum kept in global memory (device-scope integer atomics) for
// plans whose C column sums do not fit in LDS.
__device__ __forceinline__ void fx_add_global(unsigned long long* acc, int col, double v,
                                              double fs) {
  if (v != 0.0) atomicAdd(&acc[col], (unsigned long long)__double2ll_rn(v * fs));
}

// D^T cD + L^T cL over the active rows only.  Contributions are rounded to 64-bit
// fixed point (scale 2^61 / bound from the residual pass) and added with integer LDS
// atomics: integer sums do not depend on the order of the additions, so the waves of
// a workgroup take rows concurrently and the result is still reproducible bit for
// bit.  Workgroup w takes a contiguous share of the list; the column kernel adds
// the shares.
template <int VT>
__device__ __forceinline__ void scatter_share(const DevPlan* __restrict__ plans, const ScItem item,
                                              unsigned long long* facc) {
  const DevPlan* __restrict__ P = plans + item.plan;
  const int wg = item.idx;
  if (halted(P) || !P->st->proj_scatter) return;
  const int C = (int)P->C;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  // column sums in LDS, or (plans too wide for LDS) in global memory, where the
  // column update reads them and leaves them zero for the next sweep
  const bool glob = P->scatter_global != 0;
  unsigned long long* acc = glob ? (unsigned long long*)P->spart : facc;
  if (!glob)
    for (int j = tid; j < C; j += kScatterBlock) facc[j] = 0ull;
  __syncthreads();
  const int64_t A = P->st->n_active, NW = P->n_scatter;
  const int i0 = (int)(wg * A / NW), i1 = (int)((wg + 1) * A / NW);
  // groups of G lanes take one row each (G from the plan's mean row length); a row's
  // entries are contiguous in the row copy, and so are neighbouring rows of the list,
  // so a wave reads whole lines
  const int lg2 = P->sc_lg2, G = 1 << lg2, rg = kWave >> lg2;
  const int grp = lane >> lg2, gl = lane & (G - 1);
  const double fs = P->st->fx_scale;
  const ActRow* list = P->alist;
  // the next row's record is loaded while this row's entries stream, and a row's
  // quads go out two steps at a time before their additions
  const int stride = (kScatterBlock / kWave) * rg;
  int i = i0 + wave * rg + grp;
  v4i n0 = v4i{0, 0, 0, 0}, n1 = n0;
  if (i < i1) {
    n0 = ((const FO_GLOBAL v4i*)(list + i))[0];
    n1 = ((const FO_GLOBAL v4i*)(list + i))[1];
  }
  for (; i < i1; i += stride) {
    const v4i a0 = n0, a1 = n1;
    if (i + stride < i1) {
      n0 = ((const FO_GLOBAL v4i*)(list + i + stride))[0];
      n1 = ((const FO_GLOBAL v4i*)(list + i + stride))[1];
    }
    const int64_t off = (int64_t)(((uint64_t)(uint32_t)a0.y << 32) | (uint32_t)a0.x);
    const int nq = a0.z;
    const double cd = __int_as_float(a1.x), cl = __int_as_float(a1.y);

    const FO_GLOBAL void* ci = sell_idx_ptr<VT>(P->rci, off);
    const FO_GLOBAL void* dv = value_ptr<VT>(P->rdv, off);
    const FO_GLOBAL void* lv = value_ptr<VT>(P->rlv, off);
    for (int q0 = gl; q0 < nq; q0 += 2 * G) {
      v4i c4[2];
      v4f d4[2], l4[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int q = q0 + u * G;
        c4[u] = v4i{0, 0, 0, 0};
        d4[u] = v4f{0.f, 0.f, 0.f, 0.f};
        l4[u] = d4[u];
        if (q < nq) {
          const uint32_t e = (uint32_t)q * 4u;
          c4[u] = sell_idx4<VT>(ci, e);
          d4[u] = VLoad<VT>::q4(dv, e);
          l4[u] = VLoad<VT>::q4(lv, e);
        }
      }
      // padding slots (and the second step past the row's end) hold 0 and add nothing
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (glob) {
          fx_add_global(acc, c4[u].x, cd * d4[u].x + cl * l4[u].x, fs);
          fx_add_global(acc, c4[u].y, cd * d4[u].y + cl * l4[u].y, fs);
          fx_add_global(acc, c4[u].z, cd * d4[u].z + cl * l4[u].z, fs);
          fx_add_global(acc, c4[u].w, cd * d4[u].w + cl * l4[u].w, fs);
        } else {
          fx_add(facc, c4[u].x, cd * d4[u].x + cl * l4[u].x, fs);
          fx_add(facc, c4[u].y, cd * d4[u].y + cl * l4[u].y, fs);
          fx_add(facc, c4[u].z, cd * d4[u].z + cl * l4[u].z, fs);
          fx_add(facc, c4[u].w, cd * d4[u].w + cl * l4[u].w, fs);
        }
      }
    }
  }
  if (glob) return;  // no shares: the sums are already in global memory
  __syncthreads();
  // non-zero sums only, with a bit mask per 64 columns saying which were written
  const int nwords = (C + kWave - 1) / kWave;
  FO_GLOBAL int64_t* out = gmut(P->spart) + (int64_t)wg * C;
  FO_GLOBAL uint64_t* msk = gmut(P->smask) + (int64_t)wg * nwords;
  for (int w = wave; w < nwords; w += kScatterBlock / kWave) {
    const int j = w * kWave + lane;
    const int64_t v = j < C ? (int64_t)facc[j] : 0;
    const uint64_t m = __ballot(v != 0);
    if (v != 0) out[j] = v;
    if (lane == 0) msk[w] = m;
  }
}

template <int VT>
__global__ __launch_bounds__(kScatterBlock) void k_scatter(const DevPlan* __restrict__ plans,
                                                          const ScItem* __restrict__ items) {
  extern __shared__ unsigned long long facc[];
  scatter_share<VT>(plans, items[blockIdx.x], facc);
}

// The sweep's transposed product by either path in one launch: the device chose the
// path of each plan (proj_scatter), and a kernel whose workgroups only return still
// costs a launch.  Workgroup b takes scatter share b (plans on the active-row path),
// then its part of the persistent walk over the column-major chunks (plans on the
// column-major path); VT is the row copy's storage, VC the column copy's.
template <int VT, int VC>
__global__ __launch_bounds__(kScatterBlock) void k_project(const DevPlan* __restrict__ plans,
                                                          const ScItem* __restrict__ sc, int n_sc,
                                                          const TrItem* __restrict__ tr, int n_tr,
                                                          int nb8, int single) {
  extern __shared__ unsigned long long facc[];
  if ((int)blockIdx.x < n_sc) scatter_share<VT>(plans, sc[blockIdx.x], facc);
  if (n_tr > 0) chunk_walk<VC, 1, kScatterBlock>(plans, tr, n_tr, nb8, single);
}

// The projection update of column j (Fig. 2, last loop) from the transposed sum t
// in stored units: x = max(0, y - scale t), with y = x, x - beta g or the perturbed
// point, by MODE.  The column's inputs are loaded apart from the update, so that a
// caller can have them in flight while it forms t.
struct ColIn {
  float cs;      // the column's scale of stored values (1 if none)
  double y;      // the point the update starts from
  double scale;  // the sweep's weight scale
};

template <int MODE>
__device__ __forceinline__ ColIn load_column(const DevPlan* __restrict__ P, int j) {
  constexpr bool fromy = MODE == kColProjY || MODE == kColProjYMove;
  ColIn in;
  in.cs = P->cscale ? gconst(P->cscale)[j] : 1.f;
  double y = fromy ? gconst(P->y)[j] : gconst(P->x)[j];
  if constexpr (MODE == kColProjMove) y -= P->st->step * (double)gconst(P->g)[j];
  // the perturbed point y - beta g, rounded to FP32 as the residual pass staged it
  if constexpr (MODE == kColProjYMove)
    y = (double)(float)(y - P->st->step * (double)gconst(P->g)[j]);
  in.y = y;
  in.scale = P->st->scale;
  return in;
}

template <int MODE>
__device__ __forceinline__ void apply_column(const DevPlan* __restrict__ P, int j, float t,
                                             const ColIn& in) {
  constexpr bool fromy = MODE == kColProjY || MODE == kColProjYMove;
  if (P->cscale) t *= in.cs;
  const double xn = in.y - in.scale * (double)t;
  if constexpr (MODE == kColProjNoClamp) {  // the clamp waits for the sweep's end
    gmut(P->x)[j] = (float)xn;
    return;
  }
  const float xf = xn > 0.0 ? (float)xn : 0.f;
  gmut(P->x)[j] = xf;
  if constexpr (fromy) gmut(P->y)[j] = xf;
}

template <int MODE>
__device__ __forceinline__ void project_column(const DevPlan* __restrict__ P, int j, float t) {
  apply_column<MODE>(P, j, t, load_column<MODE>(P, j));
}

// The sweep's update of 64 columns: on the active-row path, the sum of the scatter
// workgroups' shares (16 waves take every 16th share; integer sums, so the grouping
// does not matter); on the column-major path, the column's chunk partials in chunk
// order.  Then the projection update and clamp.
template <int MODE>
__global__ __launch_bounds__(kScatterBlock) void k_scatter_sum(const DevPlan* __restrict__ plans,
                                                              const ScItem* __restrict__ items) {
  __shared__ int64_t part[kScatterBlock / kWave][kWave];
  const ScItem item = items[blockIdx.x];
  const DevPlan* __restrict__ P = plans + item.plan;
  if (halted(P)) return;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int C = (int)P->C, nwords = (C + kWave - 1) / kWave;
  const int j = item.idx * kWave + lane;
  if (!P->st->proj_scatter) {
    // the column-major path: the column's chunk partials in chunk order
    if (wave == 0 && j < C) {
      const int ts = gconst(P->col_tslot0)[j], n = gconst(P->col_nch)[j];
      float t = 0.f;
      for (int c = 0; c < n; ++c) t += gconst(P->tpart)[ts + c];
      project_column<MODE>(P, j, t);
    }
    return;
  }
  if (P->scatter_global) {
    // the column sums in global memory; each is read once and set back to zero
    if (wave == 0 && j < C) {
      FO_GLOBAL int64_t* g = gmut(P->spart) + j;
      const int64_t S = *g;
      *g = 0;
      project_column<MODE>(P, j, (float)((double)S / P->st->fx_scale));
    }
    return;
  }
  // the column's own inputs go out with the masks
  ColIn in{1.f, 0.0, 0.0};
  if (wave == 0 && j < C) in = load_column<MODE>(P, j);
  const FO_GLOBAL int64_t* sp = gconst(P->spart) + j;
  const FO_GLOBAL uint64_t* mk = gconst(P->smask) + item.idx;
  // all masks first, then the shares they mark: two dependent rounds of loads
  constexpr int kNW = kScatterBlock / kWave, kPer = kScatterMaxWGs / kNW;
  const int NW = P->n_scatter;
  uint64_t m[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int w = wave + i * kNW;
    m[i] = w < NW ? mk[(int64_t)w * nwords] : 0ull;
  }
  // the marked shares' loads all go out before the first add (with the add inside
  // the bit test, each share waited for its own load); a set bit implies j < C
  int64_t v[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i)
    v[i] = ((m[i] >> lane) & 1ull) ? sp[(int64_t)(wave + i * kNW) * C] : int64_t(0);
  int64_t S = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) S += v[i];
  part[wave][lane] = S;
  __syncthreads();
  if (wave == 0) {
    for (int v = 1; v < kScatterBlock / kWave; ++v) S += part[v][lane];
    if (j < C) apply_column<MODE>(P, j, (float)((double)S / P->st->fx_scale), in);
  }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_tcol(const DevPlan* __restrict__ plans,
                                                 const ColBlock* __restrict__ blocks) {
  __shared__ double sh4[kBlock / kWave];
  const ColBlock cb = blocks[blockIdx.x];
  const DevPlan* __restrict__ P = plans + cb.plan;
  if (MODE != kColYCopy && halted(P)) return;
  const int j = cb.c0 + threadIdx.x;
  constexpr bool grad = MODE == kColGrad || MODE == kColGradMove;
  double cv = 0.0;
  if (j < cb.c1) {
    if constexpr (MODE == kColYCopy) {
      gmut(P->y)[j] = gconst(P->x)[j];
    } else if constexpr (MODE == kColClamp) {
      const float v = gconst(P->x)[j];
      gmut(P->x)[j] = v > 0.f ? v : 0.f;
    } else if constexpr (MODE == kColYMove) {
      const double b = P->st->step;
      gmut(P->y)[j] = (float)((double)gconst(P->y)[j] - b * (double)gconst(P->g)[j]);
    } else if (grad || !P->st->proj_scatter) {  // else the scatter sum updated x
      float t = 0.f;
      const int ts = grad ? gconst(P->gcol_tslot0)[j] : gconst(P->col_tslot0)[j];
      const int n = grad ? gconst(P->gcol_nch)[j] : gconst(P->col_nch)[j];
      for (int c = 0; c < n; ++c) t += gconst(P->tpart)[ts + c];
      if constexpr (grad) {
        if (P->cscale) t *= gconst(P->cscale)[j];
        if constexpr (MODE == kColGradMove) {
          const double b = P->st->step;
          gmut(P->x)[j] = (float)((double)gconst(P->x)[j] - b * (double)gconst(P->g)[j]);
        }
        gmut(P->g)[j] = t;
        cv = (double)t * (double)t;
      } else {
        project_column<MODE>(P, j, t);
      }
    }
  }
  if constexpr (grad) {
    const double s = block_sum(cv, sh4);
    if (threadIdx.x == 0) gmut(P->gpart)[cb.slot] = s;
  }
}

// ------------------------------------------------------------ finalisation ----

// finalisation: one workgroup of 10 waves per plan; 640 threads is a multiple of the
// slot count and of the wave, which the coalesced slot sums below rely on
constexpr int kFinBlock = 640;
constexpr int kFinWaves = kFinBlock / kWave;
constexpr int kFinUnroll = 8;      // loads in flight per thread in the slot sums
constexpr int kCountCap = 16384;   // groups whose active-row counts are kept in LDS
static_assert(kFinBlock % kNPart == 0 && kFinBlock % kWave == 0, "slot sums");

__device__ __forceinline__ int seg_len(int n) { return (n + kFinBlock - 1) / kFinBlock; }

struct FinShared {
  double red[2][kFinBlock];  // per-thread sums of its two slots
  double slot[kNPart];       // the slot sums
};

// Slot-wise sums of n partial slots of kNPart doubles (kNPart even), read as one flat
// array of 16-byte pairs: thread t reads pairs t, t + kFinBlock, ... (consecutive
// threads read consecutive pairs, so a wave's load covers whole lines; every round
// issues kFinUnroll loads per thread, predicated at the end), and the two doubles of
// each of its pairs always belong to slots 2t mod kNPart and 2t + 1 mod kNPart.  The
// slots' thread sums are then added in a fixed tree, so the sums do not depend on
// timing.  With cnt, slot 7 (the groups' active-row counts, integers) is also kept in
// LDS by group.  Slots not in `used` read as 0, and threads whose two slots are both
// unused read nothing.  Every thread gets the result.
//
// The thread's two slot sums (loads and additions; no barrier, so the loads of
// several calls can be in flight together).
__device__ __forceinline__ void thread_slot_sums(const double* part_, int n, unsigned used,
                                                 int* cnt, double* s0, double* s1) {
  static_assert(kNPart % 2 == 0 && kNPart == 10, "pairs of slots; slot 7 is the odd one of 6, 7");
  const FO_GLOBAL v2d* part = (const FO_GLOBAL v2d*)gconst(part_);
  const int t = threadIdx.x;
  const int pairs = n * (kNPart / 2);
  const bool keep = cnt != nullptr && (2 * t) % kNPart == 6;
  // threads whose pair holds no slot in `used` (or slot 7 for cnt) read nothing
  const bool need = ((used >> ((2 * t) % kNPart)) & 3u) != 0 || keep;
  double a0 = 0.0, a1 = 0.0;
  for (int f = need ? t : pairs; f < pairs; f += kFinBlock * kFinUnroll) {
    v2d v[kFinUnroll];
#pragma unroll
    for (int u = 0; u < kFinUnroll; ++u) {
      const int i = f + kFinBlock * u;
      v[u] = i < pairs ? part[i] : v2d{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < kFinUnroll; ++u) {
      a0 += v[u].x;
      a1 += v[u].y;
      const int i = f + kFinBlock * u;
      if (keep && i < pairs) cnt[(2 * i + 1) / kNPart] = (int)v[u].y;
    }
  }
  *s0 = a0;
  *s1 = a1;
}

// The slot sums from every thread's two sums: wave k sums slot k.  Its thread sums
// are those of threads c + 5 m (2c = k rounded down to even; the first or second
// double of their pairs), m = 0 .. 127; lane l adds m = l and m = l + 64, then a fixed
// shuffle tree.
__device__ __forceinline__ void reduce_slots(double s0, double s1, unsigned used, FinShared* sh,
                                             double* out) {
  static_assert(kFinWaves == kNPart && kFinBlock / (kNPart / 2) == 2 * kWave, "slot waves");
  const int t = threadIdx.x;
  sh->red[0][t] = s0;
  sh->red[1][t] = s1;
  __syncthreads();
  {
    const int k = t / kWave, l = t & (kWave - 1);
    const int c = k / 2, h = k & 1;
    double r = 0.0;
    if (used & (1u << k))
      r = sh->red[h][c + (kNPart / 2) * l] + sh->red[h][c + (kNPart / 2) * (l + kWave)];
    r = wave_sum(r);
    if (l == 0) sh->slot[k] = r;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kNPart; ++k) out[k] = sh->slot[k];
  __syncthreads();
}

__device__ __forceinline__ void sum_slots(const double* part_, int n, double* out,
                                          unsigned used, FinShared* sh, int* cnt = nullptr) {
  double s0, s1;
  thread_slot_sums(part_, n, used, cnt, &s0, &s1);
  reduce_slots(s0, s1, used, sh, out);
}

// SUB: the objective and direction partials come from the objective-row view.
template <int MODE, int SUB>
__global__ __launch_bounds__(kFinBlock) void k_finalize(const DevPlan* __restrict__ plans) {
  __shared__ double sh4[kFinWaves];
  __shared__ FinShared shs;
  const DevPlan* __restrict__ P = plans + blockIdx.x;
  if (halted(P)) return;
  const int ng = SUB ? P->osell.n_groups : P->sell.n_groups;
  double a[kNPart];
  if constexpr (MODE == kFinDir0 || MODE == kFinDir) {
    // the three inputs' loads first, all in flight together, then the reductions
    double b[kNPart], b0, b1, a0 = 0.0, a1 = 0.0;
    thread_slot_sums(P->spart_b, ng, 0x21u, nullptr, &b0, &b1);
    if constexpr (MODE == kFinDir0) thread_slot_sums(P->spart_a, ng, 0x21u, nullptr, &a0, &a1);
    double g = 0.0;
    for (int i = threadIdx.x; i < P->n_col_blocks; i += kFinBlock) g += gconst(P->gpart)[i];
    reduce_slots(b0, b1, 0x21u, &shs, b);
    const double G = block_sum<kFinWaves>(g, sh4);
    if constexpr (MODE == kFinDir0) reduce_slots(a0, a1, 0x21u, &shs, a);
    if (threadIdx.x == 0) {
      DevState* st = P->st;
      if constexpr (MODE == kFinDir0) {
        st->cost = a[0];
        st->cost_y = a[0];
        st->pstop = 0;
        st->capped = 0;
        st->beta = 0.0;
        st->step = 0.0;
        if (a[5] > 0.0) st->nonfinite = 1;
      }
      if (b[5] > 0.0) st->nonfinite = 1;
      if (P->prm.objective == 0)
        decide_step(P, G, b[0]);
      else
        prepare_search(P, G, b[0]);
    }
  } else if constexpr (MODE == kFinMoveObj) {
    sum_slots(P->rpart, P->n_row_items, a, 0x21u, &shs);
    if (threadIdx.x == 0) {
      P->st->cost_y = a[0];
      if (a[5] > 0.0) P->st->nonfinite = 1;
    }
  } else if constexpr (MODE == kFinResidRows) {
    sum_slots(P->rpart, P->n_row_items, a, 0x3FFu, &shs);
    if (threadIdx.x == 0) {
      finalize_residuals(P, a);
      P->st->n_active = (int)a[7];
      P->st->active_entries = (int64_t)a[9];
      P->st->proj_scatter = 0;
    }
  } else {
    // the groups' active-row counts stay in LDS for the list offsets (plans of up to
    // kCountCap groups; larger ones read them again from the partials)
    __shared__ int cnt[kCountCap];
    const int n = P->sell.n_groups;
    const bool lds_cnt = n <= kCountCap;
    sum_slots(P->spart_a, n, a, 0x3FFu, &shs, lds_cnt ? cnt : nullptr);
    const int A = (int)a[7];
    // contributions are rounded to multiples of 1 / fx_scale; with every column
    // total bounded by a[8], 2^61 / a[8] keeps all sums far inside int64
    const double B = a[8];
    const bool scatter = P->n_scatter > 0 && A <= P->scatter_max_rows && B < 1e300;
    if (scatter) {
      // exclusive scan of the groups' active-row counts (list offsets), in group
      // order: each thread scans its segment of groups after one workgroup scan of
      // the segment totals
      __shared__ int sc[kFinWaves];
      const FO_GLOBAL double* part = gconst(P->spart_a);
      const int per = seg_len(n);
      const int i0 = threadIdx.x * per, i1 = min(n, i0 + per);
      auto count = [&](int i) {
        return lds_cnt ? cnt[i] : (int)part[(int64_t)i * kNPart + 7];
      };
      int own = 0;
      for (int i = i0; i < i1; ++i) own += count(i);
      int total;
      int off = block_scan<kFinWaves>(own, sc, &total);
      for (int i = i0; i < i1; ++i) {
        gmut(P->goff)[i] = off;
        off += count(i);
      }
    }
    if (threadIdx.x == 0) {
      finalize_residuals(P, a);
      P->st->n_active = A;
      P->st->active_entries = (int64_t)a[9];
      P->st->proj_scatter = scatter ? 1 : 0;
      P->st->fx_scale = B > 0.0 ? 0x1p61 / B : 1.0;
    }
  }
}

// Step search of Fig. 3 for the one-sided objective.  Along v the cost is only
// piecewise quadratic (an OAR term switches on or off where c l crosses its target),
// so the closed form does not apply: each window evaluates
// chi^2(y - beta v) - chi^2(y) in FP64 for kSearchWindow candidate exponents
// s0 + 1, s0 + 2, ... from the d, l, D g, L g the view's passes stored, and the first
// candidate that strictly lowers the cost is taken (Fig. 3's trials, in order); the
// next window follows while none does and alpha^s >= 1e-300.  The first window is
// summed by k_search_part over many workgroups (its per-workgroup sums added here in
// workgroup order); later windows, rarely needed, by this kernel's single workgroup.
// SUB: the objective-row view.
constexpr int kSearchBlocks = 64;  // workgroups per plan of the first window

// Workgroups of k_search_part for a view of n positions: what the plan's partial area
// holds, at least kBlock positions each.
__device__ __forceinline__ int search_blocks(const DevPlan* P, int n) {
  return max(1, min(min(kSearchBlocks, P->search_cap), (n + kBlock - 1) / kBlock));
}

// The row's terms of chi^2(y - beta_j v) - chi^2(y) for the window's candidates.
template <int SUB>
__device__ __forceinline__ void search_row(const DevPlan* __restrict__ P, int i, double vs,
                                           const double* bk, double* acc) {
  const FO_GLOBAL uint16_t* kind = gconst(SUB ? P->okind : P->kind);
  const unsigned k = kind[i];
  if (!(k & (kObjDose | kObjCdl))) return;
  const double c = P->prm.c;
  const double w = gconst(SUB ? P->owo : P->wo)[i];
  if (k & kObjDose) {  // w (e0 + beta Dv)^2 - w e0^2, e0 = Dhat - d
    const double e0 = (double)gconst(SUB ? P->odt : P->dt)[i] - (double)gconst(SUB ? P->od : P->d)[i];
    const double dv = (double)gconst(SUB ? P->odg : P->dg)[i] * vs;
#pragma unroll
    for (int j = 0; j < kSearchWindow; ++j) acc[j] += w * (bk[j] * dv) * (2.0 * e0 + bk[j] * dv);
  }
  if (k & kObjCdl) {   // w min(0, f0 + beta c Lv)^2 - w min(0, f0)^2
    const double f0 = (double)gconst(SUB ? P->oct : P->ct)[i] -
                      c * (double)gconst(SUB ? P->ol : P->l)[i];
    const double lv = c * (double)gconst(SUB ? P->olg : P->lg)[i] * vs;
    const double t0 = f0 < 0.0 ? f0 * f0 : 0.0;
#pragma unroll
    for (int j = 0; j < kSearchWindow; ++j) {
      const double fb = f0 + bk[j] * lv;
      acc[j] += w * ((fb < 0.0 ? fb * fb : 0.0) - t0);
    }
  }
}

// The first window's sums over a share of the rows: workgroup b of plan blockIdx.y
// takes positions b kBlock + t, stepping by the plan's workgroups times kBlock, and
// writes its kSearchWindow sums (waves in order) to the plan's partial area.
template <int SUB>
__global__ __launch_bounds__(kBlock) void k_search_part(const DevPlan* __restrict__ plans) {
  __shared__ double sh[kBlock / kWave][kSearchWindow];
  __shared__ double sbeta[kSearchWindow];
  const DevPlan* __restrict__ P = plans + blockIdx.y;
  if (halted(P)) return;
  const DevState* st = P->st;
  if (st->pstop) return;
  const SellView& V = SUB ? P->osell : P->sell;
  const int n = V.n_slices << (6 - V.lpr_log2);
  const int nb = search_blocks(P, n);
  if ((int)blockIdx.x >= nb) return;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const double vs = P->prm.unit_dir ? 1.0 / sqrt(st->G) : 1.0;  // v = vs g
  const int64_t base = st->s + 1;
  if (tid < kSearchWindow) sbeta[tid] = pow(P->prm.alpha, (double)(base + tid));
  __syncthreads();
  double bk[kSearchWindow], acc[kSearchWindow];
#pragma unroll
  for (int j = 0; j < kSearchWindow; ++j) {
    bk[j] = sbeta[j];
    acc[j] = 0.0;
  }
  for (int i = blockIdx.x * kBlock + tid; i < n; i += nb * kBlock) search_row<SUB>(P, i, vs, bk, acc);
#pragma unroll
  for (int j = 0; j < kSearchWindow; ++j) acc[j] = wave_sum(acc[j]);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < kSearchWindow; ++j) sh[wave][j] = acc[j];
  }
  __syncthreads();
  if (tid < kSearchWindow) {
    double r = 0.0;
    for (int v = 0; v < kBlock / kWave; ++v) r += sh[v][tid];
    gmut(P->spart_b)[(int64_t)blockIdx.x * kSearchWindow + tid] = r;
  }
}

template <int SUB>
__global__ __launch_bounds__(kFinBlock) void k_linesearch(const DevPlan* __restrict__ plans) {
  __shared__ double sh[kFinWaves][kSearchWindow];
  __shared__ double sbeta[kSearchWindow];
  __shared__ int s_pick;
  const DevPlan* __restrict__ P = plans + blockIdx.x;
  if (halted(P)) return;
  DevState* st = P->st;
  if (st->pstop) return;  // no descent direction this outer iteration
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const double vs = P->prm.unit_dir ? 1.0 / sqrt(st->G) : 1.0;  // v = vs g
  const double a = P->prm.alpha;
  const SellView& V = SUB ? P->osell : P->sell;
  const int n = V.n_slices << (6 - V.lpr_log2);
  const int64_t s0 = st->s;
  for (int64_t base = s0 + 1;; base += kSearchWindow) {
    if (tid < kSearchWindow) sbeta[tid] = pow(a, (double)(base + tid));
    __syncthreads();
    double bk[kSearchWindow];
#pragma unroll
    for (int j = 0; j < kSearchWindow; ++j) bk[j] = sbeta[j];
    if (base == s0 + 1) {
      // the first window: k_search_part's per-workgroup sums, in workgroup order
      const int nb = search_blocks(P, n);
      if (tid < kSearchWindow) {
        double r = 0.0;
        for (int b = 0; b < nb; ++b) r += gconst(P->spart_b)[(int64_t)b * kSearchWindow + tid];
        sh[0][tid] = r;
        for (int v = 1; v < kFinWaves; ++v) sh[v][tid] = 0.0;
      }
    } else {
      double acc[kSearchWindow];
#pragma unroll
      for (int j = 0; j < kSearchWindow; ++j) acc[j] = 0.0;
      for (int i = tid; i < n; i += kFinBlock) search_row<SUB>(P, i, vs, bk, acc);
#pragma unroll
      for (int j = 0; j < kSearchWindow; ++j) acc[j] = wave_sum(acc[j]);
      if (lane == 0) {
#pragma unroll
        for (int j = 0; j < kSearchWindow; ++j) sh[wave][j] = acc[j];
      }
    }
    __syncthreads();
    if (tid == 0) {
      int pick = -1;  // -1: none in this window, -2: beta below the floor first
      for (int j = 0; j < kSearchWindow && pick == -1; ++j) {
        if (bk[j] < kBetaFloor) {
          pick = -2;
          break;
        }
        double dchi = 0.0;
        for (int v = 0; v < kFinWaves; ++v) dchi += sh[v][j];
        if (!isfinite(dchi)) {
          st->nonfinite = 1;
          pick = -2;
        } else if (dchi < 0.0) {
          pick = j;
        }
      }
      s_pick = pick;
    }
    __syncthreads();
    const int pick = s_pick;
    if (pick != -1) {
      if (tid == 0) {
        if (pick >= 0) {
          st->s = base + pick;
          st->beta = bk[pick];
          st->step = bk[pick] * vs;
        } else {  // s unchanged, no perturbation (as a search that finds no step)
          st->beta = 0.0;
          st->step = 0.0;
          st->pstop = 1;
          st->capped = 1;
        }
      }
      return;
    }
    __syncthreads();  // sbeta and sh are rewritten by the next window
  }
}

// Band arrays before a robustness evaluation (min = encoded +inf, max = encoded
// -inf; a fill kernel, not a memset, so the sequence can be captured in a graph) and
// after it (decoded in place to floats).
__global__ __launch_bounds__(kBlock) void k_band_fill(int64_t n, uint32_t* lo, uint32_t* hi) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    lo[i] = band_enc(__uint_as_float(0x7F800000u));
    hi[i] = band_enc(__uint_as_float(0xFF800000u));
  }
}

__global__ __launch_bounds__(kBlock) void k_band_finish(int64_t n, uint32_t* lo, uint32_t* hi) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    lo[i] = __float_as_uint(band_dec(lo[i]));
    hi[i] = __float_as_uint(band_dec(hi[i]));
  }
}

// ---------------------------------------------------------------- launchers ----

template <int VT, int SUB>
static void launch_forward_vs(int mode, const DevPlan* plans, const FwdGroup* groups,
                              int n_groups, int grid, int lds_floats, uint32_t* ctr, int vsel,
                              hipStream_t s) {
  const size_t lds = (size_t)lds_floats * sizeof(float);
  switch (mode) {
    case kFwdDoseLet:
      k_forward<VT, kFwdDoseLet, SUB><<<grid, kFwdBlock, lds, s>>>(plans, groups, n_groups,
                                                                    lds_floats, ctr, vsel);
      break;
    case kFwdObj:
      k_forward<VT, kFwdObj, SUB><<<grid, kFwdBlock, lds, s>>>(plans, groups, n_groups,
                                                                lds_floats, ctr, vsel);
      break;
    case kFwdDir:
      k_forward<VT, kFwdDir, SUB><<<grid, kFwdBlock, lds, s>>>(plans, groups, n_groups,
                                                                lds_floats, ctr, vsel);
      break;
    default:
      k_forward<VT, kFwdResid, SUB><<<grid, kFwdBlock, lds, s>>>(plans, groups, n_groups,
                                                                  lds_floats, ctr, vsel);
      break;
  }
}

void launch_forward(int vtype, int mode, int sub, const DevPlan* plans, const FwdGroup* groups,
                    int n_groups, int grid, int lds_floats, uint32_t* ctr, int vsel,
                    hipStream_t s) {
  if (vtype == kF16I) {
    if (sub) launch_forward_vs<kF16I, 1>(mode, plans, groups, n_groups, grid, lds_floats, ctr, vsel, s);
    else launch_forward_vs<kF16I, 0>(mode, plans, groups, n_groups, grid, lds_floats, ctr, vsel, s);
  } else if (vtype == kBF16I) {
    if (sub) launch_forward_vs<kBF16I, 1>(mode, plans, groups, n_groups, grid, lds_floats, ctr, vsel, s);
    else launch_forward_vs<kBF16I, 0>(mode, plans, groups, n_groups, grid, lds_floats, ctr, vsel, s);
  } else if (vtype == kF16) {
    if (sub) launch_forward_vs<kF16, 1>(mode, plans, groups, n_groups, grid, lds_floats, ctr, vsel, s);
    else launch_forward_vs<kF16, 0>(mode, plans, groups, n_groups, grid, lds_floats, ctr, vsel, s);
  } else if (vtype == kBF16) {
    if (sub) launch_forward_vs<kBF16, 1>(mode, plans, groups, n_groups, grid, lds_floats, ctr, vsel, s);
    else launch_forward_vs<kBF16, 0>(mode, plans, groups, n_groups, grid, lds_floats, ctr, vsel, s);
  } else {
    if (sub) launch_forward_vs<kF32, 1>(mode, plans, groups, n_groups, grid, lds_floats, ctr, vsel, s);
    else launch_forward_vs<kF32, 0>(mode, plans, groups, n_groups, grid, lds_floats, ctr, vsel, s);
  }
}

void launch_rows(int mode, const DevPlan* plans, const RowItem* items, int n_items,
                 hipStream_t s) {
  if (mode == kRowsMoveObj)
    k_rows<kRowsMoveObj><<<n_items, kBlock, 0, s>>>(plans, items);
  else
    k_rows<kRowsMoveResid><<<n_items, kBlock, 0, s>>>(plans, items);
}

template <int TAG>
static void launch_tr_tag(int vtype, const DevPlan* plans, const TrItem* items, int n_items,
                          int grid, int nb8, int single, hipStream_t s) {
  vtype = value_of(vtype);  // the column-major copy keeps int32 row indices
  if (vtype == kF16)
    k_tr_chunks<kF16, TAG><<<grid, kBlock, 0, s>>>(plans, items, n_items, nb8, single);
  else if (vtype == kBF16)
    k_tr_chunks<kBF16, TAG><<<grid, kBlock, 0, s>>>(plans, items, n_items, nb8, single);
  else
    k_tr_chunks<kF32, TAG><<<grid, kBlock, 0, s>>>(plans, items, n_items, nb8, single);
}

void launch_tr_chunks(int vtype, int tag, const DevPlan* plans, const TrItem* items,
                      int n_items, int max_grid, int single, hipStream_t s) {
  if (n_items <= 0) return;  // no stored entries
  const int per = kBlock / kWave;
  const int nblocks = (n_items + per - 1) / per;
  const int nb8 = (nblocks + 7) / 8;
  const int cap = std::max(8, max_grid / 8 * 8);
  const int grid = std::min(nb8 * 8, cap);
  if (tag == 0)
    launch_tr_tag<0>(vtype, plans, items, n_items, grid, nb8, single, s);
  else
    launch_tr_tag<1>(vtype, plans, items, n_items, grid, nb8, single, s);
}

void launch_active_list(const DevPlan* plans, const FwdGroup* groups, int n_groups, int block,
                        hipStream_t s) {
  if (n_groups > 0) k_active_list<<<n_groups, block, 0, s>>>(plans, groups, n_groups);
}

void launch_scatter(int vtype, const DevPlan* plans, const ScItem* items, int n_items,
                    size_t lds_bytes, hipStream_t s) {
  if (n_items <= 0) return;
  if (vtype == kF16I)
    k_scatter<kF16I><<<n_items, kScatterBlock, lds_bytes, s>>>(plans, items);
  else if (vtype == kBF16I)
    k_scatter<kBF16I><<<n_items, kScatterBlock, lds_bytes, s>>>(plans, items);
  else if (vtype == kF16)
    k_scatter<kF16><<<n_items, kScatterBlock, lds_bytes, s>>>(plans, items);
  else if (vtype == kBF16)
    k_scatter<kBF16><<<n_items, kScatterBlock, lds_bytes, s>>>(plans, items);
  else
    k_scatter<kF32><<<n_items, kScatterBlock, lds_bytes, s>>>(plans, items);
}

void launch_project(int vtype, const DevPlan* plans, const ScItem* sc, int n_sc, size_t lds_bytes,
                    const TrItem* tr, int n_tr, int max_grid, int single, hipStream_t s) {
  // the chunk walk's virtual blocks of kScatterBlock / kWave items, grouped by 8
  constexpr int per = kScatterBlock / kWave;
  const int nb8 = n_tr > 0 ? ((n_tr + per - 1) / per + 7) / 8 : 0;
  const int walk = n_tr > 0 ? std::min(nb8 * 8, std::max(8, max_grid / 8 * 8)) : 0;
  const int grid = std::max(n_sc, walk);
  if (grid <= 0) return;
  switch (vtype) {
    case kF16I:
      k_project<kF16I, kF16><<<grid, kScatterBlock, lds_bytes, s>>>(plans, sc, n_sc, tr, n_tr, nb8, single);
      break;
    case kBF16I:
      k_project<kBF16I, kBF16><<<grid, kScatterBlock, lds_bytes, s>>>(plans, sc, n_sc, tr, n_tr, nb8, single);
      break;
    case kF16:
      k_project<kF16, kF16><<<grid, kScatterBlock, lds_bytes, s>>>(plans, sc, n_sc, tr, n_tr, nb8, single);
      break;
    case kBF16:
      k_project<kBF16, kBF16><<<grid, kScatterBlock, lds_bytes, s>>>(plans, sc, n_sc, tr, n_tr, nb8, single);
      break;
    default:
      k_project<kF32, kF32><<<grid, kScatterBlock, lds_bytes, s>>>(plans, sc, n_sc, tr, n_tr, nb8, single);
      break;
  }
}

hipError_t set_project_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
  for (const void* f : {(const void*)k_project<kF32, kF32>, (const void*)k_project<kF16, kF16>,
                        (const void*)k_project<kBF16, kBF16>, (const void*)k_project<kF16I, kF16>,
                        (const void*)k_project<kBF16I, kBF16>}) {
    const hipError_t r =
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (r != hipSuccess) e = r;
  }
  return e;
}

void launch_scatter_sum(int mode, const DevPlan* plans, const ScItem* items, int n_items,
                        hipStream_t s) {
  if (n_items <= 0) return;
  if (mode == kColProjNoClamp)
    k_scatter_sum<kColProjNoClamp><<<n_items, kScatterBlock, 0, s>>>(plans, items);
  else if (mode == kColProjYMove)
    k_scatter_sum<kColProjYMove><<<n_items, kScatterBlock, 0, s>>>(plans, items);
  else if (mode == kColProjY)
    k_scatter_sum<kColProjY><<<n_items, kScatterBlock, 0, s>>>(plans, items);
  else if (mode == kColProjMove)
    k_scatter_sum<kColProjMove><<<n_items, kScatterBlock, 0, s>>>(plans, items);
  else
    k_scatter_sum<kColProj><<<n_items, kScatterBlock, 0, s>>>(plans, items);
}

hipError_t set_scatter_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
  for (const void* f : {(const void*)k_scatter<kF32>, (const void*)k_scatter<kF16>,
                        (const void*)k_scatter<kBF16>, (const void*)k_scatter<kF16I>,
                        (const void*)k_scatter<kBF16I>}) {
    const hipError_t r =
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (r != hipSuccess) e = r;
  }
  return e;
}

void launch_tcol(int mode, const DevPlan* plans, const ColBlock* blocks, int n_blocks,
                 hipStream_t s) {
  switch (mode) {
    case kColGrad: k_tcol<kColGrad><<<n_blocks, kBlock, 0, s>>>(plans, blocks); break;
    case kColGradMove: k_tcol<kColGradMove><<<n_blocks, kBlock, 0, s>>>(plans, blocks); break;
    case kColProj: k_tcol<kColProj><<<n_blocks, kBlock, 0, s>>>(plans, blocks); break;
    case kColProjMove: k_tcol<kColProjMove><<<n_blocks, kBlock, 0, s>>>(plans, blocks); break;
    case kColProjY: k_tcol<kColProjY><<<n_blocks, kBlock, 0, s>>>(plans, blocks); break;
    case kColYMove: k_tcol<kColYMove><<<n_blocks, kBlock, 0, s>>>(plans, blocks); break;
    case kColClamp: k_tcol<kColClamp><<<n_blocks, kBlock, 0, s>>>(plans, blocks); break;
    default: k_tcol<kColYCopy><<<n_blocks, kBlock, 0, s>>>(plans, blocks); break;
  }
}

void launch_band(int finish, int64_t n, uint32_t* lo, uint32_t* hi, hipStream_t s) {
  if (n <= 0 || !lo) return;
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  if (finish)
    k_band_finish<<<grid, kBlock, 0, s>>>(n, lo, hi);
  else
    k_band_fill<<<grid, kBlock, 0, s>>>(n, lo, hi);
}

void launch_search_part(int sub, const DevPlan* plans, int n_plans, hipStream_t s) {
  if (n_plans <= 0) return;
  const dim3 grid(kSearchBlocks, n_plans);
  if (sub)
    k_search_part<1><<<grid, kBlock, 0, s>>>(plans);
  else
    k_search_part<0><<<grid, kBlock, 0, s>>>(plans);
}

void launch_linesearch(int sub, const DevPlan* plans, int n_plans, hipStream_t s) {
  if (n_plans <= 0) return;
  if (sub)
    k_linesearch<1><<<n_plans, kFinBlock, 0, s>>>(plans);
  else
    k_linesearch<0><<<n_plans, kFinBlock, 0, s>>>(plans);
}

void launch_finalize(int mode, int sub, const DevPlan* plans, int n_plans, hipStream_t s) {
  switch (mode) {
    case kFinDir0:
      if (sub) k_finalize<kFinDir0, 1><<<n_plans, kFinBlock, 0, s>>>(plans);
      else k_finalize<kFinDir0, 0><<<n_plans, kFinBlock, 0, s>>>(plans);
      break;
    case kFinDir:
      if (sub) k_finalize<kFinDir, 1><<<n_plans, kFinBlock, 0, s>>>(plans);
      else k_finalize<kFinDir, 0><<<n_plans, kFinBlock, 0, s>>>(plans);
      break;
    case kFinMoveObj: k_finalize<kFinMoveObj, 0><<<n_plans, kFinBlock, 0, s>>>(plans); break;
    case kFinResidRows: k_finalize<kFinResidRows, 0><<<n_plans, kFinBlock, 0, s>>>(plans); break;
    default: k_finalize<kFinResidFwd, 0><<<n_plans, kFinBlock, 0, s>>>(plans); break;
  }
}

template <int VT>
static hipError_t set_lds_vt(size_t bytes) {
  hipError_t e = hipSuccess;
  auto set = [&](const void* f) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (r != hipSuccess) e = r;
  };
  set((const void*)k_forward<VT, kFwdDoseLet, 0>);
  set((const void*)k_forward<VT, kFwdObj, 0>);
  set((const void*)k_forward<VT, kFwdDir, 0>);
  set((const void*)k_forward<VT, kFwdResid, 0>);
  set((const void*)k_forward<VT, kFwdDoseLet, 1>);
  set((const void*)k_forward<VT, kFwdObj, 1>);
  set((const void*)k_forward<VT, kFwdDir, 1>);
  set((const void*)k_forward<VT, kFwdResid, 1>);
  return e;
}

hipError_t set_forward_lds_limit(int vtype, size_t bytes) {
  if (vtype == kF16I) return set_lds_vt<kF16I>(bytes);
  if (vtype == kBF16I) return set_lds_vt<kBF16I>(bytes);
  if (vtype == kF16) return set_lds_vt<kF16>(bytes);
  if (vtype == kBF16) return set_lds_vt<kBF16>(bytes);
  return set_lds_vt<kF32>(bytes);
}

}  // namespace fo
