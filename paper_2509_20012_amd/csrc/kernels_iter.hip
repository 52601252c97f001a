// Iteration kernels of the superiorized dose / LETd feasibility-seeking loop
// (Borys et al., arXiv 2509.20012, Figs. 2-3, Eq. 2) for gfx950.
//
//  k_forward     rows of D and L (CSR, rows padded to 4 slots, shared indices,
//                planar values) times a vector staged in LDS; one group of G lanes
//                per row, each lane streaming 4 slots per step with 16-byte loads,
//                butterfly shuffles for the row sum.  Epilogues: dose/LETd/cDL
//                (Eq. 1), Eq. (2) value and gradient coefficients, the direction
//                products with Q and the step-size decision, or the constraint
//                residuals of Fig. 2 folded into projection coefficients.
//  k_rows        moves d and l along the accepted perturbation and evaluates the
//                constraint residuals (or the next gradient coefficients).
//  k_transposed  columns of D^T and L^T (CSC, rows ascending) against the per-row
//                coefficient pair, chunked with fixed-order combination of chunk
//                partials (no floating-point atomics, so results are bitwise
//                reproducible); the epilogue writes the gradient, or applies the
//                projection, the pending perturbation and the x >= 0 clamp.
//
// Every plan-level scalar (cost, ||g||^2, Q, proximity, weights) is reduced in
// FP64: one partial slot per work item, then the last item of the plan (ticket
// counter) sums the slots in index order.
//
// Partial slot layout (kNPart doubles):
//   objective pass  [0] chi^2                         [5] non-finite rows
//   direction pass  [0] Q                             [5] non-finite rows
//   residual pass   [0] sum w (enabled) [1] sum w (violated) [2] sum w v^2/||a||^2
//                   [3] violated  [4] degenerate  [5] non-finite  [6] chi^2
#include "fredopt_device.h"
#include "kernels.h"

#include <math.h>

namespace fo {

template <int VT>
struct VLoad;

template <>
struct VLoad<kF32> {
  static __device__ __forceinline__ float4 q4(const void* p, int64_t q) {
    return *reinterpret_cast<const float4*>(static_cast<const float*>(p) + q);
  }
};

template <>
struct VLoad<kF16> {
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ float4 q4(const void* p, int64_t q) {
    const h4 h = *reinterpret_cast<const h4*>(static_cast<const _Float16*>(p) + q);
    return make_float4((float)h.x, (float)h.y, (float)h.z, (float)h.w);
  }
};

template <>
struct VLoad<kBF16> {
  static __device__ __forceinline__ float4 q4(const void* p, int64_t q) {
    const uint2 u = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(p) + q);
    return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                       __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
  }
};

// ------------------------------------------------------------------ reductions --

// Sum of v over the 256 threads in a fixed order (butterfly in each wave, then the
// four wave sums in order).  Every thread receives the result.
__device__ __forceinline__ double block_sum(double v, double* sh4) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int tid = threadIdx.x;
  __syncthreads();
  if ((tid & (kWave - 1)) == 0) sh4[tid / kWave] = v;
  __syncthreads();
  const double r = (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
  __syncthreads();
  return r;
}

// Sum of the plan's partial slots in a fixed order (thread-strided, then
// block_sum); run by the whole workgroup that took the last ticket.
__device__ __forceinline__ void sum_slots(const double* part, int n, double* out,
                                          double* sh4) {
  __threadfence();
  double s[kNPart];
#pragma unroll
  for (int k = 0; k < kNPart; ++k) s[k] = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const double* p = part + (int64_t)i * kNPart;
#pragma unroll
    for (int k = 0; k < kNPart; ++k) s[k] += __builtin_nontemporal_load(p + k);
  }
#pragma unroll
  for (int k = 0; k < kNPart; ++k) out[k] = block_sum(s[k], sh4);
}

// ---------------------------------------------------------------- epilogues ----

// Eq. (2) terms of row r at (d, l): adds the value to *chi and stores the gradient
// coefficients (-2 w (Dhat - d), -2 c w (cDLhat - c l)) of the row.
__device__ __forceinline__ void objective_row(const DevPlan* P, int r, float d, float l,
                                              double* chi) {
  const unsigned k = P->kind[r];
  double uD = 0.0, uL = 0.0;
  if (k & (kObjDose | kObjCdl)) {
    const double w = P->wo[r], c = P->prm.c;
    if (k & kObjDose) {
      const double e = (double)P->dt[r] - (double)d;
      *chi += w * e * e;
      uD = -2.0 * w * e;
    }
    if (k & kObjCdl) {
      const double f = (double)P->ct[r] - c * (double)l;
      *chi += w * f * f;
      uL = -2.0 * c * w * f;
    }
  }
  P->coef[r] = make_float2((float)uD, (float)uL);
}

__device__ __forceinline__ double objective_value(const DevPlan* P, int r, float d, float l) {
  const unsigned k = P->kind[r];
  double s = 0.0;
  if (k & (kObjDose | kObjCdl)) {
    const double w = P->wo[r], c = P->prm.c;
    if (k & kObjDose) {
      const double e = (double)P->dt[r] - (double)d;
      s += w * e * e;
    }
    if (k & kObjCdl) {
      const double f = (double)P->ct[r] - c * (double)l;
      s += w * f * f;
    }
  }
  return s;
}

// Fig. 2 at (d, l) for every enabled kind of row r: signed violation v (strict
// comparisons, equality is feasible), unscaled step lambda * w_i * v / ||a||^2
// folded into the (D, L) coefficient pair of the row.  ||a||^2 comes from the row
// moments: ||D_i||^2, c^2 ||L_i||^2, ||L_i - T D_i||^2 = sum L^2 - 2T sum DL +
// T^2 sum D^2.  Accumulates slots [0]..[4] of the residual layout.
__device__ __forceinline__ void residual_row(const DevPlan* P, int r, float d, float l,
                                             double* acc) {
  const unsigned k = P->kind[r];
  double kD = 0.0, kL = 0.0;
  if (k & kConstraintBits) {
    const double w = P->wf[r], lam = P->prm.lambda, c = P->prm.c;
    const double dd = d, ll = l;
    const double* m = P->mom + 3 * (int64_t)r;
    const double sdd = m[0], sll = m[1], sdl = m[2];
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
      const double b = P->dhi[r];
      if (dd > b) take(dd - b, sdd, sdd, 0, 0.0);
    }
    if (k & kDoseLo) {
      acc[0] += w;
      const double b = P->dlo[r];
      if (dd < b) take(dd - b, sdd, sdd, 0, 0.0);
    }
    if (k & kCdlHi) {
      acc[0] += w;
      const double b = P->chi[r], ax = c * ll;
      if (ax > b) take(ax - b, c * c * sll, c * c * sll, 1, 0.0);
    }
    if (k & kCdlLo) {
      acc[0] += w;
      const double b = P->clo[r], ax = c * ll;
      if (ax < b) take(ax - b, c * c * sll, c * c * sll, 1, 0.0);
    }
    if (k & kLetdHi) {
      acc[0] += w;
      const double T = P->tmax[r], ax = ll - T * dd;
      if (ax > 0.0) take(ax, sll - 2.0 * T * sdl + T * T * sdd, sll + T * T * sdd, 2, T);
    }
  }
  P->coef[r] = make_float2((float)kD, (float)kL);
}

__device__ __forceinline__ bool finite2(float a, float b) { return isfinite(a) && isfinite(b); }

// Plan-level completion of a residual pass: proximity, weights, the projection
// scale weight_scale / W, and the outer counter (Fig. 3: weights eta^k w).
__device__ void finalize_residuals(const DevPlan* P, const double* s) {
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

// Step decision of Fig. 3 on the device.  Along g the cost is quadratic:
// chi^2(y - beta g) - chi^2(y) = -beta G + beta^2 Q, so a trial beta = alpha^s
// strictly lowers it iff beta Q < G.  s is the smallest integer above the previous
// s with that property (the inner loop of Fig. 3 tries s+1, s+2, ...).  A search
// that would need alpha^s < 1e-300 skips the perturbation and leaves s unchanged.
__device__ void decide_step(const DevPlan* P, double Q) {
  DevState* st = P->st;
  st->Q = Q;
  const double G = st->G;
  if (!isfinite(G) || !isfinite(Q)) st->nonfinite = 1;
  if (st->pstop || !(G > 0.0) || !isfinite(G) || !isfinite(Q)) {
    st->beta = 0.0;
    st->pstop = 1;
    return;
  }
  const double a = P->prm.alpha;
  const int64_t s0 = st->s;
  auto ok = [&](int64_t s) { return pow(a, (double)s) * Q < G; };
  int64_t s = s0 + 1;
  if (!ok(s)) {
    // here Q > 0: a^s Q < G  <=>  s > log(G / Q) / log(a)
    const double est = log(G / Q) / log(a);
    if (!(est < 1e6)) {
      st->beta = 0.0;
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
    st->pstop = 1;
    st->capped = 1;
    return;
  }
  st->s = s;
  st->beta = beta;
}

// Writes this work item's partials, takes a ticket, and returns (to every thread)
// whether this item was the plan's last one.
__device__ __forceinline__ bool publish_partials(double* slot, const double* s, uint32_t* ticket,
                                                 int n_items, int* s_last) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kNPart; ++k) slot[k] = s[k];
    __threadfence();
    const unsigned t = atomicAdd(ticket, 1u);
    *s_last = (t == (unsigned)n_items - 1) ? 1 : 0;
  }
  __syncthreads();
  return *s_last != 0;
}

// -------------------------------------------------------------- forward pass ---

template <int VT, int MODE>
__global__ __launch_bounds__(kBlock) void k_forward(const DevPlan* __restrict__ plans,
                                                    const FwdItem* __restrict__ items,
                                                    int n_items, int lds_floats) {
  extern __shared__ float xs[];
  __shared__ double gred[kBlock / 4][kNPart];
  __shared__ double sh4[kBlock / kWave];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  int cur = -1;
  bool use_lds = false;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const FwdItem w = items[it];
    const DevPlan* __restrict__ P = plans + w.plan;
    const float* __restrict__ vec = (MODE == kFwdDir) ? P->g : P->x;
    const float* __restrict__ cs = P->cscale;
    if (w.plan != cur) {
      __syncthreads();
      use_lds = P->C <= (int64_t)lds_floats;
      if (use_lds) {
        for (int64_t j = tid; j < P->C; j += kBlock) xs[j] = cs ? vec[j] * cs[j] : vec[j];
      }
      __syncthreads();
      cur = w.plan;
    }
    const int G = P->lanes;
    const int NG = kBlock / G;
    const int gid = tid / G, gl = tid % G;
    double acc[kNPart];
#pragma unroll
    for (int k = 0; k < kNPart; ++k) acc[k] = 0.0;
    const int64_t* __restrict__ rp = P->rp;
    const int32_t* __restrict__ ci = P->ci;
    for (int r = w.r0 + gid; r < w.r1; r += NG) {
      const int64_t q0 = rp[r], q1 = rp[r + 1];
      float ad = 0.f, al = 0.f;
      if (use_lds) {
#pragma unroll 2
        for (int64_t q = q0 + 4 * gl; q < q1; q += 4 * G) {
          const int4 c4 = *reinterpret_cast<const int4*>(ci + q);
          const float4 d4 = VLoad<VT>::q4(P->dv, q);
          const float4 l4 = VLoad<VT>::q4(P->lv, q);
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
        for (int64_t q = q0 + 4 * gl; q < q1; q += 4 * G) {
          const int4 c4 = *reinterpret_cast<const int4*>(ci + q);
          const float4 d4 = VLoad<VT>::q4(P->dv, q);
          const float4 l4 = VLoad<VT>::q4(P->lv, q);
          const float x0 = cs ? vec[c4.x] * cs[c4.x] : vec[c4.x];
          const float x1 = cs ? vec[c4.y] * cs[c4.y] : vec[c4.y];
          const float x2 = cs ? vec[c4.z] * cs[c4.z] : vec[c4.z];
          const float x3 = cs ? vec[c4.w] * cs[c4.w] : vec[c4.w];
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
      for (int o = G >> 1; o > 0; o >>= 1) {
        ad += __shfl_xor(ad, o);
        al += __shfl_xor(al, o);
      }
      if (gl == 0) {
        if constexpr (MODE == kFwdDoseLet) {
          if (P->out_dose) P->out_dose[r] = ad;
          if (P->out_letd) P->out_letd[r] = ad > 0.f ? al / ad : 0.f;
          if (P->out_cdl) P->out_cdl[r] = (float)(P->prm.c * (double)al);
        } else if constexpr (MODE == kFwdObj) {
          P->d[r] = ad;
          P->l[r] = al;
          objective_row(P, r, ad, al, &acc[0]);
          if (!finite2(ad, al)) acc[5] += 1.0;
        } else if constexpr (MODE == kFwdDir) {
          P->dg[r] = ad;
          P->lg[r] = al;
          const unsigned k = P->kind[r];
          if (k & (kObjDose | kObjCdl)) {
            const double wo = P->wo[r], c = P->prm.c;
            if (k & kObjDose) acc[0] += wo * (double)ad * (double)ad;
            if (k & kObjCdl) acc[0] += wo * c * c * (double)al * (double)al;
          }
          if (!finite2(ad, al)) acc[5] += 1.0;
        } else {
          P->d[r] = ad;
          P->l[r] = al;
          residual_row(P, r, ad, al, acc);
          acc[6] += objective_value(P, r, ad, al);
          if (!finite2(ad, al)) acc[5] += 1.0;
        }
      }
    }
    if constexpr (MODE != kFwdDoseLet) {
      if (gl == 0) {
#pragma unroll
        for (int k = 0; k < kNPart; ++k) gred[gid][k] = acc[k];
      }
      __syncthreads();
      double s[kNPart];
#pragma unroll
      for (int k = 0; k < kNPart; ++k) s[k] = 0.0;
      if (tid == 0) {
        for (int g2 = 0; g2 < NG; ++g2)
#pragma unroll
          for (int k = 0; k < kNPart; ++k) s[k] += gred[g2][k];
      }
      if (publish_partials(P->fpart + (int64_t)w.slot * kNPart, s, &P->cnt[0],
                           P->n_fwd_items, &s_last)) {
        double tot[kNPart];
        sum_slots(P->fpart, P->n_fwd_items, tot, sh4);
        if (tid == 0) {
          DevState* st = P->st;
          if constexpr (MODE == kFwdObj) {
            st->cost = tot[0];
            st->cost_y = tot[0];
            st->pstop = 0;
            st->capped = 0;
            st->beta = 0.0;
            if (tot[5] > 0.0) st->nonfinite = 1;
          } else if constexpr (MODE == kFwdDir) {
            if (tot[5] > 0.0) st->nonfinite = 1;
            decide_step(P, tot[0]);
          } else {
            finalize_residuals(P, tot);
          }
          P->cnt[0] = 0u;
        }
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ rows pass --

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_rows(const DevPlan* __restrict__ plans,
                                                 const RowItem* __restrict__ items) {
  __shared__ double sh4[kBlock / kWave];
  __shared__ int s_last;
  const RowItem w = items[blockIdx.x];
  const DevPlan* __restrict__ P = plans + w.plan;
  const int tid = threadIdx.x;
  const double beta = P->st->beta;
  double acc[kNPart];
#pragma unroll
  for (int k = 0; k < kNPart; ++k) acc[k] = 0.0;
  for (int r = w.r0 + tid; r < w.r1; r += kBlock) {
    // the accepted perturbation y = x - beta g moves d and l by -beta (D g, L g)
    const float d = (float)((double)P->d[r] - beta * (double)P->dg[r]);
    const float l = (float)((double)P->l[r] - beta * (double)P->lg[r]);
    P->d[r] = d;
    P->l[r] = l;
    if constexpr (MODE == kRowsMoveObj) {
      objective_row(P, r, d, l, &acc[0]);
    } else {
      residual_row(P, r, d, l, acc);
      acc[6] += objective_value(P, r, d, l);
    }
    if (!finite2(d, l)) acc[5] += 1.0;
  }
  double s[kNPart];
#pragma unroll
  for (int k = 0; k < kNPart; ++k) s[k] = block_sum(acc[k], sh4);
  if (publish_partials(P->rpart + (int64_t)w.slot * kNPart, s, &P->cnt[1], P->n_row_items,
                       &s_last)) {
    double tot[kNPart];
    sum_slots(P->rpart, P->n_row_items, tot, sh4);
    if (tid == 0) {
      DevState* st = P->st;
      if constexpr (MODE == kRowsMoveObj) {
        st->cost_y = tot[0];
        if (tot[5] > 0.0) st->nonfinite = 1;
      } else {
        finalize_residuals(P, tot);
      }
      P->cnt[1] = 0u;
    }
  }
}

// ------------------------------------------------------------ transposed pass --

template <int MODE>
__device__ __forceinline__ void column_epilogue(const DevPlan* P, int col, float t) {
  if (P->cscale) t *= P->cscale[col];
  if constexpr (MODE == kTrGrad || MODE == kTrGradMove) {
    if constexpr (MODE == kTrGradMove) {
      const double b = P->st->beta;
      P->x[col] = (float)((double)P->x[col] - b * (double)P->g[col]);
    }
    P->g[col] = t;
    P->colval[col] = (double)t * (double)t;
  } else {
    double y = P->x[col];
    if constexpr (MODE == kTrProjMove) y -= P->st->beta * (double)P->g[col];
    const double xn = y - P->st->scale * (double)t;
    P->x[col] = xn > 0.0 ? (float)xn : 0.f;
  }
}

template <int VT, int MODE>
__global__ __launch_bounds__(kBlock) void k_transposed(const DevPlan* __restrict__ plans,
                                                       const TrItem* __restrict__ items) {
  __shared__ float wsum[kBlock / kWave];
  __shared__ double sh4[kBlock / kWave];
  __shared__ int s_fin, s_last;
  const TrItem w = items[blockIdx.x];
  const DevPlan* __restrict__ P = plans + w.plan;
  const int tid = threadIdx.x;
  const int32_t* __restrict__ ri = P->ri;
  const float2* __restrict__ cf = P->coef;
  float acc = 0.f;
#pragma unroll 2
  for (int64_t q = w.q0 + 4 * tid; q < w.q1; q += 4 * kBlock) {
    const int4 r4 = *reinterpret_cast<const int4*>(ri + q);
    const float4 d4 = VLoad<VT>::q4(P->cdv, q);
    const float4 l4 = VLoad<VT>::q4(P->clv, q);
    const float2 c0 = cf[r4.x], c1 = cf[r4.y], c2 = cf[r4.z], c3 = cf[r4.w];
    acc = fmaf(d4.x, c0.x, acc);
    acc = fmaf(l4.x, c0.y, acc);
    acc = fmaf(d4.y, c1.x, acc);
    acc = fmaf(l4.y, c1.y, acc);
    acc = fmaf(d4.z, c2.x, acc);
    acc = fmaf(l4.z, c2.y, acc);
    acc = fmaf(d4.w, c3.x, acc);
    acc = fmaf(l4.w, c3.y, acc);
  }
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((tid & (kWave - 1)) == 0) wsum[tid / kWave] = acc;
  __syncthreads();
  if (tid == 0) {
    float t = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    int fin = 1;
    if (w.nchunks > 1) {
      P->tpart[w.tslot0 + w.chunk] = t;
      __threadfence();
      const unsigned tk = atomicAdd(&P->cnt[kPlanTickets + w.col], 1u);
      fin = (tk == (unsigned)w.nchunks - 1) ? 1 : 0;
      if (fin) {
        __threadfence();
        t = 0.f;
        for (int c = 0; c < w.nchunks; ++c) t += __builtin_nontemporal_load(P->tpart + w.tslot0 + c);
        P->cnt[kPlanTickets + w.col] = 0u;
      }
    }
    if (fin) column_epilogue<MODE>(P, w.col, t);
    s_fin = fin;
  }
  if constexpr (MODE == kTrGrad || MODE == kTrGradMove) {
    __syncthreads();
    if (s_fin) {
      // plan-level ||g||^2: the finaliser of the plan's last column sums colval
      if (tid == 0) {
        __threadfence();
        const unsigned tk = atomicAdd(&P->cnt[2], 1u);
        s_last = (tk == (unsigned)P->C - 1) ? 1 : 0;
      }
      __syncthreads();
      if (s_last) {
        __threadfence();
        double s = 0.0;
        for (int64_t j = tid; j < P->C; j += kBlock) s += __builtin_nontemporal_load(P->colval + j);
        const double G = block_sum(s, sh4);
        if (tid == 0) {
          DevState* st = P->st;
          st->G = G;
          if (!isfinite(G)) st->nonfinite = 1;
          P->cnt[2] = 0u;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- launchers ----

template <int VT>
static void launch_forward_vt(int mode, const DevPlan* plans, const FwdItem* items,
                              int n_items, int grid, int lds_floats, hipStream_t s) {
  const size_t lds = (size_t)lds_floats * sizeof(float);
  switch (mode) {
    case kFwdDoseLet:
      k_forward<VT, kFwdDoseLet><<<grid, kBlock, lds, s>>>(plans, items, n_items, lds_floats);
      break;
    case kFwdObj:
      k_forward<VT, kFwdObj><<<grid, kBlock, lds, s>>>(plans, items, n_items, lds_floats);
      break;
    case kFwdDir:
      k_forward<VT, kFwdDir><<<grid, kBlock, lds, s>>>(plans, items, n_items, lds_floats);
      break;
    default:
      k_forward<VT, kFwdResid><<<grid, kBlock, lds, s>>>(plans, items, n_items, lds_floats);
      break;
  }
}

void launch_forward(int vtype, int mode, const DevPlan* plans, const FwdItem* items,
                    int n_items, int grid, int lds_floats, hipStream_t s) {
  if (vtype == kF16)
    launch_forward_vt<kF16>(mode, plans, items, n_items, grid, lds_floats, s);
  else if (vtype == kBF16)
    launch_forward_vt<kBF16>(mode, plans, items, n_items, grid, lds_floats, s);
  else
    launch_forward_vt<kF32>(mode, plans, items, n_items, grid, lds_floats, s);
}

void launch_rows(int mode, const DevPlan* plans, const RowItem* items, int n_items,
                 hipStream_t s) {
  if (mode == kRowsMoveObj)
    k_rows<kRowsMoveObj><<<n_items, kBlock, 0, s>>>(plans, items);
  else
    k_rows<kRowsMoveResid><<<n_items, kBlock, 0, s>>>(plans, items);
}

template <int VT>
static void launch_tr_vt(int mode, const DevPlan* plans, const TrItem* items, int n_items,
                         hipStream_t s) {
  switch (mode) {
    case kTrGrad: k_transposed<VT, kTrGrad><<<n_items, kBlock, 0, s>>>(plans, items); break;
    case kTrGradMove: k_transposed<VT, kTrGradMove><<<n_items, kBlock, 0, s>>>(plans, items); break;
    case kTrProj: k_transposed<VT, kTrProj><<<n_items, kBlock, 0, s>>>(plans, items); break;
    default: k_transposed<VT, kTrProjMove><<<n_items, kBlock, 0, s>>>(plans, items); break;
  }
}

void launch_transposed(int vtype, int mode, const DevPlan* plans, const TrItem* items,
                       int n_items, hipStream_t s) {
  if (vtype == kF16)
    launch_tr_vt<kF16>(mode, plans, items, n_items, s);
  else if (vtype == kBF16)
    launch_tr_vt<kBF16>(mode, plans, items, n_items, s);
  else
    launch_tr_vt<kF32>(mode, plans, items, n_items, s);
}

hipError_t set_forward_lds_limit(int vtype, size_t bytes) {
  hipError_t e = hipSuccess;
  auto set = [&](const void* f) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (r != hipSuccess) e = r;
  };
  if (vtype == kF16) {
    set((const void*)k_forward<kF16, kFwdDoseLet>);
    set((const void*)k_forward<kF16, kFwdObj>);
    set((const void*)k_forward<kF16, kFwdDir>);
    set((const void*)k_forward<kF16, kFwdResid>);
  } else if (vtype == kBF16) {
    set((const void*)k_forward<kBF16, kFwdDoseLet>);
    set((const void*)k_forward<kBF16, kFwdObj>);
    set((const void*)k_forward<kBF16, kFwdDir>);
    set((const void*)k_forward<kBF16, kFwdResid>);
  } else {
    set((const void*)k_forward<kF32, kFwdDoseLet>);
    set((const void*)k_forward<kF32, kFwdObj>);
    set((const void*)k_forward<kF32, kFwdDir>);
    set((const void*)k_forward<kF32, kFwdResid>);
  }
  return e;
}

}  // namespace fo
