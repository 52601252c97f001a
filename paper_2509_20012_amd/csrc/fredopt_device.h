// Internal device-side layout shared by the HIP kernels and the host runtime of
// the fredopt library.  Nothing here is part of the public ABI (include/fredopt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fo {

constexpr int kBlock = 256;            // threads per workgroup of every iteration kernel
constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kNPart = 8;              // doubles per partial-sum slot
constexpr int kPlanTickets = 4;        // plan-level ticket counters before column tickets
constexpr double kDegenerateRel = 1e-12;
constexpr double kBetaFloor = 1e-300;

enum : unsigned {
  kDoseLo = 0x01u, kDoseHi = 0x02u, kCdlLo = 0x04u, kCdlHi = 0x08u, kLetdHi = 0x10u,
  kObjDose = 0x20u, kObjCdl = 0x40u, kConstraintBits = 0x1Fu
};

enum ValueType : int { kF32 = 0, kF16 = 1, kBF16 = 2 };

// forward-kernel epilogues
enum FwdMode : int { kFwdDoseLet = 0, kFwdObj = 1, kFwdDir = 2, kFwdResid = 3 };
// rows-kernel epilogues
enum RowMode : int { kRowsMoveObj = 0, kRowsMoveResid = 1 };
// transposed-kernel epilogues
enum TrMode : int { kTrGrad = 0, kTrGradMove = 1, kTrProj = 2, kTrProjMove = 3 };

struct DevParams {
  double lambda, alpha, eta, c;
  double ws_fixed;           // >= 0: weight scale used instead of eta^k
  int32_t normalization, reductions_n;
};

struct DevState {
  int64_t k, s, n_violated, n_degenerate;
  double beta, cost, cost_y, proximity, G, Q, w_all, w_viol, scale, ws;
  int32_t pstop, capped, nonfinite, pad;
};

struct DevPlan {
  int64_t R, C;
  int32_t vtype, lanes;       // value storage, lanes per row in the forward kernel
  int32_t n_fwd_items, n_row_items;
  // CSR, rows padded to a multiple of 4 slots
  const int64_t* rp;
  const int32_t* ci;
  const void* dv;
  const void* lv;
  // CSC, columns padded to a multiple of 4 slots, rows ascending in a column
  const int64_t* cp;
  const int32_t* ri;
  const void* cdv;
  const void* clv;
  const float* cscale;        // per-column scale of 16-bit storage (null for FP32)
  const double* mom;          // [3R] sum D^2, sum L^2, sum D L per row
  // problem (device arrays of R)
  const uint16_t* kind;
  const float *dlo, *dhi, *clo, *chi, *tmax, *wf, *wo, *dt, *ct;
  // vectors
  float* x;                   // fluence (caller's array during a call)
  float* d;
  float* l;
  float* dg;
  float* lg;
  float2* coef;               // per-row coefficients (dose part, LET part)
  float* g;
  float* out_dose;
  float* out_letd;
  float* out_cdl;
  // reductions
  double* fpart;              // [n_fwd_items * kNPart]
  double* rpart;              // [n_row_items * kNPart]
  float* tpart;               // [n_tr_items] chunk partials
  double* colval;             // [C]
  uint32_t* cnt;              // [kPlanTickets + C]
  DevParams prm;
  DevState* st;
};

struct FwdItem {   // a range of rows of one plan
  int32_t plan, slot, r0, r1;
};

struct RowItem {   // a range of rows of one plan (rows kernel)
  int32_t plan, slot, r0, r1;
};

struct TrItem {    // a chunk of one column of one plan
  int32_t plan, col, chunk, nchunks;
  int64_t q0, q1;  // slot range in the CSC arrays
  int32_t tslot0;  // tpart index of chunk 0 of this column
  int32_t pad;
};

}  // namespace fo
