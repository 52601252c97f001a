// Internal device-side layout shared by the HIP kernels and the host runtime of
// the fredopt library.  Nothing here is part of the public ABI (include/fredopt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Pointers read from a plan descriptor are generic; casting them to the global
// address space lets the compiler use global (not flat) loads, which do not share a
// wait counter with LDS traffic.
#define FO_GLOBAL __attribute__((address_space(1)))

namespace fo {

template <typename T>
__device__ __forceinline__ const FO_GLOBAL T* gconst(const T* p) {
  return (const FO_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ FO_GLOBAL T* gmut(T* p) {
  return (FO_GLOBAL T*)p;
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// native vector types (HIP's float4 & co. are classes and cannot live in a
// non-generic address space)
typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));
typedef double v2d __attribute__((ext_vector_type(2)));

constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kFwdBlock = 512;         // forward kernel: 8 waves, one slice each
constexpr int kFwdWaves = kFwdBlock / kWave;
constexpr int kBlock = 256;            // other kernels
constexpr int kScatterBlock = 1024;    // active-row scatter: 16 waves, one row each
constexpr int kScatterMaxWGs = 256;    // workgroups of the active-row scatter (max)
constexpr int kNPart = 10;             // doubles per partial-sum slot (slots 0-8 used)
constexpr int kCounters = 4;           // scheduling counters per batch
constexpr double kDegenerateRel = 1e-12;
constexpr double kBetaFloor = 1e-300;

enum : unsigned {
  kDoseLo = 0x01u, kDoseHi = 0x02u, kCdlLo = 0x04u, kCdlHi = 0x08u, kLetdHi = 0x10u,
  kObjDose = 0x20u, kObjCdl = 0x40u, kConstraintBits = 0x1Fu
};
constexpr int kSearchWindow = 16;      // candidate exponents per pass of the step search
constexpr int kMaxQuantiles = 16;      // ranks per quantile call
constexpr int kMaxHistBins = 32768;    // bins of a volume histogram (LDS counts)

// stored value type of a plan's matrices; kF16I / kBF16I also keep the column
// indices of the sliced-ELL copy in 16 bits (the column-major copy keeps int32 rows)
enum ValueType : int { kF32 = 0, kF16 = 1, kBF16 = 2, kF16I = 3, kBF16I = 4 };
__host__ __device__ constexpr int value_of(int vt) { return vt >= kF16I ? vt - 2 : vt; }
__host__ __device__ constexpr bool index16(int vt) { return vt >= kF16I; }

// forward-kernel epilogues
enum FwdMode : int { kFwdDoseLet = 0, kFwdObj = 1, kFwdDir = 2, kFwdResid = 3 };
// rows-kernel epilogues
enum RowMode : int { kRowsMoveObj = 0, kRowsMoveResid = 1 };
// column-finalise epilogues of the transposed product
enum ColMode : int {
  kColGrad = 0,      // g = sum
  kColGradMove = 1,  // x -= beta g (pending move), then g = sum
  kColProj = 2,      // x = max(0, x - scale sum)
  kColProjMove = 3,  // x = max(0, x - beta g - scale sum)
  kColProjY = 4,     // x = y = max(0, y - scale sum)
  kColYMove = 5,     // y -= beta g (no sum)
  kColYCopy = 6,     // y = x (no sum)
  kColProjYMove = 7, // x = y = max(0, y - beta g - scale sum)
  kColProjNoClamp = 8,  // x = x - scale sum (a block of a block-sequential sweep)
  kColClamp = 9      // x = max(0, x) (the end of a block-sequential sweep)
};
// which vector a forward pass multiplies
// kVecYMove: y - beta g, the perturbed point after the pending step (staged in LDS
// without writing y back)
enum VecSel : int { kVecX = 0, kVecY = 1, kVecG = 2, kVecYMove = 3 };
// plan-level finalisation
enum FinMode : int {
  kFinDir0 = 0,        // first perturbation of an outer iteration: cost, reset, step
  kFinDir = 1,         // later perturbations: step
  kFinMoveObj = 2,     // cost at the perturbed point (between perturbations)
  kFinResidRows = 3,   // residual pass done by the rows kernel
  kFinResidFwd = 4     // residual pass done by the forward kernel
};

struct DevParams {
  double lambda, alpha, eta, c;
  double ws_fixed;           // >= 0: weight scale used instead of eta^k
  int32_t normalization, reductions_n;
  int32_t objective;         // 0: Eq. (2) as printed, 1: one-sided OAR term
  int32_t unit_dir;          // 1: perturb along g / ||g||
};

struct DevState {
  int64_t k, s, n_violated, n_degenerate;
  double beta, cost, cost_y, proximity, G, Q, w_all, w_viol, scale, ws;
  double step;                // multiplier of g in the moves: beta, or beta / ||g||
  int32_t pstop, capped, nonfinite, pad;
  int32_t n_active;           // rows with a non-zero projection coefficient
  int32_t proj_scatter;       // 1: the projection uses the active-row scatter
  double fx_scale;            // fixed-point scale of the active-row scatter
  int64_t active_entries;     // stored entries of those rows (what the scatter reads)
};

// A row with a non-zero projection coefficient, as the scatter reads it: its
// entries in the row-contiguous copy.
struct ActRow {
  int64_t off;                // first slot of the row in the row-contiguous copy
  int32_t nq, len;            // quads (4 slots, the last one zero-padded); entries
  float cd, cl;               // projection coefficients (dose part, LET part)
  int32_t pad[2];
};

// Forward layout (sliced ELL): a slice holds rpw = 64 / lpr rows, each row spread
// over lpr lanes, each lane reading 4 consecutive entries of its row per step.  Entry
// e of the row in slice position p sits at
//   base[s] + ((e / 4) / lpr) * 256 + (p * lpr + (e / 4) % lpr) * 4 + e % 4
// so one wave step reads 1 KiB contiguously per array.  Rows are sorted by length
// (descending) inside windows of consecutive rows; srow maps slice positions back.
struct SellView {
  const int64_t* sbase;       // [n_slices + 1]
  const int32_t* swidth;      // [n_slices] steps
  const int32_t* srow;        // [n_slices * rpw] original row, -1 for padding
  const void* sci;            // int32, or uint16 for kF16I / kBF16I
  const void* sdv;
  const void* slv;
  int32_t n_slices, n_groups;
  int32_t lpr_log2, pad;      // lanes per row of this view (log2)
};

// Per-row data lives in slice-position order: the row at position sp = slice * rpw +
// place of the all-row view has its bounds, weights, moments, d, l and projection
// coefficients at index sp (padding positions hold kind 0 and zeros), so a slice's
// rows are read and written contiguously.  The objective-row view has its own
// positions for its objective terms.  The column-major copies keep row indices (a
// column's neighbouring entries are neighbouring voxels): the coefficients they
// gather are kept in row order (coef_row, gcoef).
struct DevPlan {
  int64_t R, C;
  int64_t NP;                 // positions of the all-row view (slices * rpw)
  int32_t vtype, lpr_log2;    // lanes per row (log2) of the all-row view
  int32_t n_row_items, n_col_blocks;
  int32_t search_cap;        // step-search partial sums the direction partial area holds
  int32_t search_pad;
  SellView sell;              // every row
  SellView osell;             // rows with objective terms (per problem), for Eq. (2)
  // CSC copy, columns padded to 4 slots, rows ascending in a column (projection)
  const int32_t* ri;
  const void* cdv;
  const void* clv;
  const int32_t* col_tslot0;  // [C] first chunk partial of the column
  const int32_t* col_nch;     // [C] chunks of the column
  // CSC used for the Eq. (2) gradient: only rows with objective terms (their
  // coefficients are the only non-zero ones), or the full CSC above
  const int32_t* gri;
  const void* gcdv;
  const void* gclv;
  const int32_t* gcol_tslot0;
  const int32_t* gcol_nch;
  // row-contiguous copy (active-row scatter): the row at position sp holds slots
  // [rptr[sp], rptr[sp + 1]), a multiple of 4, entries first, then zero padding
  const int64_t* rptr;        // [NP + 1]
  const int32_t* plen;        // [NP] entries of the row at each position
  const void* rci;            // int32, or uint16 for kF16I / kBF16I
  const void* rdv;
  const void* rlv;
  const float* cscale;        // per-column scale of 16-bit storage (null for FP32)
  const double* mom;          // [3 NP] sum D^2, sum L^2, sum D L per row
  const float* rsum;          // [2 NP] sum of the stored D and L values of a row
  // problem in position order (gathered from the caller's row-order arrays)
  const uint16_t* kind;
  const float *dlo, *dhi, *clo, *chi, *tmax, *wf, *wo, *dt, *ct;
  // objective terms in the objective-row view's position order
  const uint16_t* okind;
  const float *owo, *odt, *oct;
  float2* gcoef;              // [R] Eq. (2) gradient coefficients by row
  float2* coef_row;           // [R] projection coefficients by row (column-major path)
  // vectors
  float* x;                   // fluence (caller's array during a call)
  float* y;                   // perturbed point fed to the feasibility step
  float* d;
  float* l;
  float* dg;
  float* lg;
  float2* coef;               // per-position coefficients (dose part, LET part)
  float* g;
  // d, l at y and D g, L g of the objective-row view's rows (its positions), for the
  // step search of the one-sided objective
  float* od;
  float* ol;
  float* odg;
  float* olg;
  float* out_dose;
  float* out_letd;
  float* out_cdl;
  // per-voxel bands of a robustness evaluation (dose min, dose max, LETd min, LETd
  // max), order-preserving encoded floats; null outside such an evaluation
  uint32_t* band[4];
  // reductions
  double* spart_a;            // [groups * kNPart] objective / residual passes
  double* spart_b;            // [groups * kNPart] direction pass
  double* rpart;              // [n_row_items * kNPart]
  double* gpart;              // [n_col_blocks]
  float* tpart;               // [sum of chunks]
  // projection restricted to rows with non-zero coefficients
  int32_t* goff;              // [groups] first list position of each group's rows
  ActRow* alist;              // [NP] the active rows in slice order
  int64_t* spart;             // [n_scatter * C] per-workgroup fixed-point sums; with
                              // scatter_global, [C] column sums in global memory
  uint64_t* smask;            // [n_scatter * ceil(C / 64)] which of them are written
  int32_t n_scatter, scatter_max_rows;  // workgroups; largest list that uses it
  int32_t scatter_global;               // 1: the C column sums do not fit in LDS
  int32_t sc_lg2;                       // lanes per active row of the scatter (log2)
  DevParams prm;
  DevState* st;
};

struct FwdGroup {  // up to kFwdWaves consecutive slices of one plan
  int32_t plan, slice0, n, slot;  // slot: the group's partial-sum slot in its plan
};

struct RowItem {   // a range of rows of one plan (rows kernel)
  int32_t plan, slot, r0, r1;
};

struct TrItem {    // a chunk of one column of one plan
  int32_t plan, col;
  int32_t tslot, pad;
  int64_t q0, q1;  // slot range in the CSC arrays
};

struct ColBlock {  // up to kBlock consecutive columns of one plan
  int32_t plan, slot, c0, c1;
};

struct ScItem {    // a workgroup of the active-row scatter or of its share sum
  int32_t plan, idx;  // idx: the workgroup's share, or the 64-column word
};

}  // namespace fo
