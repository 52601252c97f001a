// Host-side launchers of the fredopt HIP kernels (internal).
#pragma once

#include "fredopt_device.h"

namespace fo {

// iteration kernels (kernels_iter.hip)
// sub: 0 all-row view, 1 objective-row view; vsel: VecSel
void launch_forward(int vtype, int mode, int sub, const DevPlan* plans, const FwdGroup* groups,
                    int n_groups, int grid, int lds_floats, uint32_t* ctr, int vsel,
                    hipStream_t s);
void launch_rows(int mode, const DevPlan* plans, const RowItem* items, int n_items,
                 hipStream_t s);
// persistent grid of at most max_grid workgroups; single: every item is plans[0]'s
void launch_tr_chunks(int vtype, int tag, const DevPlan* plans, const TrItem* items,
                      int n_items, int max_grid, int single, hipStream_t s);
void launch_tcol(int mode, const DevPlan* plans, const ColBlock* blocks, int n_blocks,
                 hipStream_t s);
void launch_finalize(int mode, int sub, const DevPlan* plans, int n_plans, hipStream_t s);
// band arrays of a robustness evaluation: fill (finish 0) or decode (finish 1)
void launch_band(int finish, int64_t n, uint32_t* lo, uint32_t* hi, hipStream_t s);
// step search of the one-sided objective, one workgroup per plan (sub: objective view)
// The one-sided step search's first window summed by many workgroups per plan.
void launch_search_part(int sub, const DevPlan* plans, int n_plans, hipStream_t s);
void launch_linesearch(int sub, const DevPlan* plans, int n_plans, hipStream_t s);
hipError_t set_forward_lds_limit(int vtype, size_t bytes);
void launch_active_list(const DevPlan* plans, const FwdGroup* groups, int n_groups, int block,
                        hipStream_t s);
// one workgroup per item: items[i] = {plan, share}; lds_bytes = 8 x the widest plan's C
void launch_scatter(int vtype, const DevPlan* plans, const ScItem* items, int n_items,
                    size_t lds_bytes, hipStream_t s);
hipError_t set_scatter_lds_limit(size_t bytes);
// The sweep's transposed product by the path each plan's device state chose: the
// active-row scatter shares and the column-major chunk walk in one launch (grid: the
// larger of n_sc and the walk's, which max_grid caps in workgroups of kScatterBlock).
void launch_project(int vtype, const DevPlan* plans, const ScItem* sc, int n_sc, size_t lds_bytes,
                    const TrItem* tr, int n_tr, int max_grid, int single, hipStream_t s);
hipError_t set_project_lds_limit(size_t bytes);
// mode: the ColMode of the projection update (kColProj, kColProjMove, kColProjY,
// kColProjYMove)
// items[i] = {plan, 64-column word}
void launch_scatter_sum(int mode, const DevPlan* plans, const ScItem* items, int n_items,
                        hipStream_t s);

// evaluation kernels (kernels_eval.hip)
// cum[b], b = 0..n_bins: rows of the list with value >= b vmax / n_bins (last bin: >= vmax)
void launch_volume_histogram(const float* values, int64_t n_rows, const int32_t* rows,
                             int64_t n, double vmax, int n_bins, uint32_t* cum, int n_cu,
                             hipStream_t s);
hipError_t set_histogram_lds_limit(size_t bytes);
// out[k]: the value at 1-based rank ranks[k] of the list's values in ascending order
void launch_quantiles(const float* values, int64_t n_rows, const int32_t* rows, int64_t n,
                      const int64_t* ranks, int n_q, float* out, hipStream_t s);

// load kernels (kernels_load.hip)
// flags bits: 1 column index out of range, 2 columns not strictly increasing,
//             4 non-finite or negative value
void launch_validate(int64_t R, int64_t C, const int64_t* row_ptr, const int32_t* col,
                     const float* dv, const float* lv, uint32_t* flags, hipStream_t s);
void launch_col_stats(int64_t nnz, const int64_t* row_ptr, const int32_t* col, const float* dv,
                      const float* lv, uint32_t* col_count, uint32_t* col_max_bits,
                      hipStream_t s);
void launch_col_scale(int64_t C, const uint32_t* col_max_bits, float* scale, hipStream_t s);
// vtype: value type (kF32, kF16, kBF16); idx16: column indices stored as uint16
void launch_pack_sell(int vtype, int64_t R, int lpr_log2, const int64_t* row_ptr,
                      const int32_t* col, const float* dv, const float* lv, const float* scale,
                      const int32_t* rslice, const int64_t* sbase, void* sci, int idx16,
                      void* sdv, void* slv, hipStream_t s);
// row-contiguous copy of every row at its position (active-row scatter); plen gets
// the rows' entry counts
void launch_pack_rows(int vtype, int64_t R, const int64_t* row_ptr, const int32_t* col,
                      const float* dv, const float* lv, const float* scale,
                      const int32_t* rslice, const int64_t* rptr, void* rci, int idx16,
                      void* rdv, void* rlv, int32_t* plen, hipStream_t s);
void launch_block_count(int64_t R, int64_t C, int rows_per_block, const int64_t* row_ptr,
                        const int32_t* col, uint32_t* bc, hipStream_t s);
void launch_block_offsets(int64_t C, int nb, const int64_t* cp, uint32_t* bc, hipStream_t s);
// rows ascending within each column; ri holds row indices
void launch_fill_csc(int vtype, int64_t R, int64_t C, int rows_per_block,
                     const int64_t* row_ptr, const int32_t* col, const float* dv,
                     const float* lv, const float* scale, uint32_t* bc, int32_t* ri, void* cdv,
                     void* clv, hipStream_t s);
// mom: sum D^2, sum L^2, sum D L per row; rsum: sum of the stored D and L values
// written at the rows' positions rslice[row]
void launch_moments(int vtype, int64_t R, const int64_t* row_ptr, const int32_t* col,
                    const float* dv, const float* lv, const float* scale, const int32_t* rslice,
                    double* mom, float* rsum, hipStream_t s);
// count[j]: entries of column j (len[j] real entries from cp[j]) in rows with
// objective terms.
void launch_obj_count(int64_t C, const int64_t* cp, const uint32_t* len, const int32_t* ri,
                      const uint16_t* kind, uint32_t* count, hipStream_t s);
// kind in row order
void launch_obj_fill(int vtype, int64_t C, const int64_t* cp, const uint32_t* len,
                     const int32_t* ri, const void* cdv, const void* clv, const uint16_t* kind,
                     const int64_t* ocp, int32_t* ori, void* ocdv,
                     void* oclv, hipStream_t s);
// copies the objective rows' entries from the all-row sliced-ELL view into the
// objective-row view: row obj_row[i] sits at slice position src_pos[i] of the full
// view and dst_pos[i] of the objective view and has len[i] entries
void launch_pack_sub(int vtype, int src_lg2, int dst_lg2, int64_t n, const int32_t* src_pos,
                     const int32_t* dst_pos, const int32_t* len, const int64_t* src_base,
                     const void* src_ci, const void* src_dv, const void* src_lv,
                     const int64_t* dst_base, void* dst_ci, int idx16, void* dst_dv,
                     void* dst_lv, hipStream_t s);
struct GatherArrays {  // kind and up to 9 float arrays of a problem
  uint16_t* kind;
  float* f[9];
};
void launch_gather_problem(int64_t n, const int32_t* pos_row, const GatherArrays& src,
                           const GatherArrays& dst, int nf, hipStream_t s);
void launch_check_problem(int64_t R, const uint16_t* kind, const float* dlo, const float* dhi,
                          const float* clo, const float* chi, const float* tmax,
                          const float* wf, const float* wo, const float* dt, const float* ct,
                          uint32_t* flags, hipStream_t s);

}  // namespace fo
