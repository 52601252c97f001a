// Host-side launchers of the fredopt HIP kernels (internal).
#pragma once

#include "fredopt_device.h"

namespace fo {

// iteration kernels (kernels_iter.hip)
void launch_forward(int vtype, int mode, const DevPlan* plans, const FwdItem* items,
                    int n_items, int grid, int lds_floats, hipStream_t s);
void launch_rows(int mode, const DevPlan* plans, const RowItem* items, int n_items,
                 hipStream_t s);
void launch_transposed(int vtype, int mode, const DevPlan* plans, const TrItem* items,
                       int n_items, hipStream_t s);
hipError_t set_forward_lds_limit(int vtype, size_t bytes);

// load kernels (kernels_load.hip)
// flags bits: 1 column index out of range, 2 columns not strictly increasing,
//             4 non-finite or negative value
void launch_validate(int64_t R, int64_t C, const int64_t* row_ptr, const int32_t* col,
                     const float* dv, const float* lv, uint32_t* flags, hipStream_t s);
void launch_col_stats(int64_t R, const int64_t* row_ptr, const int32_t* col, const float* dv,
                      const float* lv, uint32_t* col_count, uint32_t* col_max_bits,
                      hipStream_t s);
void launch_col_scale(int64_t C, const uint32_t* col_max_bits, float* scale, hipStream_t s);
void launch_pack_csr(int vtype, int64_t R, const int64_t* row_ptr, const int32_t* col,
                     const float* dv, const float* lv, const float* scale, const int64_t* rp,
                     int32_t* ci, void* pdv, void* plv, hipStream_t s);
void launch_block_count(int64_t R, int64_t C, int rows_per_block, const int64_t* row_ptr,
                        const int32_t* col, uint32_t* bc, hipStream_t s);
void launch_block_offsets(int64_t C, int nb, const int64_t* cp, uint32_t* bc, hipStream_t s);
void launch_fill_csc(int vtype, int64_t R, int64_t C, int rows_per_block,
                     const int64_t* row_ptr, const int32_t* col, const float* dv,
                     const float* lv, const float* scale, uint32_t* bc, int32_t* ri,
                     void* cdv, void* clv, hipStream_t s);
void launch_moments(int vtype, int64_t R, const int64_t* rp, const void* pdv, const void* plv,
                    const int32_t* ci, const float* scale, double* mom, hipStream_t s);
void launch_check_problem(int64_t R, const uint16_t* kind, const float* dlo, const float* dhi,
                          const float* clo, const float* chi, const float* tmax,
                          const float* wf, const float* wo, const float* dt, const float* ct,
                          uint32_t* flags, hipStream_t s);

}  // namespace fo
