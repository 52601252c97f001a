// Evaluation kernels around the optimisation loop (Borys et al., arXiv 2509.20012,
// Sections 2.4.1 and 2.5): cumulative volume histograms of dose, LETd or cDL over a
// region of interest (the DVH / LVH / cDLVH of Figs. 4-5), and exact nearest-rank
// quantiles of a region's values (D95, D98, and the cDL30 that sets a percentile
// constraint from the forward calculation of a plan).
//
//  k_hist_fill / k_hist / k_hist_cumulate  integer counts per bin (LDS atomics, then
//               global atomics: exact and independent of the order of the additions),
//               then suffix sums: cum[b] = rows with value >= b vmax / n_bins.
//  k_quantile   radix selection over an order-preserving 32-bit encoding of the
//               floats, 8 bits per pass: after 4 passes the encoding of the value at
//               the requested rank is known exactly (equal to a sort's).
#include "fredopt_device.h"
#include "kernels.h"

#include <math.h>

namespace fo {

namespace {

constexpr int kEvalBlock = 1024;

// Order-preserving map of a float's bits to an unsigned integer (negative values
// below positive ones; a positive NaN above +inf).
__device__ __forceinline__ uint32_t enc(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float dec(uint32_t e) {
  return __uint_as_float((e & 0x80000000u) ? (e & 0x7FFFFFFFu) : ~e);
}

// The bin of value v: floor(v n_bins / vmax) in FP64, values at or above vmax in bin
// n_bins; -1 for values below 0 and NaN (counted in no bin).
__device__ __forceinline__ int bin_of(float v, double vmax, int n_bins) {
  if (!(v >= 0.f)) return -1;
  const double t = floor((double)v * (double)n_bins / vmax);
  return t >= (double)n_bins ? n_bins : (int)t;
}

__global__ __launch_bounds__(kEvalBlock) void k_hist_fill(uint32_t* cum, int n) {
  const int i = blockIdx.x * kEvalBlock + threadIdx.x;
  if (i < n) cum[i] = 0u;
}

// Rows outside [0, n_rows) are skipped (the caller's list is not trusted to stay in
// bounds).  The workgroup's counts gather in LDS, then go to the global array.
__global__ __launch_bounds__(kEvalBlock) void k_hist(const float* __restrict__ values,
                                                     int64_t n_rows,
                                                     const int32_t* __restrict__ rows, int64_t n,
                                                     double vmax, int n_bins, uint32_t* cum) {
  extern __shared__ uint32_t hist[];
  for (int b = threadIdx.x; b <= n_bins; b += kEvalBlock) hist[b] = 0u;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kEvalBlock) {
    const int32_t r = rows[i];
    if (r < 0 || (int64_t)r >= n_rows) continue;
    const int b = bin_of(values[r], vmax, n_bins);
    if (b >= 0) atomicAdd(&hist[b], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b <= n_bins; b += kEvalBlock)
    if (hist[b]) atomicAdd(&cum[b], hist[b]);
}

// In place: counts per bin to the number of rows at or above each bin's lower edge.
// One workgroup: each thread sums a contiguous run of bins, then the runs from the top.
__global__ __launch_bounds__(kEvalBlock) void k_hist_cumulate(uint32_t* cum, int n_bins) {
  __shared__ uint32_t run[kEvalBlock];
  const int n = n_bins + 1, per = (n + kEvalBlock - 1) / kEvalBlock;
  const int b0 = threadIdx.x * per, b1 = min(n, b0 + per);
  uint32_t s = 0;
  for (int b = b0; b < b1; ++b) s += cum[b];
  run[threadIdx.x] = s;
  __syncthreads();
  uint32_t above = 0;  // rows in the runs of the threads after this one
  for (int t = threadIdx.x + 1; t < kEvalBlock; ++t) above += run[t];
  for (int b = b1 - 1; b >= b0; --b) {
    above += cum[b];
    cum[b] = above;
  }
}

struct Ranks {
  int64_t r[kMaxQuantiles];  // 1-based ranks in ascending order
};

// One workgroup per requested rank: 4 passes of 8 bits, each a 256-bin histogram of
// the next digit among the values whose higher digits match the prefix found so far.
__global__ __launch_bounds__(kEvalBlock) void k_quantile(const float* __restrict__ values,
                                                         int64_t n_rows,
                                                         const int32_t* __restrict__ rows,
                                                         int64_t n, Ranks ranks, float* out) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t s_prefix, s_mask;
  __shared__ int64_t s_rank;
  if (threadIdx.x == 0) {
    s_prefix = 0u;
    s_mask = 0u;
    s_rank = ranks.r[blockIdx.x];
  }
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    for (int b = threadIdx.x; b < 256; b += kEvalBlock) hist[b] = 0u;
    __syncthreads();
    const uint32_t prefix = s_prefix, mask = s_mask;
    for (int64_t i = threadIdx.x; i < n; i += kEvalBlock) {
      const int32_t r = rows[i];
      if (r < 0 || (int64_t)r >= n_rows) continue;
      const uint32_t e = enc(values[r]);
      if ((e & mask) == prefix) atomicAdd(&hist[(e >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t rank = s_rank;
      int d = 0;
      for (; d < 255; ++d) {
        if ((int64_t)hist[d] >= rank) break;
        rank -= hist[d];
      }
      s_rank = rank;
      s_prefix = prefix | ((uint32_t)d << shift);
      s_mask = mask | (255u << shift);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = dec(s_prefix);
}

}  // namespace

void launch_volume_histogram(const float* values, int64_t n_rows, const int32_t* rows,
                             int64_t n, double vmax, int n_bins, uint32_t* cum, int n_cu,
                             hipStream_t s) {
  const int nb = n_bins + 1;
  k_hist_fill<<<(nb + kEvalBlock - 1) / kEvalBlock, kEvalBlock, 0, s>>>(cum, nb);
  if (n > 0) {
    const int64_t want = (n + kEvalBlock - 1) / kEvalBlock;
    const int grid = (int)std::min<int64_t>(want, (int64_t)std::max(n_cu, 1));
    k_hist<<<grid, kEvalBlock, sizeof(uint32_t) * nb, s>>>(values, n_rows, rows, n, vmax, n_bins,
                                                           cum);
  }
  k_hist_cumulate<<<1, kEvalBlock, 0, s>>>(cum, n_bins);
}

hipError_t set_histogram_lds_limit(size_t bytes) {
  return hipFuncSetAttribute((const void*)k_hist, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

void launch_quantiles(const float* values, int64_t n_rows, const int32_t* rows, int64_t n,
                      const int64_t* ranks, int n_q, float* out, hipStream_t s) {
  Ranks rk{};
  for (int k = 0; k < n_q; ++k) rk.r[k] = ranks[k];
  k_quantile<<<n_q, kEvalBlock, 0, s>>>(values, n_rows, rows, n, rk, out);
}

}  // namespace fo
