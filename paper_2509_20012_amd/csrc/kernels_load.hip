// Load-time kernels: the device side of Table 2 step (iii) of Borys et al.
// (arXiv 2509.20012), loading the dose and LETd influence matrices.  They
// validate the CSR input, build the sliced-ELL copy used by the forward kernels,
// build the CSC copy (rows ascending inside every column, so the transposed
// products are deterministic) with a row-block counting sort, quantise values for
// 16-bit storage, and compute the per-row FP64 moments sum D^2, sum L^2, sum D L
// that give the projection denominators of Fig. 2.
#include "fredopt_device.h"
#include "kernels.h"

#include <math.h>

namespace fo {

namespace {

constexpr int kRowsPerWg = kBlock / kWave;  // one wavefront per row

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}

__device__ __forceinline__ void store_value(int vtype, void* base, int64_t pos, float v,
                                            float scale) {
  if (vtype == kF32) {
    static_cast<float*>(base)[pos] = v;
  } else if (vtype == kF16) {
    static_cast<_Float16*>(base)[pos] = (_Float16)(v / scale);
  } else {
    static_cast<uint16_t*>(base)[pos] = f32_to_bf16_rne(v / scale);
  }
}

// The value a 16-bit slot holds for input v with column scale sc, as a double.
__device__ __forceinline__ double stored_value(int vtype, float v, float sc) {
  if (vtype == kF16) return (double)(float)(_Float16)(v / sc);
  return (double)__uint_as_float((uint32_t)f32_to_bf16_rne(v / sc) << 16);
}

__global__ __launch_bounds__(kBlock) void k_validate(int64_t R, int64_t C,
                                                     const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col,
                                                     const float* __restrict__ dv,
                                                     const float* __restrict__ lv,
                                                     uint32_t* flags) {
  const int64_t row = (int64_t)blockIdx.x * kRowsPerWg + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (row >= R) return;
  const int64_t a = row_ptr[row], b = row_ptr[row + 1];
  uint32_t f = 0;
  for (int64_t k = a + lane; k < b; k += kWave) {
    const int32_t c = col[k];
    if (c < 0 || (int64_t)c >= C) f |= 1u;
    if (k > a && !(col[k - 1] < c)) f |= 2u;
    const float d = dv[k], l = lv[k];
    if (!isfinite(d) || !isfinite(l) || d < 0.f || l < 0.f) f |= 4u;
  }
  if (f) atomicOr(flags, f);
}

__global__ __launch_bounds__(kBlock) void k_col_stats(int64_t nnz, const int32_t* __restrict__ col,
                                                      const float* __restrict__ dv,
                                                      const float* __restrict__ lv,
                                                      uint32_t* col_count,
                                                      uint32_t* col_max_bits) {
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * kBlock) {
    const int32_t c = col[k];
    atomicAdd(&col_count[c], 1u);
    if (col_max_bits) {
      const float m = fmaxf(dv[k], lv[k]);  // both >= 0: bit patterns order like values
      atomicMax(&col_max_bits[c], __float_as_uint(m));
    }
  }
}

__global__ void k_col_scale(int64_t C, const uint32_t* __restrict__ bits, float* scale) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= C) return;
  const float m = __uint_as_float(bits[j]);
  scale[j] = m > 0.f ? m : 1.f;
}

// Sliced-ELL packing: every row is written by one wavefront into its slice position
// sp = slice * rpw + position (chosen on the host after the length sort).  Slots that
// no entry reaches keep the zero fill (index 0, value 0).
__global__ __launch_bounds__(kBlock) void k_pack_sell(int vtype, int64_t R, int lpr_log2,
                                                      const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col,
                                                      const float* __restrict__ dv,
                                                      const float* __restrict__ lv,
                                                      const float* __restrict__ scale,
                                                      const int32_t* __restrict__ rslice,
                                                      const int64_t* __restrict__ sbase,
                                                      void* sci, int idx16, void* sdv,
                                                      void* slv) {
  const int64_t row = (int64_t)blockIdx.x * kRowsPerWg + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (row >= R) return;
  const int rpw_log2 = 6 - lpr_log2;
  const int sp = rslice[row];
  const int64_t s = sp >> rpw_log2;
  const int p = sp & ((1 << rpw_log2) - 1);
  const int lpr = 1 << lpr_log2;
  const int64_t base = sbase[s];
  const int64_t a = row_ptr[row], n = row_ptr[row + 1] - a;
  for (int64_t e = lane; e < n; e += kWave) {
    const int64_t quad = e >> 2;
    const int64_t t = quad >> lpr_log2;
    const int64_t j = quad & (lpr - 1);
    const int64_t slot = base + t * 256 + ((int64_t)p * lpr + j) * 4 + (e & 3);
    const int32_t c = col[a + e];
    const float sc = scale ? scale[c] : 1.f;
    if (idx16)
      static_cast<uint16_t*>(sci)[slot] = (uint16_t)c;
    else
      static_cast<int32_t*>(sci)[slot] = c;
    store_value(vtype, sdv, slot, dv[a + e], sc);
    store_value(vtype, slv, slot, lv[a + e], sc);
  }
}

// Row-contiguous copy for the active-row scatter: the row at position sp = rslice[row]
// fills slots [rptr[sp], rptr[sp] + n) in column order (the remaining slots of the
// position, up to a multiple of 4, stay zero); plen[sp] = n.
__global__ __launch_bounds__(kBlock) void k_pack_rows(int vtype, int64_t R,
                                                      const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col,
                                                      const float* __restrict__ dv,
                                                      const float* __restrict__ lv,
                                                      const float* __restrict__ scale,
                                                      const int32_t* __restrict__ rslice,
                                                      const int64_t* __restrict__ rptr,
                                                      void* rci, int idx16, void* rdv,
                                                      void* rlv, int32_t* plen) {
  const int64_t row = (int64_t)blockIdx.x * kRowsPerWg + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (row >= R) return;
  const int sp = rslice[row];
  const int64_t base = rptr[sp];
  const int64_t a = row_ptr[row], n = row_ptr[row + 1] - a;
  if (lane == 0) plen[sp] = (int32_t)n;
  for (int64_t e = lane; e < n; e += kWave) {
    const int64_t slot = base + e;
    const int32_t c = col[a + e];
    const float sc = scale ? scale[c] : 1.f;
    if (idx16)
      static_cast<uint16_t*>(rci)[slot] = (uint16_t)c;
    else
      static_cast<int32_t*>(rci)[slot] = c;
    store_value(vtype, rdv, slot, dv[a + e], sc);
    store_value(vtype, rlv, slot, lv[a + e], sc);
  }
}

__global__ __launch_bounds__(kBlock) void k_block_count(int64_t R, int64_t C, int rows_per_block,
                                                        const int64_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col,
                                                        uint32_t* bc) {
  const int64_t row = (int64_t)blockIdx.x * kRowsPerWg + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (row >= R) return;
  const int64_t b = row / rows_per_block;
  uint32_t* base = bc + b * C;
  for (int64_t k = row_ptr[row] + lane; k < row_ptr[row + 1]; k += kWave)
    atomicAdd(&base[col[k]], 1u);
}

// counts per (row block, column) -> first CSC slot of that block inside the column
__global__ void k_block_offsets(int64_t C, int nb, const int64_t* __restrict__ cp, uint32_t* bc) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= C) return;
  uint32_t run = (uint32_t)cp[j];
  for (int b = 0; b < nb; ++b) {
    const uint32_t t = bc[(int64_t)b * C + j];
    bc[(int64_t)b * C + j] = run;
    run += t;
  }
}

// One workgroup per row block; its rows are visited in ascending order, the entries
// of one row in parallel (a row's columns are distinct, so no two lanes share a
// cursor), with a barrier between rows.  Inside every column the rows therefore come
// out ascending, independent of scheduling.
// One workgroup per block of rows, rows in order: within a column the entries end up
// in ascending row order (neighbouring voxels next to each other, which keeps the
// coefficient gathers of the transposed products local).
__global__ __launch_bounds__(kBlock) void k_fill_csc(int vtype, int64_t R, int64_t C,
                                                     int rows_per_block,
                                                     const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col,
                                                     const float* __restrict__ dv,
                                                     const float* __restrict__ lv,
                                                     const float* __restrict__ scale,
                                                     uint32_t* bc, int32_t* ri, void* cdv,
                                                     void* clv) {
  const int64_t b = blockIdx.x;
  const int64_t r0 = b * rows_per_block;
  int64_t r1 = r0 + rows_per_block;
  if (r1 > R) r1 = R;
  uint32_t* cur = bc + b * C;
  for (int64_t row = r0; row < r1; ++row) {
    for (int64_t k = row_ptr[row] + threadIdx.x; k < row_ptr[row + 1]; k += kBlock) {
      const int32_t c = col[k];
      const uint32_t pos = atomicAdd(&cur[c], 1u);
      const float s = scale ? scale[c] : 1.f;
      ri[pos] = (int32_t)row;
      store_value(vtype, cdv, pos, dv[k], s);
      store_value(vtype, clv, pos, lv[k], s);
    }
    __syncthreads();
  }
}

// Per-row FP64 moments sum D^2, sum L^2, sum D L of the values the kernels multiply
// (for 16-bit storage: the quantised value times the column scale), and the row sums
// of the stored values (rounded up: they bound the active-row scatter's sums).
__global__ __launch_bounds__(kBlock) void k_moments(int vtype, int64_t R,
                                                    const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col,
                                                    const float* __restrict__ dv,
                                                    const float* __restrict__ lv,
                                                    const float* __restrict__ scale,
                                                    const int32_t* __restrict__ rslice,
                                                    double* mom, float* rsum) {
  const int64_t row = (int64_t)blockIdx.x * kRowsPerWg + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (row >= R) return;
  double sdd = 0.0, sll = 0.0, sdl = 0.0, sd = 0.0, sl = 0.0;
  for (int64_t k = row_ptr[row] + lane; k < row_ptr[row + 1]; k += kWave) {
    double d = dv[k], l = lv[k];
    if (vtype != kF32) {
      const float sc = scale[col[k]];
      const double qd = stored_value(vtype, dv[k], sc), ql = stored_value(vtype, lv[k], sc);
      sd += qd;
      sl += ql;
      d = qd * (double)sc;
      l = ql * (double)sc;
    } else {
      sd += d;
      sl += l;
    }
    sdd += d * d;
    sll += l * l;
    sdl += d * l;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    sdd += __shfl_xor(sdd, o);
    sll += __shfl_xor(sll, o);
    sdl += __shfl_xor(sdl, o);
    sd += __shfl_xor(sd, o);
    sl += __shfl_xor(sl, o);
  }
  if (lane == 0) {
    const int64_t sp = rslice[row];
    mom[3 * sp] = sdd;
    mom[3 * sp + 1] = sll;
    mom[3 * sp + 2] = sdl;
    rsum[2 * sp] = __double2float_ru(sd);
    rsum[2 * sp + 1] = __double2float_ru(sl);
  }
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  // SplitMix64 finaliser (Steele, Lea, Flood 2014)
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// flags[0]: 1 non-finite bound/weight/target of an enabled kind, 2 lower > upper bound,
// 4 non-positive AMS weight or negative objective weight, 8 unknown kind bits.
// flags[2..3]: order-independent 64-bit fingerprint of the kind array (a sum of
// hashes of (row, kind) pairs), so per-problem preprocessing can be reused.
__global__ void k_check_problem(int64_t R, const uint16_t* __restrict__ kind,
                                const float* __restrict__ dlo, const float* __restrict__ dhi,
                                const float* __restrict__ clo, const float* __restrict__ chi,
                                const float* __restrict__ tmax, const float* __restrict__ wf,
                                const float* __restrict__ wo, const float* __restrict__ dt,
                                const float* __restrict__ ct, uint32_t* flags) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
       r += (int64_t)gridDim.x * blockDim.x) {
    const unsigned k = kind[r];
    uint32_t f = 0;
    if (k & ~0x7Fu) f |= 8u;
    if (k & kDoseLo && !isfinite(dlo[r])) f |= 1u;
    if (k & kDoseHi && !isfinite(dhi[r])) f |= 1u;
    if (k & kCdlLo && !isfinite(clo[r])) f |= 1u;
    if (k & kCdlHi && !isfinite(chi[r])) f |= 1u;
    if (k & kLetdHi && !isfinite(tmax[r])) f |= 1u;
    if ((k & (kDoseLo | kDoseHi)) == (kDoseLo | kDoseHi) && dlo[r] > dhi[r]) f |= 2u;
    if ((k & (kCdlLo | kCdlHi)) == (kCdlLo | kCdlHi) && clo[r] > chi[r]) f |= 2u;
    if (k & kConstraintBits) {
      const float w = wf[r];
      if (!isfinite(w) || !(w > 0.f)) f |= 4u;
    }
    if (k & (kObjDose | kObjCdl)) {
      const float w = wo[r];
      if (!isfinite(w) || w < 0.f) f |= 4u;
      if (k & kObjDose && !isfinite(dt[r])) f |= 1u;
      if (k & kObjCdl && !isfinite(ct[r])) f |= 1u;
    }
    if (f) atomicOr(flags, f);
    atomicAdd(reinterpret_cast<unsigned long long*>(flags + 2),
              (unsigned long long)mix64(((uint64_t)r << 16) | k));
  }
}

// Entries of column j whose row carries an objective term.
__global__ __launch_bounds__(kBlock) void k_obj_count(int64_t C, const int64_t* __restrict__ cp,
                                                      const uint32_t* __restrict__ len,
                                                      const int32_t* __restrict__ ri,
                                                      const uint16_t* __restrict__ kind,
                                                      uint32_t* count) {
  const int64_t j = (int64_t)blockIdx.x * kRowsPerWg + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (j >= C) return;
  uint32_t n = 0;
  // only the real entries of the column (padding slots hold row 0)
  for (int64_t k = cp[j] + lane; k < cp[j] + (int64_t)len[j]; k += kWave)
    n += (kind[ri[k]] & (kObjDose | kObjCdl)) ? 1u : 0u;
  for (int o = kWave / 2; o > 0; o >>= 1) n += __shfl_xor(n, o);
  if (lane == 0) count[j] = n;
}

// Order-preserving compaction of the objective-row entries of every column into
// the gradient CSC (one wavefront per column, ballot prefix sums per 64 entries).
__global__ __launch_bounds__(kBlock) void k_obj_fill(int vtype, int64_t C,
                                                     const int64_t* __restrict__ cp,
                                                     const uint32_t* __restrict__ len,
                                                     const int32_t* __restrict__ ri,
                                                     const void* __restrict__ cdv,
                                                     const void* __restrict__ clv,
                                                     const uint16_t* __restrict__ kind,
                                                     const int64_t* __restrict__ ocp,
                                                     int32_t* ori, void* ocdv, void* oclv) {
  const int64_t j = (int64_t)blockIdx.x * kRowsPerWg + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (j >= C) return;
  const int64_t a = cp[j], b = cp[j] + (int64_t)len[j];
  int64_t out = ocp[j];
  for (int64_t k0 = a; k0 < b; k0 += kWave) {
    const int64_t k = k0 + lane;
    const bool take = k < b && (kind[ri[k]] & (kObjDose | kObjCdl));
    const uint64_t m = __ballot(take);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (take) {
      const int64_t o = out + before;
      ori[o] = ri[k];
      if (vtype == kF32) {
        static_cast<float*>(ocdv)[o] = static_cast<const float*>(cdv)[k];
        static_cast<float*>(oclv)[o] = static_cast<const float*>(clv)[k];
      } else {
        static_cast<uint16_t*>(ocdv)[o] = static_cast<const uint16_t*>(cdv)[k];
        static_cast<uint16_t*>(oclv)[o] = static_cast<const uint16_t*>(clv)[k];
      }
    }
    out += __popcll(m);
  }
}

// Objective-row view: every listed row is copied by one wavefront from its slice
// position in the all-row view to its position in the objective-row view (values
// as stored).  Unreached slots keep the zero fill.
__global__ __launch_bounds__(kBlock) void k_pack_sub(int vtype, int src_lg2, int dst_lg2, int64_t n,
                                                     const int32_t* __restrict__ src_pos,
                                                     const int32_t* __restrict__ dst_pos,
                                                     const int32_t* __restrict__ len,
                                                     const int64_t* __restrict__ src_base,
                                                     const void* __restrict__ src_ci,
                                                     const void* __restrict__ src_dv,
                                                     const void* __restrict__ src_lv,
                                                     const int64_t* __restrict__ dst_base,
                                                     void* dst_ci, int idx16, void* dst_dv,
                                                     void* dst_lv) {
  const int64_t i = (int64_t)blockIdx.x * kRowsPerWg + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (i >= n) return;
  // the two views may spread a row over different lane counts
  const int srpw = 6 - src_lg2, drpw = 6 - dst_lg2;
  const int slpr = 1 << src_lg2, dlpr = 1 << dst_lg2;
  const int sp = src_pos[i], dp = dst_pos[i];
  const int64_t sb = src_base[sp >> srpw], db = dst_base[dp >> drpw];
  const int64_t spp = sp & ((1 << srpw) - 1), dpp = dp & ((1 << drpw) - 1);
  for (int64_t e = lane; e < len[i]; e += kWave) {
    const int64_t quad = e >> 2;
    const int64_t os = sb + (quad >> src_lg2) * 256 + (spp * slpr + (quad & (slpr - 1))) * 4 + (e & 3);
    const int64_t od = db + (quad >> dst_lg2) * 256 + (dpp * dlpr + (quad & (dlpr - 1))) * 4 + (e & 3);
    if (idx16)
      static_cast<uint16_t*>(dst_ci)[od] = static_cast<const uint16_t*>(src_ci)[os];
    else
      static_cast<int32_t*>(dst_ci)[od] = static_cast<const int32_t*>(src_ci)[os];
    if (vtype == kF32) {
      static_cast<float*>(dst_dv)[od] = static_cast<const float*>(src_dv)[os];
      static_cast<float*>(dst_lv)[od] = static_cast<const float*>(src_lv)[os];
    } else {
      static_cast<uint16_t*>(dst_dv)[od] = static_cast<const uint16_t*>(src_dv)[os];
      static_cast<uint16_t*>(dst_lv)[od] = static_cast<const uint16_t*>(src_lv)[os];
    }
  }
}

// Problem arrays from the caller's row order into a view's position order: position
// i takes row pos_row[i] (padding positions, row -1, get kind 0 and zeros).
__global__ __launch_bounds__(kBlock) void k_gather_problem(int64_t n,
                                                           const int32_t* __restrict__ pos_row,
                                                           GatherArrays src, GatherArrays dst,
                                                           int nf) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int row = pos_row[i];
  dst.kind[i] = row >= 0 ? src.kind[row] : (uint16_t)0;
  for (int f = 0; f < nf; ++f) dst.f[f][i] = row >= 0 ? src.f[f][row] : 0.f;
}

inline unsigned row_grid(int64_t R) { return (unsigned)((R + kRowsPerWg - 1) / kRowsPerWg); }

}  // namespace

void launch_validate(int64_t R, int64_t C, const int64_t* row_ptr, const int32_t* col,
                     const float* dv, const float* lv, uint32_t* flags, hipStream_t s) {
  if (R > 0) k_validate<<<row_grid(R), kBlock, 0, s>>>(R, C, row_ptr, col, dv, lv, flags);
}

void launch_col_stats(int64_t nnz, const int64_t* /*row_ptr*/, const int32_t* col,
                      const float* dv, const float* lv, uint32_t* col_count,
                      uint32_t* col_max_bits, hipStream_t s) {
  if (nnz <= 0) return;
  int64_t g = (nnz + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  k_col_stats<<<(unsigned)g, kBlock, 0, s>>>(nnz, col, dv, lv, col_count, col_max_bits);
}

void launch_col_scale(int64_t C, const uint32_t* bits, float* scale, hipStream_t s) {
  if (C > 0) k_col_scale<<<(unsigned)((C + 255) / 256), 256, 0, s>>>(C, bits, scale);
}

void launch_pack_sell(int vtype, int64_t R, int lpr_log2, const int64_t* row_ptr,
                      const int32_t* col, const float* dv, const float* lv, const float* scale,
                      const int32_t* rslice, const int64_t* sbase, void* sci, int idx16,
                      void* sdv, void* slv, hipStream_t s) {
  if (R > 0)
    k_pack_sell<<<row_grid(R), kBlock, 0, s>>>(vtype, R, lpr_log2, row_ptr, col, dv, lv, scale,
                                                rslice, sbase, sci, idx16, sdv, slv);
}

void launch_pack_rows(int vtype, int64_t R, const int64_t* row_ptr, const int32_t* col,
                      const float* dv, const float* lv, const float* scale,
                      const int32_t* rslice, const int64_t* rptr, void* rci, int idx16,
                      void* rdv, void* rlv, int32_t* plen, hipStream_t s) {
  if (R > 0)
    k_pack_rows<<<row_grid(R), kBlock, 0, s>>>(vtype, R, row_ptr, col, dv, lv, scale, rslice,
                                                rptr, rci, idx16, rdv, rlv, plen);
}

void launch_block_count(int64_t R, int64_t C, int rows_per_block, const int64_t* row_ptr,
                        const int32_t* col, uint32_t* bc, hipStream_t s) {
  if (R > 0)
    k_block_count<<<row_grid(R), kBlock, 0, s>>>(R, C, rows_per_block, row_ptr, col, bc);
}

void launch_block_offsets(int64_t C, int nb, const int64_t* cp, uint32_t* bc, hipStream_t s) {
  if (C > 0) k_block_offsets<<<(unsigned)((C + 255) / 256), 256, 0, s>>>(C, nb, cp, bc);
}

void launch_fill_csc(int vtype, int64_t R, int64_t C, int rows_per_block,
                     const int64_t* row_ptr, const int32_t* col, const float* dv,
                     const float* lv, const float* scale, uint32_t* bc, int32_t* ri, void* cdv,
                     void* clv, hipStream_t s) {
  if (R <= 0) return;
  const unsigned nb = (unsigned)((R + rows_per_block - 1) / rows_per_block);
  k_fill_csc<<<nb, kBlock, 0, s>>>(vtype, R, C, rows_per_block, row_ptr, col, dv, lv, scale, bc,
                                    ri, cdv, clv);
}

void launch_moments(int vtype, int64_t R, const int64_t* row_ptr, const int32_t* col,
                    const float* dv, const float* lv, const float* scale, const int32_t* rslice,
                    double* mom, float* rsum, hipStream_t s) {
  if (R > 0)
    k_moments<<<row_grid(R), kBlock, 0, s>>>(vtype, R, row_ptr, col, dv, lv, scale, rslice, mom,
                                             rsum);
}

void launch_obj_count(int64_t C, const int64_t* cp, const uint32_t* len, const int32_t* ri,
                      const uint16_t* kind, uint32_t* count, hipStream_t s) {
  if (C > 0) k_obj_count<<<row_grid(C), kBlock, 0, s>>>(C, cp, len, ri, kind, count);
}

void launch_obj_fill(int vtype, int64_t C, const int64_t* cp, const uint32_t* len,
                     const int32_t* ri, const void* cdv, const void* clv, const uint16_t* kind,
                     const int64_t* ocp, int32_t* ori, void* ocdv,
                     void* oclv, hipStream_t s) {
  if (C > 0)
    k_obj_fill<<<row_grid(C), kBlock, 0, s>>>(vtype, C, cp, len, ri, cdv, clv, kind, ocp,
                                               ori, ocdv, oclv);
}

void launch_pack_sub(int vtype, int src_lg2, int dst_lg2, int64_t n, const int32_t* src_pos,
                     const int32_t* dst_pos, const int32_t* len, const int64_t* src_base,
                     const void* src_ci, const void* src_dv, const void* src_lv,
                     const int64_t* dst_base, void* dst_ci, int idx16, void* dst_dv,
                     void* dst_lv, hipStream_t s) {
  if (n > 0)
    k_pack_sub<<<row_grid(n), kBlock, 0, s>>>(vtype, src_lg2, dst_lg2, n, src_pos, dst_pos, len,
                                               src_base, src_ci, src_dv, src_lv, dst_base, dst_ci,
                                               idx16, dst_dv, dst_lv);
}

void launch_gather_problem(int64_t n, const int32_t* pos_row, const GatherArrays& src,
                           const GatherArrays& dst, int nf, hipStream_t s) {
  if (n > 0)
    k_gather_problem<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(n, pos_row, src,
                                                                            dst, nf);
}

void launch_check_problem(int64_t R, const uint16_t* kind, const float* dlo, const float* dhi,
                          const float* clo, const float* chi, const float* tmax,
                          const float* wf, const float* wo, const float* dt, const float* ct,
                          uint32_t* flags, hipStream_t s) {
  if (R <= 0) return;
  int64_t g = (R + 255) / 256;
  if (g > 16384) g = 16384;
  k_check_problem<<<(unsigned)g, 256, 0, s>>>(R, kind, dlo, dhi, clo, chi, tmax, wf, wo, dt, ct,
                                               flags);
}

}  // namespace fo
