// stencil_bins.hip -- size binning of the stencil work.
//
// Targets are split by neighbour count N into bins: bin 0 holds targets with
// fewer sample rows than basis functions (rank deficient by construction);
// bin b >= 1 holds 64*(b-1) < N <= 64*b.  Each bin is a contiguous slice of
// one packed index list, filled with block-aggregated atomics; the per-bin
// stencil kernels are persistent and take targets from their slice through
// an atomic work counter (work stealing between waves).
#include <math.h>

#include "gmls_internal.hpp"

namespace gmls {

constexpr int kBinBlock = 256;

__device__ __forceinline__ int bin_of(int64_t n, int Q, int C) {
  if (n * C < Q) return 0;
  if (n > kMaxRows) return -1;
  return (int)((n + 63) / 64);
}

__global__ __launch_bounds__(kBinBlock) void k_bin_count(const int64_t *row_ptr, int n_tgt, int Q, int C,
                                                         BinMeta *meta) {
  __shared__ int cnt[kNumBins];
  if (threadIdx.x < kNumBins) cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_tgt; t += gridDim.x * blockDim.x) {
    const int b = bin_of(row_ptr[t + 1] - row_ptr[t], Q, C);
    if (b < 0)
      atomicOr(&meta->err, 1);
    else
      atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  if (threadIdx.x < kNumBins && cnt[threadIdx.x]) atomicAdd(&meta->count[threadIdx.x], cnt[threadIdx.x]);
}

__global__ void k_bin_offsets(BinMeta *meta) {
  if (threadIdx.x != 0) return;
  int acc = 0;
  for (int b = 0; b < kNumBins; ++b) {
    meta->offset[b] = acc;
    meta->cursor[b] = 0;
    acc += meta->count[b];
  }
}

// Block-aggregated scatter: one global atomic per bin per block, so each
// bin's slice keeps the blocks' target order (targets stay roughly in input
// order inside a bin).
__global__ __launch_bounds__(kBinBlock) void k_bin_scatter(const int64_t *row_ptr, int n_tgt, int Q, int C,
                                                           BinMeta *meta, int *list) {
  __shared__ int cnt[kNumBins];
  __shared__ int base[kNumBins];
  for (int t0 = blockIdx.x * blockDim.x; t0 < n_tgt; t0 += gridDim.x * blockDim.x) {
    if (threadIdx.x < kNumBins) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int t = t0 + threadIdx.x;
    int b = -1, pos = 0;
    if (t < n_tgt) {
      b = bin_of(row_ptr[t + 1] - row_ptr[t], Q, C);
      if (b >= 0) pos = atomicAdd(&cnt[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < kNumBins && cnt[threadIdx.x])
      base[threadIdx.x] = meta->offset[threadIdx.x] + atomicAdd(&meta->cursor[threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (b >= 0) list[base[b] + pos] = t;
    __syncthreads();
  }
}

__global__ void k_bin_reset(BinMeta *meta) {
  if (threadIdx.x != 0) return;
  for (int b = 0; b < kNumBins; ++b) meta->cursor[b] = 0;
  meta->fb_count = 0;
  meta->fb_cursor = 0;
}

hipError_t launch_binning(const int64_t *row_ptr, int n_tgt, int Q, int C, BinMeta *meta, int *list,
                          hipStream_t s) {
  int g = (n_tgt + kBinBlock - 1) / kBinBlock;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  hipError_t e = hipMemsetAsync(meta, 0, sizeof(BinMeta), s);
  if (e != hipSuccess) return e;
  k_bin_count<<<g, kBinBlock, 0, s>>>(row_ptr, n_tgt, Q, C, meta);
  k_bin_offsets<<<1, 64, 0, s>>>(meta);
  k_bin_scatter<<<g, kBinBlock, 0, s>>>(row_ptr, n_tgt, Q, C, meta, list);
  k_bin_reset<<<1, 64, 0, s>>>(meta);
  return hipGetLastError();
}

// Targets of bin 0: NaN weights, rank-deficient status.
__global__ void k_rank_deficient(StencilArgs a, int C, const int *list, const BinMeta *meta) {
  const int n = meta->count[0];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int t = list[meta->offset[0] + i];
    const int64_t base = a.row_ptr[t];
    const int64_t len = (a.row_ptr[t + 1] - base) * a.F * C;
    for (int64_t q = threadIdx.x; q < len; q += blockDim.x) a.weights[(int64_t)a.F * C * base + q] = NAN;
    if (threadIdx.x == 0) a.status[t] = GMLS_TARGET_RANK_DEFICIENT;
  }
}

hipError_t launch_rank_deficient(const StencilArgs &a, int C, const int *list, BinMeta *meta, hipStream_t s) {
  k_rank_deficient<<<256, 64, 0, s>>>(a, C, list, meta);
  return hipGetLastError();
}

}  // namespace gmls
