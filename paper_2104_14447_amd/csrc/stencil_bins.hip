// stencil_bins.hip -- size binning of the stencil work.
//
// Targets are split by neighbour count N into bins: bin 0 holds targets with
// fewer sample rows than basis functions (rank deficient by construction);
// bin b >= 1 holds 64*(b-1) < N <= 64*b.  Each bin is a contiguous slice of
// one packed index list.  Inside a bin the targets follow a Morton (Z-order)
// curve over the targets' bounding box: consecutive targets are spatial
// neighbours, so their neighbour rows overlap and the coordinate gathers of
// the stencil kernels hit in cache.  The list is the value array of one
// radix sort of (bin, Morton code) keys.
#include <float.h>
#include <math.h>

#include <hipcub/hipcub.hpp>

#include "common.hpp"
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

// ---- target bounding box (two stages) ----
constexpr int kBoxBlocks = 256;

__global__ __launch_bounds__(256) void k_tbox_partial(const double *x, int n, int dim, double *partial) {
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    for (int d = 0; d < dim; ++d) {
      const double v = x[(int64_t)t * dim + d];
      lo[d] = fmin(lo[d], v);
      hi[d] = fmax(hi[d], v);
    }
  __shared__ double sm[4][6];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int d = 0; d < 3; ++d) {
    const double a = wave_min(lo[d]), b = wave_max(hi[d]);
    if (lane == 0) {
      sm[wid][d] = a;
      sm[wid][3 + d] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = sm[0][threadIdx.x];
    for (int w = 1; w < 4; ++w) v = threadIdx.x < 3 ? fmin(v, sm[w][threadIdx.x]) : fmax(v, sm[w][threadIdx.x]);
    partial[blockIdx.x * 6 + threadIdx.x] = v;
  }
}

// one wave: reduce the partial boxes; box[0..2] = lo, box[3..5] = 1/extent
__global__ __launch_bounds__(64) void k_tbox_final(const double *partial, int nb, double *box) {
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  for (int b = threadIdx.x; b < nb; b += 64)
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], partial[b * 6 + d]);
      hi[d] = fmax(hi[d], partial[b * 6 + 3 + d]);
    }
  for (int d = 0; d < 3; ++d) {
    lo[d] = wave_min(lo[d]);
    hi[d] = wave_max(hi[d]);
  }
  if (threadIdx.x == 0)
    for (int d = 0; d < 3; ++d) {
      const double ext = hi[d] - lo[d];
      box[d] = lo[d];
      box[3 + d] = ext > 0 ? 1.0 / ext : 0.0;
    }
}

// spread the low 10 bits of v to every third bit
__device__ __forceinline__ unsigned spread3(unsigned v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// spread the low 13 bits of v to every second bit
__device__ __forceinline__ unsigned spread2(unsigned v) {
  v &= 0x1fffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

// grid coordinate of v on 2^bits cells over [lo, lo + 1/inv]
__device__ __forceinline__ unsigned quant(double v, double lo, double inv, int bits) {
  const double f = (v - lo) * inv * (double)(1 << bits);
  const double c = fmin(fmax(f, 0.0), (double)((1 << bits) - 1));
  return (unsigned)c;
}

// key = bin in bits 28-30 (7 for rows over the compiled maximum) | Morton
// code in bits 0-27 (3D: 9 bits per axis, 2D: 13, 1D: 26)
__global__ __launch_bounds__(256) void k_bin_keys(const int64_t *row_ptr, const double *x, int n_tgt, int dim,
                                                  int Q, int C, const double *box, BinMeta *meta, unsigned *key,
                                                  int *val) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_tgt; t += gridDim.x * blockDim.x) {
    int b = bin_of(row_ptr[t + 1] - row_ptr[t], Q, C);
    if (b < 0) b = 7;
    unsigned m;
    if (dim == 3)
      m = spread3(quant(x[(int64_t)t * 3], box[0], box[3], 9)) |
          (spread3(quant(x[(int64_t)t * 3 + 1], box[1], box[4], 9)) << 1) |
          (spread3(quant(x[(int64_t)t * 3 + 2], box[2], box[5], 9)) << 2);
    else if (dim == 2)
      m = spread2(quant(x[(int64_t)t * 2], box[0], box[3], 13)) |
          (spread2(quant(x[(int64_t)t * 2 + 1], box[1], box[4], 13)) << 1);
    else
      m = quant(x[t], box[0], box[3], 26);
    key[t] = ((unsigned)b << 28) | m;
    val[t] = t;
  }
}

__global__ void k_bin_reset(BinMeta *meta) {
  if (threadIdx.x != 0) return;
  for (int b = 0; b < kNumBins; ++b) meta->cursor[b] = 0;
  meta->fb_count = 0;
  meta->fb_cursor = 0;
}

static size_t sort_bytes(int n_tgt) {
  size_t bytes = 0;
  hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const unsigned *)nullptr, (unsigned *)nullptr,
                                     (const int *)nullptr, (int *)nullptr, n_tgt, 0, 31);
  return bytes;
}

// layout of the temporary buffer: partial boxes, box, keys in, keys out,
// values in, then the sort's own storage (256-byte aligned)
static size_t sort_offset(int n_tgt) {
  const size_t off = sizeof(double) * (6 * kBoxBlocks + 6) + (2 * sizeof(unsigned) + sizeof(int)) * (size_t)n_tgt;
  return (off + 255) & ~(size_t)255;
}

size_t binning_temp_bytes(int n_tgt) { return sort_offset(n_tgt) + sort_bytes(n_tgt); }

hipError_t launch_binning(const int64_t *row_ptr, const double *targets, int n_tgt, int dim, int Q, int C,
                          BinMeta *meta, int *list, void *temp, size_t temp_bytes, hipStream_t s) {
  int g = (n_tgt + kBinBlock - 1) / kBinBlock;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  if (temp_bytes < binning_temp_bytes(n_tgt)) return hipErrorInvalidValue;
  char *p = (char *)temp;
  double *partial = (double *)p;
  double *box = partial + 6 * kBoxBlocks;
  unsigned *kin = (unsigned *)(box + 6);
  unsigned *kout = kin + n_tgt;
  int *vin = (int *)(kout + n_tgt);
  size_t sb = temp_bytes - sort_offset(n_tgt);
  hipError_t e = hipMemsetAsync(meta, 0, sizeof(BinMeta), s);
  if (e != hipSuccess) return e;
  k_bin_count<<<g, kBinBlock, 0, s>>>(row_ptr, n_tgt, Q, C, meta);
  k_bin_offsets<<<1, 64, 0, s>>>(meta);
  k_tbox_partial<<<kBoxBlocks, 256, 0, s>>>(targets, n_tgt, dim, partial);
  k_tbox_final<<<1, 64, 0, s>>>(partial, kBoxBlocks, box);
  k_bin_keys<<<g, kBinBlock, 0, s>>>(row_ptr, targets, n_tgt, dim, Q, C, box, meta, kin, vin);
  e = hipcub::DeviceRadixSort::SortPairs((void *)(p + sort_offset(n_tgt)), sb, kin, kout, vin, list, n_tgt, 0, 31,
                                         s);
  if (e != hipSuccess) return e;
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
