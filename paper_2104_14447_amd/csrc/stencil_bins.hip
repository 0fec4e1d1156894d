// stencil_bins.hip -- size binning of the stencil work.
//
// Targets are split by neighbour count N into bins: bin 0 holds targets with
// fewer sample rows than basis functions (rank deficient by construction);
// bin b = 1..4 holds 64*(b-1) < N <= 64*b, bin 5 the longer rows (the
// kernels take those in chunks).  Each bin is a contiguous slice of
// one packed index list.  Inside a bin the targets follow a Morton (Z-order)
// curve of cells over the targets' bounding box: consecutive targets are
// spatial neighbours, so their neighbour rows overlap and the coordinate
// gathers of the stencil kernels hit in cache.  The list comes from one
// counting sort over (bin, Morton cell) buckets; the order inside a bucket
// (a few targets) is that of the atomic counter and does not affect any
// result.  No step waits for the host, and no buffer is cleared by a memset.
#include <float.h>
#include <math.h>

#include "common.hpp"
#include "gmls_internal.hpp"

namespace gmls {

constexpr int kBinBlock = 256;

__device__ __forceinline__ int bin_of(int64_t n, int Q, int C) {
  if (n * C < Q) return 0;
  if (n > kMaxRows) return -1;
  if (n > 256) return kLongBin;
  return (int)((n + 63) / 64);
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

constexpr int kCellBits = 18;                  // Morton cells per bin
constexpr int64_t kBuckets = 8ll << kCellBits;  // bins 0..7 (7: rows over the maximum)
static_assert(kNumBins <= 7, "bin 7 holds the rows over the maximum");

// bucket = bin << 18 | Morton cell (3D: 6 bits per axis, 2D: 9, 1D: 18);
// rank = the target's place in its bucket
__global__ __launch_bounds__(256) void k_bucket_rank(const int64_t *row_ptr, const double *x, int n_tgt, int dim,
                                                     int Q, int C, const double *box, int *cnt, int *bucket,
                                                     int *rank) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_tgt; t += gridDim.x * blockDim.x) {
    int b = bin_of(row_ptr[t + 1] - row_ptr[t], Q, C);
    if (b < 0) b = 7;
    unsigned m;
    if (dim == 3)
      m = spread3(quant(x[(int64_t)t * 3], box[0], box[3], 6)) |
          (spread3(quant(x[(int64_t)t * 3 + 1], box[1], box[4], 6)) << 1) |
          (spread3(quant(x[(int64_t)t * 3 + 2], box[2], box[5], 6)) << 2);
    else if (dim == 2)
      m = spread2(quant(x[(int64_t)t * 2], box[0], box[3], 9)) |
          (spread2(quant(x[(int64_t)t * 2 + 1], box[1], box[4], 9)) << 1);
    else
      m = quant(x[t], box[0], box[3], kCellBits);
    const int key = (b << kCellBits) | (int)m;
    bucket[t] = key;
    rank[t] = atomicAdd(&cnt[key], 1);
  }
}

__global__ __launch_bounds__(256) void k_bucket_scatter(int n_tgt, const int *bucket, const int *rank,
                                                        const int *start, int *list) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_tgt; t += gridDim.x * blockDim.x)
    list[start[bucket[t]] + rank[t]] = t;
}

// bin table from the bucket starts
__global__ void k_bin_table(const int *start, BinMeta *meta) {
  if (threadIdx.x != 0) return;
  for (int b = 0; b < kNumBins; ++b) {
    meta->offset[b] = start[(int64_t)b << kCellBits];
    meta->count[b] = start[(int64_t)(b + 1) << kCellBits] - meta->offset[b];
    meta->cursor[b] = 0;
  }
  meta->err = start[kBuckets] - start[(int64_t)7 << kCellBits] > 0 ? 1 : 0;
  meta->fb_count = 0;
  meta->fb_cursor = 0;
}


__global__ void k_fill_zero(uint32_t *p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Buffers cleared here are whole 32-bit words (counters, tables, flags).
hipError_t fill_zero(void *p, size_t bytes, hipStream_t s) {
  const int64_t words = (int64_t)(bytes / 4);
  if (words == 0) return hipSuccess;
  int64_t g = (words + 255) / 256;
  if (g > 4096) g = 4096;
  k_fill_zero<<<(unsigned)g, 256, 0, s>>>((uint32_t *)p, words);
  return hipGetLastError();
}

__global__ void k_or_error_bit(int *dst, const int *src, int mask, int bit) {
  if (threadIdx.x == 0 && (*src & mask)) atomicOr(dst, bit);
}

hipError_t or_error_bit(int *dst, const int *src, int mask, int bit, hipStream_t s) {
  k_or_error_bit<<<1, 64, 0, s>>>(dst, src, mask, bit);
  return hipGetLastError();
}

__global__ void k_fill_f32(float *p, float v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t fill_f32(float *p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  k_fill_f32<<<(unsigned)g, 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

// ---- report counters ----
// per-status counts: block-local counts, then one atomic per status and block
__global__ __launch_bounds__(256) void k_status_count(const uint8_t *st, int n, ReportCounts *rc) {
  __shared__ unsigned int c[4];
  if (threadIdx.x < 4) c[threadIdx.x] = 0u;
  __syncthreads();
  unsigned int mine[4] = {0u, 0u, 0u, 0u};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int v = st[i];
    if (v < 4) mine[v] += 1u;
  }
  for (int k = 0; k < 4; ++k) {
    const unsigned int w = (unsigned int)wave_sum((int)mine[k]);
    if ((threadIdx.x & 63) == 0 && w) atomicAdd(&c[k], w);
  }
  __syncthreads();
  if (threadIdx.x < 4 && c[threadIdx.x]) atomicAdd(&rc->status[threadIdx.x], (unsigned long long)c[threadIdx.x]);
}

hipError_t launch_status_count(const uint8_t *status, int n, ReportCounts *rc, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  k_status_count<<<g, 256, 0, s>>>(status, n, rc);
  return hipGetLastError();
}

// condition numbers: a block-local histogram in LDS over log2 bins, merged
// into the call's histogram with one atomic per non-empty bin and block
__global__ __launch_bounds__(256) void k_cond_stats(const float *cond, int n, ReportCounts *rc) {
  __shared__ unsigned int h[kCondBins];
  __shared__ unsigned int cmin_inv, cnt;  // ~bits of the smallest value (0: none)
  for (int b = threadIdx.x; b < kCondBins; b += blockDim.x) h[b] = 0u;
  if (threadIdx.x == 0) {
    cmin_inv = 0u;
    cnt = 0u;
  }
  __syncthreads();
  unsigned int mymin_inv = 0u, mycnt = 0u;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float c = cond[i];
    if (!(c >= 0.f) || !isfinite(c)) continue;  // NaN: not computed by the mixed kernels
    const unsigned int inv = ~__float_as_uint(c);
    mymin_inv = inv > mymin_inv ? inv : mymin_inv;
    mycnt += 1u;
    int b = c >= 1.f ? (int)floorf(log2f(c) * (float)kCondBinsPerOctave) : 0;
    b = b < 0 ? 0 : (b >= kCondBins ? kCondBins - 1 : b);
    atomicAdd(&h[b], 1u);
  }
  atomicMax(&cmin_inv, mymin_inv);
  atomicAdd(&cnt, mycnt);
  __syncthreads();
  for (int b = threadIdx.x; b < kCondBins; b += blockDim.x)
    if (h[b]) atomicAdd(&rc->cond_hist[b], h[b]);
  if (threadIdx.x == 0) {
    if (cnt) atomicAdd(&rc->n_cond, (unsigned long long)cnt);
    atomicMax(&rc->cond_min_inv, cmin_inv);
  }
}

hipError_t launch_cond_stats(const float *cond, int n, ReportCounts *rc, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int g = (n + 255) / 256;
  if (g > 512) g = 512;
  k_cond_stats<<<g, 256, 0, s>>>(cond, n, rc);
  return hipGetLastError();
}

// layout of the temporary buffer (8-byte aligned pieces): partial boxes,
// box, bucket counters, bucket starts, per-target bucket and rank, scan
// scratch
static size_t scan_words(int n_tgt) { (void)n_tgt; return (size_t)scan_i32_tmp_words(kBuckets); }

size_t binning_temp_bytes(int n_tgt) {
  const size_t nb = (size_t)(n_tgt > 0 ? n_tgt : 1);
  return sizeof(double) * (6 * kBoxBlocks + 6) + sizeof(int) * ((size_t)kBuckets + (size_t)kBuckets + 2 + 2 * nb) +
         sizeof(int) * scan_words(n_tgt) + 64;
}

hipError_t launch_binning(const int64_t *row_ptr, const double *targets, int n_tgt, int dim, int Q, int C,
                          BinMeta *meta, int *list, void *temp, size_t temp_bytes, hipStream_t s) {
  int g = (n_tgt + kBinBlock - 1) / kBinBlock;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  if (temp_bytes < binning_temp_bytes(n_tgt)) return hipErrorInvalidValue;
  double *partial = (double *)temp;
  double *box = partial + 6 * kBoxBlocks;
  int *cnt = (int *)(box + 6);
  int *start = cnt + kBuckets;
  int *bucket = start + kBuckets + 2;
  int *rank = bucket + n_tgt;
  int *stmp = rank + n_tgt;
  hipError_t e = fill_zero(cnt, sizeof(int) * (size_t)kBuckets, s);
  if (e == hipSuccess) e = fill_zero(meta, sizeof(BinMeta), s);
  if (e != hipSuccess) return e;
  k_tbox_partial<<<kBoxBlocks, 256, 0, s>>>(targets, n_tgt, dim, partial);
  k_tbox_final<<<1, 64, 0, s>>>(partial, kBoxBlocks, box);
  k_bucket_rank<<<g, kBinBlock, 0, s>>>(row_ptr, targets, n_tgt, dim, Q, C, box, cnt, bucket, rank);
  e = scan_i32_exclusive(cnt, start, kBuckets, stmp, s);
  if (e != hipSuccess) return e;
  k_bucket_scatter<<<g, kBinBlock, 0, s>>>(n_tgt, bucket, rank, start, list);
  k_bin_table<<<1, 64, 0, s>>>(start, meta);
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
    if (a.hweights && (int)threadIdx.x < a.F) a.hweights[(int64_t)t * a.F + threadIdx.x] = NAN;
    if (threadIdx.x == 0) a.status[t] = GMLS_TARGET_RANK_DEFICIENT;
  }
}

// The targets of bin `bin` handed to the FP64 QR kernels: status FALLBACK,
// queued on fb_list (counter *fb_count), counted in stats (may be null).
// The wavefront and fused mixed kernels hold a row's sample in registers and
// take the long bin this way; the QR kernels factor long rows in chunks.
__global__ void k_defer_bin(uint8_t *status, const int *list, const BinMeta *meta, int bin, int *fb_list,
                            int *fb_count, Stats *stats) {
  const int n = meta->count[bin], off = meta->offset[bin];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int t = list[off + i];
    status[t] = GMLS_TARGET_FALLBACK;
    fb_list[atomicAdd(fb_count, 1)] = t;
  }
  if (stats && blockIdx.x == 0 && threadIdx.x == 0 && n > 0) atomicAdd(&stats->n_fallback, (unsigned long long)n);
}

hipError_t launch_defer_bin(uint8_t *status, const int *list, const BinMeta *meta, int bin, int *fb_list,
                            int *fb_count, Stats *stats, hipStream_t s) {
  k_defer_bin<<<64, 256, 0, s>>>(status, list, meta, bin, fb_list, fb_count, stats);
  return hipGetLastError();
}

hipError_t launch_rank_deficient(const StencilArgs &a, int C, const int *list, BinMeta *meta, hipStream_t s) {
  k_rank_deficient<<<256, 64, 0, s>>>(a, C, list, meta);
  return hipGetLastError();
}

}  // namespace gmls
