// search.hip -- neighbour search on gfx950 (Section 2.1: the neighbours of a
// target are the particles inside its kernel support).
//
// Cell list: the sources are binned into a uniform grid of cubic cells by a
// counting sort (histogram with atomics, exclusive scan, scatter) and stored
// cell-ordered as (x, y, z, index) records, so that one row of cells along x
// is one contiguous range of memory.  Targets are processed in cell order so
// that neighbouring waves read the same cells.
//
// Query: one wavefront per target.  Candidates from a block of cells are
// streamed through LDS 64 at a time; squared distances use the fixed
// evaluation order (dx*dx + dy*dy) + dz*dz without fused multiply-add.
//  - kNN: the k best (squared distance, index) pairs are kept by sorting the
//    LDS buffer (bitonic network) whenever it fills; the search block grows
//    until the k-th distance is provably smaller than the distance to every
//    unscanned cell.
//  - radius: every source with d^2 < r^2 (count pass, scan, fill pass); a
//    target with fewer than k_min falls back to its k_min nearest.  Rows of
//    up to 256 entries are compacted into a small LDS buffer and sorted in
//    registers by a wave-wide bitonic network; longer rows take a second
//    kernel with a large LDS buffer.
// Every output row is sorted by (squared distance, index).
#include <float.h>
#include <limits.h>

#include "common.hpp"
#include "gmls_internal.hpp"

namespace gmls {

constexpr int kCap = 2048;       // candidate buffer per target (LDS)
constexpr int kScanBlock = 256;  // threads per scan block, 4 items each
constexpr int kScanItems = 4;

// ---------------------------------------------------------------------------
// exclusive scan: out[i] = sum_{q<i} in[q], out[n] = total
// ---------------------------------------------------------------------------
template <typename T>
__device__ T block_exclusive_scan(T v, T *smem, T *total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) smem[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int w = 0; w < nw; ++w) {
      T t = smem[w];
      smem[w] = acc;
      acc += t;
    }
    smem[nw] = acc;
  }
  __syncthreads();
  T res = x - v + smem[wid];
  *total = smem[nw];
  __syncthreads();
  return res;
}

template <typename Tin, typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_local(const Tin *in, T *out, T *block_sums, int64_t n) {
  __shared__ T smem[17];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanItems + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T sum = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = (base + q < n) ? (T)in[base + q] : (T)0;
    sum += v[q];
  }
  T total;
  T pre = block_exclusive_scan<T>(sum, smem, &total);
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    if (base + q < n) out[base + q] = pre;
    pre += v[q];
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_scan_sums(T *block_sums, int64_t nb) {
  __shared__ T smem[17];
  T carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    int64_t i = b0 + threadIdx.x;
    T v = i < nb ? block_sums[i] : (T)0;
    T total;
    T pre = block_exclusive_scan<T>(v, smem, &total);
    if (i < nb) block_sums[i] = pre + carry;
    carry += total;
  }
  if (threadIdx.x == 0) block_sums[nb] = carry;
}

template <typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_add(T *out, const T *block_sums, int64_t n, int64_t nb) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanItems + (int64_t)threadIdx.x * kScanItems;
  const T add = block_sums[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kScanItems; ++q)
    if (base + q < n) out[base + q] += add;
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = block_sums[nb];
}

// out must hold n + 1 entries; tmp must hold nb + 1 entries of T
template <typename Tin, typename T>
static hipError_t exclusive_scan(const Tin *in, T *out, int64_t n, T *tmp, hipStream_t s) {
  const int64_t per = (int64_t)kScanBlock * kScanItems;
  const int64_t nb = (n + per - 1) / per > 0 ? (n + per - 1) / per : 1;
  k_scan_local<Tin, T><<<(unsigned)nb, kScanBlock, 0, s>>>(in, out, tmp, n);
  k_scan_sums<T><<<1, 1024, 0, s>>>(tmp, nb);
  k_scan_add<T><<<(unsigned)nb, kScanBlock, 0, s>>>(out, tmp, n, nb);
  return hipGetLastError();
}

static int64_t scan_tmp_entries(int64_t n) {
  const int64_t per = (int64_t)kScanBlock * kScanItems;
  return (n + per - 1) / per + 2;
}

// ---------------------------------------------------------------------------
// grid construction
// ---------------------------------------------------------------------------
constexpr int kBBoxBlock = 256;

__global__ __launch_bounds__(kBBoxBlock) void k_bbox_partial(const double *pts, int64_t n, int dim,
                                                              double *partial) {
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    for (int d = 0; d < dim; ++d) {
      double v = pts[j * dim + d];
      lo[d] = fmin(lo[d], v);
      hi[d] = fmax(hi[d], v);
    }
  __shared__ double sm[4][6];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int d = 0; d < 3; ++d) {
    double a = wave_min(lo[d]);
    double b = wave_max(hi[d]);
    if (lane == 0) {
      sm[wid][d] = a;
      sm[wid][3 + d] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = sm[0][threadIdx.x];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      v = threadIdx.x < 3 ? fmin(v, sm[w][threadIdx.x]) : fmax(v, sm[w][threadIdx.x]);
    partial[blockIdx.x * 6 + threadIdx.x] = v;
  }
}

// mode 0: kNN with neighbour count k; mode 1: radius r (cells no smaller than r)
__global__ void k_grid_setup(const double *partial, int nb, int dim, int mode, double radius, int k, int64_t n,
                             int64_t ncell_max, GridParams *gp) {
  // one wave reduces the partial boxes, then lane 0 sizes the grid
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  for (int b = threadIdx.x; b < nb; b += 64)
    for (int d = 0; d < dim; ++d) {
      lo[d] = fmin(lo[d], partial[b * 6 + d]);
      hi[d] = fmax(hi[d], partial[b * 6 + 3 + d]);
    }
  for (int d = 0; d < 3; ++d) {
    lo[d] = wave_min(lo[d]);
    hi[d] = wave_max(hi[d]);
  }
  if (threadIdx.x != 0) return;
  for (int d = dim; d < 3; ++d) lo[d] = hi[d] = 0.0;
  double ext_max = 0;
  for (int d = 0; d < dim; ++d) ext_max = fmax(ext_max, hi[d] - lo[d]);
  double c;
  if (mode == 1) {
    c = radius;
  } else if (!(ext_max > 0)) {
    c = 1.0;
  } else {
    double vol = 1.0;
    for (int d = 0; d < dim; ++d) vol *= fmax(hi[d] - lo[d], 1e-3 * ext_max);
    const double omega = dim == 1 ? 2.0 : (dim == 2 ? 3.141592653589793 : 4.188790204786391);
    const double dk = pow(vol * (double)k / ((double)n * omega), 1.0 / dim);
    c = dk / 1.9;
  }
  if (!(c > 0)) c = 1.0;
  int64_t ncell;
  int nc[3];
  for (;;) {
    ncell = 1;
    for (int d = 0; d < 3; ++d) nc[d] = 1;
    for (int d = 0; d < dim; ++d) {
      double f = floor((hi[d] - lo[d]) / c) + 1.0;
      nc[d] = f > 2097152.0 ? 2097152 : (int)f;
      ncell *= nc[d];
    }
    if (ncell <= ncell_max) break;
    c *= 1.25;
  }
  for (int d = 0; d < 3; ++d) gp->lo[d] = d < dim ? lo[d] : 0.0;
  gp->c = c;
  gp->inv_c = 1.0 / c;
  for (int d = 0; d < 3; ++d) gp->nc[d] = nc[d];
  gp->ncell = (int)ncell;
}

__device__ __forceinline__ int cell_coord(const GridParams &g, double x, int d) {
  double f = floor((x - g.lo[d]) * g.inv_c);
  f = fmax(f, 0.0);
  f = fmin(f, (double)(g.nc[d] - 1));
  return (int)f;
}

template <int DIM>
__device__ __forceinline__ int cell_id(const GridParams &g, const double *x) {
  int id = cell_coord(g, x[0], 0);
  if (DIM > 1) id += g.nc[0] * cell_coord(g, x[1], 1);
  if (DIM > 2) id += g.nc[0] * g.nc[1] * cell_coord(g, x[2], 2);
  return id;
}

template <int DIM>
__global__ void k_cell_keys(const GridParams *gp, const double *pts, int64_t n, int *key, int *count) {
  const GridParams g = *gp;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    int id = cell_id<DIM>(g, pts + j * DIM);
    key[j] = id;
    atomicAdd(count + id, 1);
  }
}

template <int DIM>
__global__ void k_cell_scatter(const double *pts, int64_t n, const int *key, const int *start, int *cursor,
                               SPoint *sorted) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    int id = key[j];
    int pos = start[id] + atomicAdd(cursor + id, 1);
    SPoint p;
    p.x = pts[j * DIM];
    p.y = DIM > 1 ? pts[j * DIM + 1] : 0.0;
    p.z = DIM > 2 ? pts[j * DIM + 2] : 0.0;
    p.idx = (int)j;
    p.pad = 0;
    sorted[pos] = p;
  }
}

__global__ void k_index_scatter(int64_t n, const int *key, const int *start, int *cursor, int *order) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    int id = key[j];
    order[start[id] + atomicAdd(cursor + id, 1)] = (int)j;
  }
}

__global__ void k_sorted_order(const SPoint *sorted, int64_t n, int *order) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    order[j] = sorted[j].idx;
}

__global__ void k_knn_rowptr(int64_t n, int k, int64_t *row_ptr) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= n; j += (int64_t)gridDim.x * blockDim.x)
    row_ptr[j] = j * (int64_t)k;
}

// ---------------------------------------------------------------------------
// per-target selection (one wavefront, LDS buffer of kCap candidates)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool key_less(double ad, int ai, double bd, int bi) {
  return ad < bd || (ad == bd && ai < bi);
}

template <int DIM>
__device__ __forceinline__ double dist2_exact(const SPoint &p, const double *x) {
#pragma clang fp contract(off)
  double dx = p.x - x[0];
  double s = dx * dx;
  if (DIM > 1) {
    double dy = p.y - x[1];
    s = s + dy * dy;
  }
  if (DIM > 2) {
    double dz = p.z - x[2];
    s = s + dz * dz;
  }
  return s;
}

// ascending bitonic sort of (d2, idx) over [0, n) in LDS; uses [n, pow2(n))
__device__ void lds_sort(double *d2, int *idx, int n) {
  const int lane = lane_id();
  int np = 1;
  while (np < n) np <<= 1;
  for (int i = n + lane; i < np; i += 64) {
    d2[i] = DBL_MAX;
    idx[i] = INT_MAX;
  }
  __syncthreads();
  for (int size = 2; size <= np; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = lane; i < (np >> 1); i += 64) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        double a = d2[lo], b = d2[hi];
        int ia = idx[lo], ib = idx[hi];
        bool sw = up ? key_less(b, ib, a, ia) : key_less(a, ia, b, ib);
        if (sw) {
          d2[lo] = b;
          d2[hi] = a;
          idx[lo] = ib;
          idx[hi] = ia;
        }
      }
      __syncthreads();
    }
  }
}

// The k nearest sources of x, sorted, in d2[0..k) / idx[0..k); returns the
// count found (k unless there are fewer sources).  r_start: first block radius.
template <int DIM, int CAP>
__device__ int knn_select(const GridParams &g, const SPoint *pts, const int *cell_start, const double *x, int k,
                          int r_start, double *d2, int *idx) {
  const int lane = lane_id();
  int ct[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) ct[d] = cell_coord(g, x[d], d);
  for (int r = r_start;; ++r) {
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    bool covers = true;
    double delta = DBL_MAX;
    for (int d = 0; d < DIM; ++d) {
      lo[d] = ct[d] - r;
      if (lo[d] > 0) {
        covers = false;
        delta = fmin(delta, x[d] - (g.lo[d] + (double)lo[d] * g.c));
      } else
        lo[d] = 0;
      hi[d] = ct[d] + r;
      if (hi[d] < g.nc[d] - 1) {
        covers = false;
        delta = fmin(delta, (g.lo[d] + (double)(hi[d] + 1) * g.c) - x[d]);
      } else
        hi[d] = g.nc[d] - 1;
    }
    int fill = 0;
    bool have_thr = false;
    double thr_d = DBL_MAX;
    int thr_i = INT_MAX;
    for (int cz = lo[2]; cz <= hi[2]; ++cz)
      for (int cy = lo[1]; cy <= hi[1]; ++cy) {
        const int row = g.nc[0] * (cy + g.nc[1] * cz);
        const int beg = readfirstlane_i(cell_start[row + lo[0]]);
        const int end = readfirstlane_i(cell_start[row + hi[0] + 1]);
        for (int b = beg; b < end; b += 64) {
          if (fill + 64 > CAP) {
            lds_sort(d2, idx, fill);
            fill = fill < k ? fill : k;
            if (fill == k) {
              have_thr = true;
              thr_d = uniform_d(d2[k - 1]);
              thr_i = readfirstlane_i(idx[k - 1]);
            }
            __syncthreads();
          }
          const int p = b + lane;
          bool ok = false;
          double dd = 0.0;
          int id = 0;
          if (p < end) {
            const SPoint sp = pts[p];
            dd = dist2_exact<DIM>(sp, x);
            id = sp.idx;
            ok = !have_thr || key_less(dd, id, thr_d, thr_i);
          }
          uint64_t m;
          const int pre = ballot_prefix(ok, &m);
          if (ok) {
            d2[fill + pre] = dd;
            idx[fill + pre] = id;
          }
          fill += __popcll(m);
        }
      }
    __syncthreads();
    lds_sort(d2, idx, fill);
    fill = fill < k ? fill : k;
    if (covers) return fill;
    if (fill == k && uniform_d(d2[k - 1]) < delta * delta * (1.0 - 1e-9)) return fill;
    __syncthreads();
  }
}

template <int DIM>
__global__ __launch_bounds__(64) void k_knn(const GridParams *gp, const SPoint *pts, const int *cell_start,
                                            const double *targets, const int *order, int64_t n_tgt, int k,
                                            double eps_mult, int32_t *col, double *eps) {
  __shared__ double d2[kCap];
  __shared__ int idx[kCap];
  const int64_t w = blockIdx.x;
  if (w >= n_tgt) return;
  const GridParams g = *gp;
  const int t = readfirstlane_i(order[w]);
  double x[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) x[d] = uniform_d(targets[(int64_t)t * DIM + d]);
  const int got = knn_select<DIM, kCap>(g, pts, cell_start, x, k, 2, d2, idx);
  for (int q = lane_id(); q < k; q += 64) col[(int64_t)t * k + q] = q < got ? idx[q] : -1;
  if (lane_id() == 0) eps[t] = eps_mult * sqrt(d2[got - 1]);
}

// block radius needed for a search radius r on cells of side c >= r
__device__ __forceinline__ int radius_blocks(const GridParams &g, double r) {
  int R = (int)ceil(r * g.inv_c);
  return R < 1 ? 1 : R;
}

template <int DIM>
__global__ __launch_bounds__(64) void k_radius_count(const GridParams *gp, const SPoint *pts, const int *cell_start,
                                                     const double *targets, const int *order, int64_t n_tgt,
                                                     double r0, int k_min, int64_t *counts, int *flags) {
  const int64_t w = blockIdx.x;
  if (w >= n_tgt) return;
  const GridParams g = *gp;
  const int t = readfirstlane_i(order[w]);
  const int lane = lane_id();
  double x[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) x[d] = uniform_d(targets[(int64_t)t * DIM + d]);
  const double r2 = r0 * r0;
  const int R = radius_blocks(g, r0);
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) {
    const int c = cell_coord(g, x[d], d);
    lo[d] = max(c - R, 0);
    hi[d] = min(c + R, g.nc[d] - 1);
  }
  int count = 0;
  for (int cz = lo[2]; cz <= hi[2]; ++cz)
    for (int cy = lo[1]; cy <= hi[1]; ++cy) {
      const int row = g.nc[0] * (cy + g.nc[1] * cz);
      const int beg = readfirstlane_i(cell_start[row + lo[0]]);
      const int end = readfirstlane_i(cell_start[row + hi[0] + 1]);
      for (int b = beg; b < end; b += 64) {
        const int p = b + lane;
        bool ok = false;
        if (p < end) ok = dist2_exact<DIM>(pts[p], x) < r2;
        count += __popcll(__ballot(ok));
      }
    }
  if (count > kCap) {
    if (lane == 0) atomicOr(flags, 1);
    count = kCap;
  }
  if (count < k_min) count = k_min;
  if (lane == 0) counts[t] = count;
}

// Ascending bitonic sort of 64*EPL (d2, idx) keys held in registers, element
// e = lane*EPL + r in slot r; pairs further apart than EPL are exchanged with
// the partner lane through shuffles.
template <int EPL>
__device__ __forceinline__ void wave_sort(double (&kd)[EPL], int (&ki)[EPL], int lane) {
  constexpr int E = 64 * EPL;
#pragma unroll
  for (int size = 2; size <= E; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= EPL) {
        const int lmask = stride / EPL;
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
          const int e = lane * EPL + r;
          const double od = __shfl_xor(kd[r], lmask, 64);
          const int oi = __shfl_xor(ki[r], lmask, 64);
          const bool lower = (e & stride) == 0;
          const bool up = (e & size) == 0;
          const bool other_less = key_less(od, oi, kd[r], ki[r]);
          // lower element of an ascending pair keeps the smaller key, etc.
          const bool take = (lower == up) ? other_less : !other_less;
          if (take) {
            kd[r] = od;
            ki[r] = oi;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
          if (r & stride) continue;
          const int e = lane * EPL + r;
          const bool up = (e & size) == 0;
          const int r2 = r + stride;
          const bool sw = up ? key_less(kd[r2], ki[r2], kd[r], ki[r]) : key_less(kd[r], ki[r], kd[r2], ki[r2]);
          if (sw) {
            const double td = kd[r];
            const int ti = ki[r];
            kd[r] = kd[r2];
            ki[r] = ki[r2];
            kd[r2] = td;
            ki[r2] = ti;
          }
        }
      }
    }
  }
}

// load n <= 64*EPL candidates from LDS, sort them in registers, write the row
template <int EPL>
__device__ __forceinline__ void sort_and_store(const double *d2, const int *idx, int n, int32_t *out, int lane) {
  double kd[EPL];
  int ki[EPL];
#pragma unroll
  for (int r = 0; r < EPL; ++r) {
    const int e = lane * EPL + r;
    kd[r] = e < n ? d2[e] : DBL_MAX;
    ki[r] = e < n ? idx[e] : INT_MAX;
  }
  wave_sort<EPL>(kd, ki, lane);
#pragma unroll
  for (int r = 0; r < EPL; ++r) {
    const int e = lane * EPL + r;
    if (e < n) out[e] = ki[r];
  }
}

constexpr int kSmallCap = 256;  // candidates per target in the common-case kernel

// Common case: at most kSmallCap sources inside the radius and a floor that
// fits the small buffer.  Other targets are appended to `overflow` for
// k_radius_fill_big.
template <int DIM>
__global__ __launch_bounds__(64) void k_radius_fill(const GridParams *gp, const SPoint *pts, const int *cell_start,
                                                    const double *targets, const int *order, int64_t n_tgt,
                                                    double r0, int k_min, const int64_t *row_ptr, int32_t *col,
                                                    double *eps, int *overflow, int *n_overflow) {
  __shared__ double d2[kSmallCap];
  __shared__ int idx[kSmallCap];
  const int64_t w = blockIdx.x;
  if (w >= n_tgt) return;
  const GridParams g = *gp;
  const int t = readfirstlane_i(order[w]);
  const int lane = lane_id();
  double x[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) x[d] = uniform_d(targets[(int64_t)t * DIM + d]);
  const double r2 = r0 * r0;
  const int R = radius_blocks(g, r0);
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) {
    const int c = cell_coord(g, x[d], d);
    lo[d] = max(c - R, 0);
    hi[d] = min(c + R, g.nc[d] - 1);
  }
  int fill = 0;
  for (int cz = lo[2]; cz <= hi[2]; ++cz)
    for (int cy = lo[1]; cy <= hi[1]; ++cy) {
      const int row = g.nc[0] * (cy + g.nc[1] * cz);
      const int beg = readfirstlane_i(cell_start[row + lo[0]]);
      const int end = readfirstlane_i(cell_start[row + hi[0] + 1]);
      for (int b = beg; b < end; b += 64) {
        const int p = b + lane;
        bool ok = false;
        double dd = 0.0;
        int id = 0;
        if (p < end) {
          const SPoint sp = pts[p];
          dd = dist2_exact<DIM>(sp, x);
          id = sp.idx;
          ok = dd < r2;
        }
        uint64_t m;
        const int pre = ballot_prefix(ok, &m);
        if (ok && fill + pre < kSmallCap) {
          d2[fill + pre] = dd;
          idx[fill + pre] = id;
        }
        fill += __popcll(m);
      }
    }
  const bool big = fill > kSmallCap || (fill < k_min && k_min + 65 > kSmallCap);
  if (big) {
    if (lane == 0) overflow[atomicAdd(n_overflow, 1)] = t;
    return;
  }
  const int64_t base = row_ptr[t];
  __syncthreads();
  if (fill >= k_min) {
    if (fill <= 64)
      sort_and_store<1>(d2, idx, fill, col + base, lane);
    else if (fill <= 128)
      sort_and_store<2>(d2, idx, fill, col + base, lane);
    else
      sort_and_store<4>(d2, idx, fill, col + base, lane);
    if (lane == 0) eps[t] = r0;
  } else {
    const int got = knn_select<DIM, kSmallCap>(g, pts, cell_start, x, k_min + 1, 1, d2, idx);
    for (int q = lane; q < k_min; q += 64) col[base + q] = idx[q];
    if (lane == 0) eps[t] = got > k_min ? 0.5 * (sqrt(d2[k_min - 1]) + sqrt(d2[k_min])) : r0;
  }
}

// Targets with more candidates than the small buffer (or a large floor):
// LDS buffer of kCap entries and a bitonic sort in LDS.
template <int DIM>
__global__ __launch_bounds__(64) void k_radius_fill_big(const GridParams *gp, const SPoint *pts,
                                                        const int *cell_start, const double *targets, double r0,
                                                        int k_min, const int64_t *row_ptr, int32_t *col, double *eps,
                                                        const int *overflow, const int *n_overflow) {
  __shared__ double d2[kCap];
  __shared__ int idx[kCap];
  const GridParams g = *gp;
  const int lane = lane_id();
  const int n = readfirstlane_i(*n_overflow);
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int t = readfirstlane_i(overflow[w]);
    double x[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) x[d] = uniform_d(targets[(int64_t)t * DIM + d]);
    const double r2 = r0 * r0;
    const int R = radius_blocks(g, r0);
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) {
      const int c = cell_coord(g, x[d], d);
      lo[d] = max(c - R, 0);
      hi[d] = min(c + R, g.nc[d] - 1);
    }
    int fill = 0;
    for (int cz = lo[2]; cz <= hi[2]; ++cz)
      for (int cy = lo[1]; cy <= hi[1]; ++cy) {
        const int row = g.nc[0] * (cy + g.nc[1] * cz);
        const int beg = readfirstlane_i(cell_start[row + lo[0]]);
        const int end = readfirstlane_i(cell_start[row + hi[0] + 1]);
        for (int b = beg; b < end; b += 64) {
          const int p = b + lane;
          bool ok = false;
          double dd = 0.0;
          int id = 0;
          if (p < end) {
            const SPoint sp = pts[p];
            dd = dist2_exact<DIM>(sp, x);
            id = sp.idx;
            ok = dd < r2;
          }
          uint64_t m;
          const int pre = ballot_prefix(ok, &m);
          if (ok && fill + pre < kCap) {
            d2[fill + pre] = dd;
            idx[fill + pre] = id;
          }
          fill += __popcll(m);
        }
      }
    const int64_t base = row_ptr[t];
    __syncthreads();
    if (fill >= k_min) {
      if (fill > kCap) fill = kCap;  // flagged by the count pass; the call fails
      lds_sort(d2, idx, fill);
      for (int q = lane; q < fill; q += 64) col[base + q] = idx[q];
      if (lane == 0) eps[t] = r0;
    } else {
      const int got = knn_select<DIM, kCap>(g, pts, cell_start, x, k_min + 1, 1, d2, idx);
      for (int q = lane; q < k_min; q += 64) col[base + q] = idx[q];
      if (lane == 0) eps[t] = got > k_min ? 0.5 * (sqrt(d2[k_min - 1]) + sqrt(d2[k_min])) : r0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
static inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

#define GMLS_HIP(...)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (__VA_ARGS__);                                                                     \
    if (e_ != hipSuccess) return gmls_set_error(ctx, GMLS_ERR_HIP, std::string(#__VA_ARGS__) + ": " +  \
                                                hipGetErrorString(e_));                         \
  } while (0)

#define GMLS_WS(ptr, type, slot, count)                                                             \
  type *ptr = (type *)ctx->ws(slot, sizeof(type) * (size_t)(count));                                \
  if (!ptr) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed (" #ptr ")")

template <int DIM>
static gmls_status neighbors_dim(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                                 int64_t n_tgt, const gmls_search &spec, int64_t *row_ptr, int32_t *col,
                                 int64_t col_capacity, double *eps, int64_t *nnz_host) {
  hipStream_t s = ctx->stream;
  const bool knn = spec.mode == GMLS_SEARCH_KNN;
  if (knn) {
    const int64_t nnz = n_tgt * (int64_t)spec.k;
    *nnz_host = nnz;
    if (nnz > col_capacity)
      return gmls_set_error(ctx, GMLS_ERR_CAPACITY, "col_capacity " + std::to_string(col_capacity) +
                                                        " < required " + std::to_string(nnz));
  }
  const int64_t ncell_max = 4 * n_src + 64;
  const unsigned nb_bbox = grid_for(n_src, kBBoxBlock * 4) > 1024 ? 1024 : grid_for(n_src, kBBoxBlock * 4);
  GMLS_WS(bbox, double, WS_BBOX, nb_bbox * 6);
  GMLS_WS(gp, GridParams, WS_GRID, 1);
  GMLS_WS(key, int, WS_CELL_KEY, n_src);
  GMLS_WS(cnt, int, WS_CELL_COUNT, ncell_max + 1);
  GMLS_WS(start, int, WS_CELL_START, ncell_max + 1);
  GMLS_WS(sorted, SPoint, WS_SORTED, n_src);
  GMLS_WS(order, int, WS_TGT_ORDER, n_tgt > 0 ? n_tgt : 1);
  GMLS_WS(tmp, int64_t, WS_SCAN_TMP, scan_tmp_entries(ncell_max + 1 > n_tgt + 1 ? ncell_max + 1 : n_tgt + 1));
  GMLS_WS(flags, int, WS_FLAGS, 4);

  k_bbox_partial<<<nb_bbox, kBBoxBlock, 0, s>>>(coords, n_src, DIM, bbox);
  k_grid_setup<<<1, 64, 0, s>>>(bbox, (int)nb_bbox, DIM, knn ? 0 : 1, spec.radius, spec.k, n_src, ncell_max, gp);
  GMLS_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * (size_t)(ncell_max + 1), s));
  GMLS_HIP(hipMemsetAsync(flags, 0, sizeof(int) * 4, s));
  k_cell_keys<DIM><<<grid_for(n_src, 256), 256, 0, s>>>(gp, coords, n_src, key, cnt);
  GMLS_HIP(exclusive_scan<int, int>(cnt, start, ncell_max, (int *)tmp, s));
  GMLS_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * (size_t)(ncell_max + 1), s));
  k_cell_scatter<DIM><<<grid_for(n_src, 256), 256, 0, s>>>(coords, n_src, key, start, cnt, sorted);
  GMLS_HIP(hipGetLastError());
  if (n_tgt > 0) {
    if (targets == coords && n_tgt == n_src) {
      k_sorted_order<<<grid_for(n_tgt, 256), 256, 0, s>>>(sorted, n_tgt, order);
    } else {
      GMLS_WS(tkey, int, WS_TGT_KEY, n_tgt);
      GMLS_WS(tcnt, int, WS_TGT_COUNT, ncell_max + 1);
      GMLS_WS(tstart, int, WS_TGT_START, ncell_max + 1);
      GMLS_HIP(hipMemsetAsync(tcnt, 0, sizeof(int) * (size_t)(ncell_max + 1), s));
      k_cell_keys<DIM><<<grid_for(n_tgt, 256), 256, 0, s>>>(gp, targets, n_tgt, tkey, tcnt);
      GMLS_HIP(exclusive_scan<int, int>(tcnt, tstart, ncell_max, (int *)tmp, s));
      GMLS_HIP(hipMemsetAsync(tcnt, 0, sizeof(int) * (size_t)(ncell_max + 1), s));
      k_index_scatter<<<grid_for(n_tgt, 256), 256, 0, s>>>(n_tgt, tkey, tstart, tcnt, order);
    }
    GMLS_HIP(hipGetLastError());
  }
  if (knn) {
    k_knn_rowptr<<<grid_for(n_tgt + 1, 256), 256, 0, s>>>(n_tgt, spec.k, row_ptr);
    if (n_tgt > 0)
      k_knn<DIM><<<(unsigned)n_tgt, 64, 0, s>>>(gp, sorted, start, targets, order, n_tgt, spec.k, spec.eps_mult,
                                                col, eps);
    GMLS_HIP(hipGetLastError());
    GMLS_HIP(hipStreamSynchronize(s));
    return GMLS_OK;
  }
  GMLS_WS(counts, int64_t, WS_ROW_COUNT, n_tgt > 0 ? n_tgt : 1);
  if (n_tgt > 0)
    k_radius_count<DIM><<<(unsigned)n_tgt, 64, 0, s>>>(gp, sorted, start, targets, order, n_tgt, spec.radius,
                                                       spec.k_min, counts, flags);
  GMLS_HIP(exclusive_scan<int64_t, int64_t>(counts, row_ptr, n_tgt, tmp, s));
  int64_t nnz = 0;
  int hflags = 0;
  GMLS_HIP(hipMemcpyAsync(&nnz, row_ptr + n_tgt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  GMLS_HIP(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s));
  GMLS_HIP(hipStreamSynchronize(s));
  *nnz_host = nnz;
  if (hflags & 1)
    return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "a target has more than 2048 sources inside the radius");
  if (nnz > col_capacity)
    return gmls_set_error(ctx, GMLS_ERR_CAPACITY,
                          "col_capacity " + std::to_string(col_capacity) + " < required " + std::to_string(nnz));
  if (n_tgt > 0) {
    GMLS_HIP(hipMemsetAsync(flags + 1, 0, sizeof(int), s));
    k_radius_fill<DIM><<<(unsigned)n_tgt, 64, 0, s>>>(gp, sorted, start, targets, order, n_tgt, spec.radius,
                                                      spec.k_min, row_ptr, col, eps, (int *)counts, flags + 1);
    k_radius_fill_big<DIM><<<1024, 64, 0, s>>>(gp, sorted, start, targets, spec.radius, spec.k_min, row_ptr, col,
                                               eps, (int *)counts, flags + 1);
  }
  GMLS_HIP(hipGetLastError());
  GMLS_HIP(hipStreamSynchronize(s));
  return GMLS_OK;
}

gmls_status run_neighbors(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                          int64_t n_tgt, int dim, const gmls_search &spec, int64_t *row_ptr, int32_t *col,
                          int64_t col_capacity, double *eps, int64_t *nnz_host) {
  switch (dim) {
    case 1:
      return neighbors_dim<1>(ctx, coords, n_src, targets, n_tgt, spec, row_ptr, col, col_capacity, eps, nnz_host);
    case 2:
      return neighbors_dim<2>(ctx, coords, n_src, targets, n_tgt, spec, row_ptr, col, col_capacity, eps, nnz_host);
    case 3:
      return neighbors_dim<3>(ctx, coords, n_src, targets, n_tgt, spec, row_ptr, col, col_capacity, eps, nnz_host);
    default:
      return gmls_set_error(ctx, GMLS_ERR_ARG, "dim must be 1, 2 or 3");
  }
}

}  // namespace gmls
