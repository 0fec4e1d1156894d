// search.hip -- neighbour search on gfx950 (Section 2.1: the neighbours of a
// target are the particles inside its kernel support).
//
// Cell list: the sources are binned into a uniform grid of cubic cells by a
// counting sort (histogram with atomics, exclusive scan, scatter) and stored
// cell-ordered as (x, y, z, index) records, so that one row of cells along x
// is one contiguous range of memory.  Targets are processed in cell order so
// that neighbouring waves read the same cells.
//
// kNN query (cells of side about d_k/1.9): one wavefront per target.  The
// block of cells within 2 (then 3) of the target's cell is read as runs of
// cells along x, whose bounds are fetched together so that a chunk of 64
// candidate loads goes out at once; exact squared distances (fixed order
// (dx*dx + dy*dy) + dz*dz, no fused multiply-add) closer than the block's
// inner margin are kept, a bisection on d^2 (ballot counts over registers)
// trims them to the capacity of a register bitonic sort of (d^2, index)
// pairs, and the k smallest are the row.  Targets with fewer than k inside
// the margin go to a second register pass with a wider block, then to a
// per-target kernel that expands the block until the k-th distance is
// provably below the distance to every unscanned cell.
//
// Radius query (cells of side >= r): a workgroup stages the sources of the
// 3^dim block around one target cell in LDS and its four wavefronts share
// them among the cell's targets, several targets per wavefront reading each
// staged candidate once.  Accepted sources are compacted by ballot prefix
// sums into a scratch row of up to 256 entries per target (one-pass mode) or
// straight into `col` after a count pass and a scan (two-pass mode, when the
// scratch does not fit its budget); the scratch rows are copied into place
// after the scan of the counts (k_rows_copy).  Targets that need the k_min
// floor, rows over 256 entries and crowded blocks are finished by
// per-target kernels.
//
// kNN rows are sorted by (squared distance, index).  Radius rows, which are
// sets, come out in cell order, by (cell of the source, index): each cell's
// sources are put in ascending index once per search, and the staged scan
// emits them in that order with no sort.  GMLS_OPT_ROW_ORDER = 1 sorts each
// row by index instead (a register bitonic network per row).
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

int64_t scan_i32_tmp_words(int64_t n) { return scan_tmp_entries(n); }

hipError_t scan_i32_exclusive(const int *in, int *out, int64_t n, int *tmp, hipStream_t s) {
  return exclusive_scan<int, int>(in, out, n, tmp, s);
}

hipError_t scan_i64_exclusive(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s) {
  return exclusive_scan<int64_t, int64_t>(in, out, n, tmp, s);
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

// Sources of each cell in ascending index (the scatter above places them in
// atomic order): one wavefront per cell, from `in` to `out`.  The rank of an
// entry is the number of smaller indices in its cell, taken from an LDS copy
// of the cell's indices (from `in` directly for cells over kSortCellCap).
constexpr int kSortCellCap = 1024;
__global__ __launch_bounds__(64) void k_cell_sort(const GridParams *gp, const int *start,
                                                  const SPoint *__restrict__ in, SPoint *__restrict__ out) {
  __shared__ int ids[kSortCellCap];
  const int lane = lane_id();
  const int ncell = gp->ncell;
  for (int c = blockIdx.x; c < ncell; c += gridDim.x) {
    const int b = start[c], n = start[c + 1] - b;
    if (n == 0) continue;
    const bool staged = n <= kSortCellCap;
    if (staged) {
      for (int q = lane; q < n; q += 64) ids[q] = in[b + q].idx;
      __syncthreads();
    }
    for (int q0 = 0; q0 < n; q0 += 64) {
      const int q = q0 + lane;
      SPoint p{};
      int rank = 0;
      if (q < n) {
        p = in[b + q];
        for (int j = 0; j < n; ++j) rank += (staged ? ids[j] : in[b + j].idx) < p.idx ? 1 : 0;
        out[b + rank] = p;
      }
    }
    __syncthreads();
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


// block radius needed for a search radius r on cells of side c >= r
__device__ __forceinline__ int radius_blocks(const GridParams &g, double r) {
  int R = (int)ceil(r * g.inv_c);
  return R < 1 ? 1 : R;
}

// Cells and rows of the (2R+1)^DIM block around the cell of x.
template <int DIM>
__device__ __forceinline__ void radius_block(const GridParams &g, const double *x, int R, int *lo, int *hi) {
  for (int d = 0; d < 3; ++d) lo[d] = hi[d] = 0;
  for (int d = 0; d < DIM; ++d) {
    const int c = cell_coord(g, x[d], d);
    lo[d] = max(c - R, 0);
    hi[d] = min(c + R, g.nc[d] - 1);
  }
}

// ---------------------------------------------------------------------------
// radius rows: ascending bitonic sort of up to 64*EPL indices in registers
// (element e = lane*EPL + r in slot r; partners further apart than EPL are
// exchanged through shuffles)
// ---------------------------------------------------------------------------
// v of lane (lane ^ lm) for a compile-time lm (after unrolling): DPP for
// lm = 1, 2, 8 (quad permutes, rotation by 8 within a row of 16), swizzles
// for lm = 4, 16, a permute through LDS only for lm = 32
__device__ __forceinline__ int xor_lane(int v, int lm) {
  switch (lm) {
    case 1: return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    case 2: return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    case 4: return __builtin_amdgcn_ds_swizzle(v, 0x101F);                     // xor 4 within 32
    case 8: return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);  // row_ror:8
    case 16: return __builtin_amdgcn_ds_swizzle(v, 0x401F);                    // xor 16 within 32
    default: return __shfl_xor(v, lm, 64);
  }
}

template <int EPL>
__device__ __forceinline__ void wave_sort_int(int (&k)[EPL], int lane) {
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
          const int o = xor_lane(k[r], lmask);
          const bool keep_min = ((e & stride) == 0) == ((e & size) == 0);
          k[r] = keep_min ? min(k[r], o) : max(k[r], o);
        }
      } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
          if (r & stride) continue;
          const int e = lane * EPL + r;
          const bool up = (e & size) == 0;
          const int lo = min(k[r], k[r + stride]), hi = max(k[r], k[r + stride]);
          k[r] = up ? lo : hi;
          k[r + stride] = up ? hi : lo;
        }
      }
    }
  }
}

// NT_ independent bitonic networks, stage by stage (same network as above)
template <int EPL, int NT_>
__device__ __forceinline__ void wave_sort_multi(int (&k)[NT_][EPL], int lane) {
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
          const bool keep_min = ((e & stride) == 0) == ((e & size) == 0);
          int o[NT_];
#pragma unroll
          for (int u = 0; u < NT_; ++u) o[u] = xor_lane(k[u][r], lmask);
#pragma unroll
          for (int u = 0; u < NT_; ++u) k[u][r] = keep_min ? min(k[u][r], o[u]) : max(k[u][r], o[u]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
          if (r & stride) continue;
          const int e = lane * EPL + r;
          const bool up = (e & size) == 0;
#pragma unroll
          for (int u = 0; u < NT_; ++u) {
            const int lo = min(k[u][r], k[u][r + stride]), hi = max(k[u][r], k[u][r + stride]);
            k[u][r] = up ? lo : hi;
            k[u][r + stride] = up ? hi : lo;
          }
        }
      }
    }
  }
}

// sort n <= 64*EPL indices of an LDS buffer and write them to out[0 .. n)
template <int EPL>
__device__ __forceinline__ void sort_idx_store(const int *buf, int n, int32_t *out, int lane) {
  int k[EPL];
#pragma unroll
  for (int r = 0; r < EPL; ++r) {
    const int e = lane * EPL + r;
    k[r] = e < n ? buf[e] : INT_MAX;
  }
  wave_sort_int<EPL>(k, lane);
#pragma unroll
  for (int r = 0; r < EPL; ++r) {
    const int e = lane * EPL + r;
    if (e < n) out[e] = k[r];
  }
}

__device__ __forceinline__ void sort_idx_any(const int *buf, int n, int32_t *out, int lane) {
  if (n <= 64)
    sort_idx_store<1>(buf, n, out, lane);
  else if (n <= 128)
    sort_idx_store<2>(buf, n, out, lane);
  else
    sort_idx_store<4>(buf, n, out, lane);
}

// NT independent rows sorted together (interleaved networks): row u has
// n[u] <= 64*EPL entries in buf[u] and goes to out[u]; n[u] = 0 is skipped
template <int EPL, int NT_, int ROWLEN>
__device__ __forceinline__ void sort_idx_multi(const int (*buf)[ROWLEN], const int *n, int32_t *const *out,
                                               int lane) {
  int k[NT_][EPL];
#pragma unroll
  for (int u = 0; u < NT_; ++u)
#pragma unroll
    for (int r = 0; r < EPL; ++r) {
      const int e = lane * EPL + r;
      k[u][r] = e < n[u] ? buf[u][e] : INT_MAX;
    }
  wave_sort_multi<EPL, NT_>(k, lane);
#pragma unroll
  for (int u = 0; u < NT_; ++u)
#pragma unroll
    for (int r = 0; r < EPL; ++r) {
      const int e = lane * EPL + r;
      if (e < n[u]) out[u][e] = k[u][r];
    }
}

// ascending bitonic sort of idx[0, n) in LDS (one-wavefront blocks)
__device__ void lds_sort_int(int *idx, int n) {
  const int lane = lane_id();
  int np = 1;
  while (np < n) np <<= 1;
  for (int i = n + lane; i < np; i += 64) idx[i] = INT_MAX;
  __syncthreads();
  for (int size = 2; size <= np; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = lane; i < (np >> 1); i += 64) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const int a = idx[lo], b = idx[hi];
        if (up ? b < a : a < b) {
          idx[lo] = b;
          idx[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// kNN, register path: one wavefront per target scans the block of cells
// within R = 2 of its cell (cells have side ~ d_k / 1.9, so the block covers
// the k-th neighbour with a margin), keeps the candidates closer than the
// block's inner margin delta (every source closer than delta lies in the
// block), and sorts them by (d^2, index) in registers.  When fewer than k
// candidates lie within delta, or more than 64*EPL, the target goes to the
// per-target expanding kernel above (k_knn_list).  The k smallest of the kept
// set are the k smallest of all sources, since the set holds every source
// within delta and at least k of them.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double xor_lane_d(double v, int lm) {
  int2 b = __builtin_bit_cast(int2, v);
  b.x = xor_lane(b.x, lm);
  b.y = xor_lane(b.y, lm);
  return __builtin_bit_cast(double, b);
}

// ascending bitonic sort of 64*EPL (d, id) pairs by (d, id), element
// e = lane*EPL + r in slot r (the network of wave_sort_int)
template <int EPL>
__device__ __forceinline__ void wave_sort_pair(double (&d)[EPL], int (&id)[EPL], int lane) {
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
          const double od = xor_lane_d(d[r], lmask);
          const int oi = xor_lane(id[r], lmask);
          const bool keep_min = ((e & stride) == 0) == ((e & size) == 0);
          const bool mine_less = key_less(d[r], id[r], od, oi);
          const bool take = keep_min ? !mine_less : mine_less;
          d[r] = take ? od : d[r];
          id[r] = take ? oi : id[r];
        }
      } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
          if (r & stride) continue;
          const int e = lane * EPL + r;
          const bool up = (e & size) == 0;
          const bool sw = up ? key_less(d[r + stride], id[r + stride], d[r], id[r])
                             : key_less(d[r], id[r], d[r + stride], id[r + stride]);
          const double td = d[r];
          const int ti = id[r];
          d[r] = sw ? d[r + stride] : d[r];
          id[r] = sw ? id[r + stride] : id[r];
          d[r + stride] = sw ? td : d[r + stride];
          id[r + stride] = sw ? ti : id[r + stride];
        }
      }
    }
  }
}

// the n <= 64*EPL pairs of bd/bi sorted by (d^2, index); the first k are the
// target's row, the k-th distance defines eps
template <int EPL>
__device__ __forceinline__ void knn_sort_write(const double *bd, const int *bi, int n, int k, int t,
                                               double eps_mult, int32_t *col, double *eps, int lane) {
  double kd[EPL];
  int kid[EPL];
#pragma unroll
  for (int r = 0; r < EPL; ++r) {
    const int e = lane * EPL + r;
    kd[r] = e < n ? bd[e] : DBL_MAX;
    kid[r] = e < n ? bi[e] : INT_MAX;
  }
  wave_sort_pair<EPL>(kd, kid, lane);
#pragma unroll
  for (int r = 0; r < EPL; ++r) {
    const int e = lane * EPL + r;
    if (e < k) col[(int64_t)t * k + e] = kid[r];
    if (e == k - 1) eps[t] = eps_mult * sqrt(kd[r]);
  }
}

// One wavefront per target of `list` (or of order[0, n_tgt) when n_list is
// null): candidates of the block of cells within R of the target's cell that
// are closer than the block's inner margin delta go to LDS (at most 64*EPLL);
// when there are more than 64*EPLS of them, a bisection on the squared
// distance finds a threshold T holding at least k and at most 64*EPLS of
// them; the candidates with d^2 <= T (a superset of the k nearest: the k-th
// smallest d^2 is <= T) are sorted by (d^2, index) in registers.
template <int DIM, int EPLL, int EPLS>
__global__ __launch_bounds__(64) void k_knn_reg(const GridParams *gp, const SPoint *pts, const int *cell_start,
                                                const double *targets, const int *list, const int *n_list,
                                                int64_t n_tgt, int R, int k, double eps_mult, int32_t *col,
                                                double *eps, int *slow, int *n_slow) {
  constexpr int CAP = 64 * EPLL, SCAP = 64 * EPLS;
  __shared__ double cd[CAP];
  __shared__ int ci[CAP];
  // chunks of 64 candidates loaded together: more loads in flight cost
  // registers and occupancy, which pay only for the larger blocks
  constexpr int KU = EPLL >= 8 ? 2 : 1;
  __shared__ double sd[SCAP];
  __shared__ int si[SCAP];
  __shared__ int rpre[64], roff[64];  // per run: first candidate number, source offset
  // targets left to the next pass, gathered per wavefront and appended to
  // `slow` 64 at a time (one atomic per 64 rather than one per target: when
  // most targets are left, as for targets on the boundary of the cloud, a
  // per-target atomic on the one counter serialises the wavefronts)
  __shared__ int pend[64];
  const GridParams g = *gp;
  const int lane = lane_id();
  int npend = 0;  // uniform
  auto flush_slow = [&]() {
    wave_lds_sync();
    int b = 0;
    if (lane == 0) b = atomicAdd(n_slow, npend);
    b = readfirstlane_i(b);
    if (lane < npend) slow[b + lane] = pend[lane];
    npend = 0;
    wave_lds_sync();
  };
  auto push_slow = [&](int tt) {
    if (lane == 0) pend[npend] = tt;
    if (++npend == 64) flush_slow();
  };
  const int64_t n = n_list ? (int64_t)readfirstlane_i(*n_list) : n_tgt;
  for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
    const int t = readfirstlane_i(list[w]);
    double x[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) x[d] = uniform_d(targets[(int64_t)t * DIM + d]);
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    double delta = DBL_MAX;
    for (int d = 0; d < DIM; ++d) {
      const int c = cell_coord(g, x[d], d);
      lo[d] = c - R;
      if (lo[d] > 0)
        delta = fmin(delta, x[d] - (g.lo[d] + (double)lo[d] * g.c));
      else
        lo[d] = 0;
      hi[d] = c + R;
      if (hi[d] < g.nc[d] - 1)
        delta = fmin(delta, (g.lo[d] + (double)(hi[d] + 1) * g.c) - x[d]);
      else
        hi[d] = g.nc[d] - 1;
    }
    const double delta2 = delta == DBL_MAX ? DBL_MAX : delta * delta;
    // the block's runs of cells along x, one per lane: their bounds are
    // fetched together, and the candidates of all runs are numbered by an
    // exclusive prefix over the runs, so that a lane finds the source of
    // candidate e by a binary search and the loads of KU chunks of 64
    // candidates are in flight at once
    const int ny = hi[1] - lo[1] + 1;
    const int nrun = readfirstlane_i(ny * (hi[2] - lo[2] + 1));
    if (nrun > 64) {  // blocks wider than the wavefront: the next pass
      push_slow(t);
      continue;
    }
    int rb = 0, rl = 0;
    if (lane < nrun) {
      const int row = g.nc[0] * ((lo[1] + lane % ny) + g.nc[1] * (lo[2] + lane / ny));
      rb = cell_start[row + lo[0]];
      rl = cell_start[row + hi[0] + 1] - rb;
    }
    int incl = rl;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    const int total = readlane_i(incl, 63);
    wave_lds_sync();  // the previous target's reads of the run tables are done
    rpre[lane] = lane < nrun ? incl - rl : INT_MAX;
    roff[lane] = rb - (incl - rl);
    wave_lds_sync();
    int fill = 0;
    for (int base = 0; base < total; base += 64 * KU) {
      SPoint sp[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int e = base + 64 * u + lane;
        // the last run starting at or before e (rpre[0] = 0; rpre is
        // non-decreasing and INT_MAX past the last run)
        int q = 0;
#pragma unroll
        for (int st = 32; st >= 1; st >>= 1) q = rpre[q + st] <= e ? q + st : q;
        if (e < total) sp[u] = pts[roff[q] + e];
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int e = base + 64 * u + lane;
        bool ok = false;
        double dd = 0.0;
        int id = 0;
        if (e < total) {
          dd = dist2_exact<DIM>(sp[u], x);
          id = sp[u].idx;
          ok = dd < delta2;
        }
        uint64_t m;
        const int pre = ballot_prefix(ok, &m);
        if (ok && fill + pre < CAP) {
          cd[fill + pre] = dd;
          ci[fill + pre] = id;
        }
        fill += __popcll(m);
      }
    }
    if (fill < k || fill > CAP) {  // not provably covered, or too many: the next pass
      push_slow(t);
      continue;
    }
    wave_lds_sync();
    // the sort takes 64*EPLS pairs, or half as many when k fits in half: the
    // bisection then aims at the half (a narrower network), and keeps the
    // full width when ties leave more than half
    constexpr int EH = EPLS >= 2 ? EPLS / 2 : EPLS;
    const int cap = EPLS >= 2 && k <= 64 * EH ? 64 * EH : SCAP;
    const double *bd = cd;
    const int *bi = ci;
    int nb = fill;
    if (fill > cap) {
      double dl[EPLL];
      double hiT = 0.0;
#pragma unroll
      for (int r = 0; r < EPLL; ++r) {
        const int e = lane + 64 * r;
        dl[r] = e < fill ? cd[e] : DBL_MAX;
        if (e < fill) hiT = fmax(hiT, dl[r]);
      }
      hiT = uniform_d(wave_max(hiT));
      double loT = 0.0;
      int cnt = fill;
      // invariant: count(d^2 <= hiT) >= k; stop once it is <= cap, or after
      // 16 steps aimed at the half once the full width holds the count
      // (ties at the k-th distance can keep the count above the half)
      for (int it = 0; it < 64 && cnt > cap; ++it) {
        if (it >= 16 && cnt <= SCAP) break;
        const double mid = 0.5 * (loT + hiT);
        if (!(mid > loT && mid < hiT)) break;
        int c = 0;
#pragma unroll
        for (int r = 0; r < EPLL; ++r) c += __popcll(__ballot(dl[r] <= mid));
        if (c >= k) {
          hiT = mid;
          cnt = c;
        } else {
          loT = mid;
        }
      }
      if (cnt > SCAP) {  // ties beyond the sort capacity: the next pass
        push_slow(t);
        wave_lds_sync();
        continue;
      }
      // compact the candidates with d^2 <= hiT (in LDS order)
      int sf = 0;
#pragma unroll
      for (int r = 0; r < EPLL; ++r) {
        const int e = lane + 64 * r;
        const bool keep = e < fill && dl[r] <= hiT;
        uint64_t m;
        const int pre = ballot_prefix(keep, &m);
        if (keep) {
          sd[sf + pre] = dl[r];
          si[sf + pre] = ci[e];
        }
        sf += __popcll(m);
      }
      wave_lds_sync();
      bd = sd;
      bi = si;
      nb = sf;
    }
    if (nb <= 64 * EH)
      knn_sort_write<EH>(bd, bi, nb, k, t, eps_mult, col, eps, lane);
    else
      knn_sort_write<EPLS>(bd, bi, nb, k, t, eps_mult, col, eps, lane);
    wave_lds_sync();  // the buffers are refilled for the next target
  }
  if (npend > 0) flush_slow();
}

// The two register passes for k (block radius 2, then 3 for the targets the
// first could not settle); false when k is beyond the register path.
template <int DIM, int L1, int L2, int S>
static void knn_reg_passes(const GridParams *gp, const SPoint *pts, const int *start, const double *targets,
                           const int *order, int64_t n_tgt, int k, double mult, int32_t *col, double *eps,
                           int *lists, int64_t stride, unsigned nb, hipStream_t s) {
  k_knn_reg<DIM, L1, S><<<nb, 64, 0, s>>>(gp, pts, start, targets, order, nullptr, n_tgt, 2, k, mult, col, eps,
                                          lists + 1, lists);
  k_knn_reg<DIM, L2, S><<<nb, 64, 0, s>>>(gp, pts, start, targets, lists + 1, lists, n_tgt, 3, k, mult, col, eps,
                                          lists + stride + 1, lists + stride);
}

template <int DIM>
static bool launch_knn_reg(const GridParams *gp, const SPoint *pts, const int *start, const double *targets,
                           const int *order, int64_t n_tgt, int k, double mult, int32_t *col, double *eps,
                           int *lists, int64_t stride, unsigned nb, hipStream_t s) {
  // <L1, L2, S>: the first pass keeps up to 64*L1 candidates within the
  // block's margin, the second up to 64*L2; the register sort holds 64*S
  // pairs (k <= 64*S; half of it when k fits there).  The capacities are the
  // smallest that settle nearly every target of a cloud (interior or on its
  // boundary) in the two passes: larger ones cost registers and bisection
  // work on every target
  if (k <= 16)
    knn_reg_passes<DIM, 1, 4, 1>(gp, pts, start, targets, order, n_tgt, k, mult, col, eps, lists, stride, nb, s);
  else if (k <= 32)
    knn_reg_passes<DIM, 2, 8, 1>(gp, pts, start, targets, order, n_tgt, k, mult, col, eps, lists, stride, nb, s);
  else if (k <= 48)
    knn_reg_passes<DIM, 4, 8, 1>(gp, pts, start, targets, order, n_tgt, k, mult, col, eps, lists, stride, nb, s);
  else if (k <= 64)
    knn_reg_passes<DIM, 4, 8, 2>(gp, pts, start, targets, order, n_tgt, k, mult, col, eps, lists, stride, nb, s);
  else if (k <= 96)
    knn_reg_passes<DIM, 4, 8, 4>(gp, pts, start, targets, order, n_tgt, k, mult, col, eps, lists, stride, nb, s);
  else if (k <= 192)
    knn_reg_passes<DIM, 8, 16, 4>(gp, pts, start, targets, order, n_tgt, k, mult, col, eps, lists, stride, nb, s);
  else if (k <= 256)
    knn_reg_passes<DIM, 16, 32, 8>(gp, pts, start, targets, order, n_tgt, k, mult, col, eps, lists, stride, nb,
                                   s);
  else
    return false;
  return true;
}

// per-target expanding kNN for the targets of a list
template <int DIM>
__global__ __launch_bounds__(64) void k_knn_list(const GridParams *gp, const SPoint *pts, const int *cell_start,
                                                 const double *targets, const int *list, const int *n_list,
                                                 int64_t n_tgt, int k, double eps_mult, int32_t *col, double *eps) {
  __shared__ double d2[kCap];
  __shared__ int idx[kCap];
  const GridParams g = *gp;
  const int64_t n = n_list ? (int64_t)readfirstlane_i(*n_list) : n_tgt;
  for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
    const int t = readfirstlane_i(list[w]);
    double x[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) x[d] = uniform_d(targets[(int64_t)t * DIM + d]);
    const int got = knn_select<DIM, kCap>(g, pts, cell_start, x, k, 2, d2, idx);
    for (int q = lane_id(); q < k; q += 64) col[(int64_t)t * k + q] = q < got ? idx[q] : -1;
    if (lane_id() == 0) eps[t] = eps_mult * sqrt(d2[got - 1]);
    __syncthreads();
  }
}

constexpr int kSmallCap = 256;      // row entries sorted in registers
constexpr int kCellCap = 1280;      // candidates of one cell block staged in LDS
constexpr int kCellThreads = 256;   // four wavefronts share a cell block
constexpr int kMaxRuns = 9;         // runs of cells along x in a 3x3(x3) block
// targets a wavefront tests together: 4 in cell order; 2 when the rows are
// sorted (their LDS buffers, 1 KiB per target, limit the occupancy)
template <bool SORTED>
constexpr int cell_targets() { return SORTED ? 2 : 4; }

// ---------------------------------------------------------------------------
// radius search, cell-cooperative: a workgroup takes one target cell, stages
// the sources of its (2R+1)^DIM block of cells in LDS once, and its four
// wavefronts share the cell's targets (one target per wavefront at a time,
// the candidates 64 per step).  Modes:
//  kCount: row lengths only;
//  kFill:  rows of up to kSmallCap entries (floor not needed) are sorted by
//          index in registers and written at row_ptr[t];
//  kFused: one pass: such rows go to a scratch row of kSmallCap entries per
//          target, every processed target's length to counts[t], and the
//          rows are copied into place after the scan (k_rows_copy).
// Targets of cells whose block exceeds kCellCap sources, and (fill and fused
// modes) targets needing the k_min floor or a longer row, are appended to
// `defer` (and flagged in dflag) for the per-target kernels below.
// ---------------------------------------------------------------------------
enum RadiusMode { kCount = 0, kFill = 1, kFused = 2 };

template <int DIM, int MODE, bool SORTED>
__global__ __launch_bounds__(kCellThreads) void k_radius_cells(const GridParams *gp, const SPoint *pts,
                                                               const int *cell_start, const int *tcs,
                                                               const double *targets, const int *order, double r0,
                                                               int k_min, int64_t *counts, const int64_t *row_ptr,
                                                               int32_t *col, double *eps, int *defer, int *n_defer,
                                                               uint8_t *dflag, int *flags, int pos_rows) {
  constexpr bool ROWS = MODE != kCount;
  constexpr int NT = cell_targets<SORTED>();
  if (MODE == kFill && (*flags & 2)) return;  // over capacity: nothing is written
  __shared__ double cxyz[3][kCellCap];
  __shared__ int cid[kCellCap];
  __shared__ int cbuf[kCellThreads / 64][NT][ROWS && SORTED ? kSmallCap : 1];
  const GridParams g = *gp;
  const int tid = threadIdx.x, lane = tid & 63, wv = readfirstlane_i(tid >> 6);
  const double r2 = r0 * r0;
  const int R = radius_blocks(g, r0);
  for (int c = xcd_block(); c < g.ncell; c += gridDim.x) {
    const int tb = tcs[c], te = tcs[c + 1];
    if (tb == te) continue;
    if (R > 1) {  // cells narrower than the radius: more runs than staged here
      for (int i = tb + tid; i < te; i += kCellThreads) {
        defer[atomicAdd(n_defer, 1)] = order[i];
        if (MODE == kFused) dflag[order[i]] = 1;
      }
      continue;
    }
    const int ic[3] = {c % g.nc[0], (c / g.nc[0]) % g.nc[1], c / (g.nc[0] * g.nc[1])};
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) {
      lo[d] = max(ic[d] - R, 0);
      hi[d] = min(ic[d] + R, g.nc[d] - 1);
    }
    // the block's runs of cells along x: all bounds requested at once, then
    // every source of every run (one memory round trip each)
    const int ny = hi[1] - lo[1] + 1, nrun = ny * (hi[2] - lo[2] + 1);
    int rb[kMaxRuns], pre[kMaxRuns + 1];
    pre[0] = 0;
#pragma unroll
    for (int q = 0; q < kMaxRuns; ++q) {
      int b = 0, e = 0;
      if (q < nrun) {
        const int row = g.nc[0] * ((lo[1] + q % ny) + g.nc[1] * (lo[2] + q / ny));
        b = cell_start[row + lo[0]];
        e = cell_start[row + hi[0] + 1];
      }
      rb[q] = b;
      pre[q + 1] = pre[q] + (e - b);
    }
    const int total = pre[kMaxRuns];
    if (total > kCellCap) {
      for (int i = tb + tid; i < te; i += kCellThreads) {
        defer[atomicAdd(n_defer, 1)] = order[i];
        if (MODE == kFused) dflag[order[i]] = 1;
      }
      continue;
    }
    for (int e = tid; e < total; e += kCellThreads) {
      int q = 0;
#pragma unroll
      for (int u = 1; u < kMaxRuns; ++u) q += e >= pre[u] ? 1 : 0;
      int src = rb[0] + e;
#pragma unroll
      for (int u = 1; u < kMaxRuns; ++u)
        if (q == u) src = rb[u] + (e - pre[u]);
      const SPoint sp = pts[src];
      cxyz[0][e] = sp.x;
      cxyz[1][e] = sp.y;
      cxyz[2][e] = sp.z;
      cid[e] = pos_rows ? src : sp.idx;  // the record's position, or the source index
    }
    // this wavefront's targets (every fourth of the cell), fetched by its
    // lanes together, 64 at a time, then taken NT at a time: each staged
    // candidate is read from LDS once for the NT targets, and their NT row
    // sorts run interleaved (independent exchange chains)
    constexpr int NW = kCellThreads / 64;
    int my_t = 0;
    double my_x[3] = {0, 0, 0};
    __syncthreads();
    for (int j = 0; tb + wv + NW * j < te; j += NT) {
      if ((j & 63) == 0) {
        const int i = tb + wv + NW * (j + lane);
        my_t = i < te ? order[i] : 0;
        for (int d = 0; d < DIM; ++d) my_x[d] = i < te ? targets[(int64_t)my_t * DIM + d] : 0.0;
      }
      int t[NT];
      bool live[NT];
      double x[NT][3];
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        live[u] = tb + wv + NW * (j + u) < te;
        t[u] = readlane_i(my_t, (j + u) & 63);
#pragma unroll
        for (int d = 0; d < 3; ++d) x[u][d] = d < DIM ? readlane_d(my_x[d], (j + u) & 63) : 0.0;
      }
      unsigned fill[NT];  // row entries found so far (wave-uniform)
      int cnt[NT];
      int32_t *out[NT];
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        fill[u] = 0;
        cnt[u] = 0;
        if constexpr (ROWS)
          out[u] = MODE == kFused ? col + (int64_t)t[u] * kSmallCap : col + (live[u] ? row_ptr[t[u]] : 0);
      }
      for (int k0 = 0; k0 < total; k0 += 64) {
        const int k = k0 + lane;
        // a lane past the staged block tests a point at NaN, whose squared
        // distance compares false: it is never accepted
        const double nan = __builtin_nan("");
        double c[3] = {nan, nan, nan};
        int id = 0;
        if (k < total) {
          for (int d = 0; d < DIM; ++d) c[d] = cxyz[d][k];
          if constexpr (ROWS) id = cid[k];
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          if (!live[u]) continue;
          // (dx*dx + dy*dy) + dz*dz, unfused (the file is built without contraction)
          const double dx = c[0] - x[u][0];
          double dd = dx * dx;
          if (DIM > 1) {
            const double dy = c[1] - x[u][1];
            dd = dd + dy * dy;
          }
          if (DIM > 2) {
            const double dz = c[2] - x[u][2];
            dd = dd + dz * dz;
          }
          const bool ok = dd < r2;
          if constexpr (ROWS) {
            // a row of more than kSmallCap entries goes to the per-target
            // kernels, which write it again: once a row overflows, nothing
            // more of it is stored (a wave-uniform test, no per-lane bound)
            const uint64_t m = __ballot(ok);
            const unsigned nf = __builtin_amdgcn_readfirstlane(fill[u] + (unsigned)__popcll(m));
            if (ok && nf <= (unsigned)kSmallCap) {
              const unsigned slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)m, fill[u]));
              if constexpr (SORTED)
                cbuf[wv][u][slot] = id;
              else
                out[u][slot] = id;  // staging order is cell order: the row is final
            }
            fill[u] = nf;
          } else {
            cnt[u] += ok ? 1 : 0;
          }
        }
      }
      if constexpr (!ROWS) {
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          const int f = wave_sum(cnt[u]);
          if (lane == 0 && live[u]) {
            if (f > kCap) atomicOr(flags, 1);
            counts[t[u]] = f < k_min ? k_min : (f > kCap ? kCap : f);
          }
        }
      } else {
        // rows that go to the per-target kernels; the others are sorted
        int n_sort[NT];
        bool here[NT];  // finished by this kernel (an empty row included, when k_min is 0)
        int widest = 0;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          const bool defer_it = live[u] && (fill[u] < (unsigned)k_min || fill[u] > (unsigned)kSmallCap);
          here[u] = live[u] && !defer_it;
          n_sort[u] = here[u] ? fill[u] : 0;
          widest = max(widest, n_sort[u]);
          if (defer_it && lane == 0) {
            defer[atomicAdd(n_defer, 1)] = t[u];
            if (MODE == kFused) {
              dflag[t[u]] = 1;
              if (fill[u] > kCap) atomicOr(flags, 1);
              counts[t[u]] = fill[u] < k_min ? k_min : (fill[u] > kCap ? kCap : fill[u]);
            }
          }
        }
        if constexpr (SORTED) {
          wave_lds_sync();
          if (widest <= 64)
            sort_idx_multi<1, NT>(cbuf[wv], n_sort, out, lane);
          else if (widest <= 128)
            sort_idx_multi<2, NT>(cbuf[wv], n_sort, out, lane);
          else
            sort_idx_multi<4, NT>(cbuf[wv], n_sort, out, lane);
        }
        if (lane == 0) {
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            if (!here[u]) continue;
            eps[t[u]] = r0;
            if (MODE == kFused) {
              counts[t[u]] = n_sort[u];
              dflag[t[u]] = 0;
            }
          }
        }
        if constexpr (SORTED) wave_lds_sync();  // the buffers are refilled for the next targets
      }
    }
    __syncthreads();  // the next cell restages the candidates
  }
}

// Capture-safe mode: flag (bit 2) a total row count over the capacity.
__global__ void k_check_capacity(const int64_t *nnz, int64_t capacity, int *flags) {
  if (threadIdx.x == 0 && *nnz > capacity) atomicOr(flags, 2);
}

// Rows of the fused pass into place: 16 lanes per target, 16*kCopyLoads
// entries per step (that many loads in flight per lane before the stores, so
// that most rows take one memory round trip; consecutive lanes take
// consecutive entries, so loads and stores stay contiguous).
constexpr int kCopyLoads = 8;
__global__ __launch_bounds__(256) void k_rows_copy(int64_t n_tgt, const int64_t *row_ptr, const int32_t *rows,
                                                   const uint8_t *dflag, int32_t *col, const int *flags,
                                                   const SPoint *sorted, int32_t *pcol, const int *order) {
  if (*flags & 2) return;  // over capacity: nothing is written
  const int sub = threadIdx.x & 15;
  const int64_t g0 = (int64_t)blockIdx.x * (blockDim.x >> 4) + (threadIdx.x >> 4);
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 4);
  for (int64_t i = g0; i < n_tgt; i += stride) {
    // with record positions, targets in cell order, so that neighbouring
    // groups read the same records
    const int64_t t = pcol ? order[i] : i;
    if (dflag[t]) continue;
    const int64_t b = row_ptr[t];
    const int n = (int)(row_ptr[t + 1] - b);
    const int32_t *src = rows + t * kSmallCap;
    for (int q0 = 0; q0 < n; q0 += 16 * kCopyLoads) {
      int32_t v[kCopyLoads];
#pragma unroll
      for (int u = 0; u < kCopyLoads; ++u) {
        const int q = q0 + 16 * u + sub;
        v[u] = q < n ? src[q] : 0;
      }
      if (pcol) {
        // the scratch rows hold record positions: the source index is the
        // record's (the positions of a row are a few runs of nearby records)
        int32_t id[kCopyLoads];
#pragma unroll
        for (int u = 0; u < kCopyLoads; ++u) id[u] = q0 + 16 * u + sub < n ? sorted[v[u]].idx : 0;
#pragma unroll
        for (int u = 0; u < kCopyLoads; ++u) {
          const int q = q0 + 16 * u + sub;
          if (q < n) {
            pcol[b + q] = v[u];
            col[b + q] = id[u];
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < kCopyLoads; ++u) {
          const int q = q0 + 16 * u + sub;
          if (q < n) col[b + q] = v[u];
        }
      }
    }
  }
}

// Record positions of the rows written with source indices (every row, or
// those flagged in dflag): pcol[j] = pos[col[j]], pos the inverse of the
// record order.  16 lanes per target, as k_rows_copy.
__global__ __launch_bounds__(256) void k_rows_pos(int64_t n_tgt, const int64_t *row_ptr, const int32_t *col,
                                                  const uint8_t *dflag, const int *pos, int32_t *pcol,
                                                  const int *flags) {
  if (*flags & 2) return;  // over capacity: nothing was written
  const int sub = threadIdx.x & 15;
  const int64_t g0 = (int64_t)blockIdx.x * (blockDim.x >> 4) + (threadIdx.x >> 4);
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 4);
  for (int64_t t = g0; t < n_tgt; t += stride) {
    if (dflag && !dflag[t]) continue;
    const int64_t b = row_ptr[t];
    const int n = (int)(row_ptr[t + 1] - b);
    for (int q = sub; q < n; q += 16) pcol[b + q] = pos[col[b + q]];
  }
}

// pos[idx] = position of the source's record; the records handed out as
// (x, y, z, index) doubles
__global__ void k_source_records(const SPoint *sorted, int64_t n, int *pos, double *rec) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const SPoint p = sorted[j];
    pos[p.idx] = (int)j;
    if (rec) {
      double4 r;
      r.x = p.x;
      r.y = p.y;
      r.z = p.z;
      r.w = (double)p.idx;
      *(double4 *)(rec + 4 * j) = r;
    }
  }
}

// ---------------------------------------------------------------------------
// per-target radius kernels for the deferred targets (one wavefront each,
// candidates read from the cell-ordered sources 64 at a time)
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(64) void k_radius_count_list(const GridParams *gp, const SPoint *pts,
                                                          const int *cell_start, const double *targets,
                                                          const int *list, const int *n_list, double r0, int k_min,
                                                          int64_t *counts, int *flags) {
  const GridParams g = *gp;
  const int lane = lane_id();
  const double r2 = r0 * r0;
  const int R = radius_blocks(g, r0);
  const int n = readfirstlane_i(*n_list);
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int t = readfirstlane_i(list[w]);
    double x[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) x[d] = uniform_d(targets[(int64_t)t * DIM + d]);
    int lo[3], hi[3];
    radius_block<DIM>(g, x, R, lo, hi);
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
    if (lane == 0) {
      if (count > kCap) atomicOr(flags, 1);
      counts[t] = count < k_min ? k_min : (count > kCap ? kCap : count);
    }
  }
}

// Cell order of a floored row (the k nearest, in idx[0, k) of a one-wavefront
// block): sort by (cell of the source, index), the order the staged scans
// produce for the other rows.  d2 is overwritten with the cell numbers.
template <int DIM>
__device__ void floor_cell_order(const GridParams &g, const double *coords, int k, double *d2, int *idx) {
  __syncthreads();
  for (int q = lane_id(); q < k; q += 64) d2[q] = (double)cell_id<DIM>(g, coords + (int64_t)idx[q] * DIM);
  __syncthreads();
  lds_sort(d2, idx, k);
}

// Deferred targets of the fill pass: rows of up to kSmallCap entries, or the
// k_min floor when it fits the small buffer; everything else goes on to
// k_radius_fill_big through `overflow`.
template <int DIM, bool SORTED>
__global__ __launch_bounds__(64) void k_radius_fill_list(const GridParams *gp, const SPoint *pts,
                                                         const int *cell_start, const double *coords,
                                                         const double *targets, const int *list, const int *n_list,
                                                         double r0, int k_min, const int64_t *row_ptr, int32_t *col,
                                                         double *eps, int *overflow, int *n_overflow,
                                                         const int *flags) {
  if (*flags & 2) return;  // over capacity: nothing is written
  __shared__ double d2[kSmallCap];
  __shared__ int idx[kSmallCap];
  const GridParams g = *gp;
  const int lane = lane_id();
  const double r2 = r0 * r0;
  const int R = radius_blocks(g, r0);
  const int n = readfirstlane_i(*n_list);
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int t = readfirstlane_i(list[w]);
    double x[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) x[d] = uniform_d(targets[(int64_t)t * DIM + d]);
    int lo[3], hi[3];
    radius_block<DIM>(g, x, R, lo, hi);
    int fill = 0;
    for (int cz = lo[2]; cz <= hi[2]; ++cz)
      for (int cy = lo[1]; cy <= hi[1]; ++cy) {
        const int row = g.nc[0] * (cy + g.nc[1] * cz);
        const int beg = readfirstlane_i(cell_start[row + lo[0]]);
        const int end = readfirstlane_i(cell_start[row + hi[0] + 1]);
        for (int b = beg; b < end; b += 64) {
          const int p = b + lane;
          bool ok = false;
          int id = 0;
          if (p < end) {
            const SPoint sp = pts[p];
            ok = dist2_exact<DIM>(sp, x) < r2;
            id = sp.idx;
          }
          uint64_t m;
          const int pre = ballot_prefix(ok, &m);
          if (ok && fill + pre < kSmallCap) idx[fill + pre] = id;
          fill += __popcll(m);
        }
      }
    const bool big = fill > kSmallCap || (fill < k_min && k_min + 65 > kSmallCap);
    if (big) {
      if (lane == 0) overflow[atomicAdd(n_overflow, 1)] = t;
      __syncthreads();
      continue;
    }
    const int64_t base = row_ptr[t];
    __syncthreads();
    if (fill >= k_min) {
      if constexpr (SORTED)
        sort_idx_any(idx, fill, col + base, lane);
      else
        for (int q = lane; q < fill; q += 64) col[base + q] = idx[q];
      if (lane == 0) eps[t] = r0;
    } else {
      const int got = knn_select<DIM, kSmallCap>(g, pts, cell_start, x, k_min + 1, 1, d2, idx);
      __syncthreads();
      const double e = got > k_min ? 0.5 * (sqrt(d2[k_min - 1]) + sqrt(d2[k_min])) : r0;
      if constexpr (SORTED) {
        sort_idx_any(idx, k_min, col + base, lane);
      } else {
        floor_cell_order<DIM>(g, coords, k_min, d2, idx);
        for (int q = lane; q < k_min; q += 64) col[base + q] = idx[q];
      }
      if (lane == 0) eps[t] = e;
    }
    __syncthreads();
  }
}

// Targets with more candidates than the small buffer (or a large floor):
// LDS buffer of kCap entries and a bitonic sort in LDS.
template <int DIM, bool SORTED>
__global__ __launch_bounds__(64) void k_radius_fill_big(const GridParams *gp, const SPoint *pts,
                                                        const int *cell_start, const double *coords,
                                                        const double *targets, double r0, int k_min,
                                                        const int64_t *row_ptr, int32_t *col, double *eps,
                                                        const int *overflow, const int *n_overflow, const int *flags) {
  if (*flags & 2) return;  // over capacity: nothing is written
  __shared__ double d2[kCap];
  __shared__ int idx[kCap];
  const GridParams g = *gp;
  const int lane = lane_id();
  const double r2 = r0 * r0;
  const int R = radius_blocks(g, r0);
  const int n = readfirstlane_i(*n_overflow);
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int t = readfirstlane_i(overflow[w]);
    double x[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) x[d] = uniform_d(targets[(int64_t)t * DIM + d]);
    int lo[3], hi[3];
    radius_block<DIM>(g, x, R, lo, hi);
    int fill = 0;
    for (int cz = lo[2]; cz <= hi[2]; ++cz)
      for (int cy = lo[1]; cy <= hi[1]; ++cy) {
        const int row = g.nc[0] * (cy + g.nc[1] * cz);
        const int beg = readfirstlane_i(cell_start[row + lo[0]]);
        const int end = readfirstlane_i(cell_start[row + hi[0] + 1]);
        for (int b = beg; b < end; b += 64) {
          const int p = b + lane;
          bool ok = false;
          int id = 0;
          if (p < end) {
            const SPoint sp = pts[p];
            ok = dist2_exact<DIM>(sp, x) < r2;
            id = sp.idx;
          }
          uint64_t m;
          const int pre = ballot_prefix(ok, &m);
          if (ok && fill + pre < kCap) idx[fill + pre] = id;
          fill += __popcll(m);
        }
      }
    const int64_t base = row_ptr[t];
    __syncthreads();
    if (fill >= k_min) {
      if (fill > kCap) fill = kCap;  // flagged by the count pass; the call fails
      if constexpr (SORTED) lds_sort_int(idx, fill);
      for (int q = lane; q < fill; q += 64) col[base + q] = idx[q];
      if (lane == 0) eps[t] = r0;
    } else {
      const int got = knn_select<DIM, kCap>(g, pts, cell_start, x, k_min + 1, 1, d2, idx);
      __syncthreads();
      const double e = got > k_min ? 0.5 * (sqrt(d2[k_min - 1]) + sqrt(d2[k_min])) : r0;
      __syncthreads();
      if constexpr (SORTED)
        lds_sort_int(idx, k_min);
      else
        floor_cell_order<DIM>(g, coords, k_min, d2, idx);
      for (int q = lane; q < k_min; q += 64) col[base + q] = idx[q];
      if (lane == 0) eps[t] = e;
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

// launches with the row order chosen at run time (cell order, or ascending
// index with a sort per row)
template <int DIM, int MODE, typename... A>
static void launch_cells(bool by_index, unsigned nb, hipStream_t s, A... args) {
  if (by_index)
    k_radius_cells<DIM, MODE, true><<<nb, kCellThreads, 0, s>>>(args...);
  else
    k_radius_cells<DIM, MODE, false><<<nb, kCellThreads, 0, s>>>(args...);
}

template <int DIM, typename... A>
static void launch_fill_list(bool by_index, hipStream_t s, A... args) {
  if (by_index)
    k_radius_fill_list<DIM, true><<<4096, 64, 0, s>>>(args...);
  else
    k_radius_fill_list<DIM, false><<<4096, 64, 0, s>>>(args...);
}

template <int DIM, typename... A>
static void launch_fill_big(bool by_index, hipStream_t s, A... args) {
  if (by_index)
    k_radius_fill_big<DIM, true><<<1024, 64, 0, s>>>(args...);
  else
    k_radius_fill_big<DIM, false><<<1024, 64, 0, s>>>(args...);
}

// GPU time of the search just finished (events 4 and 5 of the context)
static void search_time(gmls_ctx ctx) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ctx->ev[4], ctx->ev[5]) == hipSuccess) ctx->t_search_ms = ms;
  (void)hipGetLastError();
}

template <int DIM>
static gmls_status neighbors_dim(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                                 int64_t n_tgt, const gmls_search &spec, int64_t *row_ptr, int32_t *col,
                                 int64_t col_capacity, double *eps, int64_t *nnz_host, double *records,
                                 int32_t *pcol) {
  hipStream_t s = ctx->stream;
  const bool knn = spec.mode == GMLS_SEARCH_KNN;
  const bool sync = !ctx->opt.capture_safe;  // capture-safe: nothing below waits for the device
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

  ctx->t_search_ms = 0.0;
  if (sync) GMLS_HIP(hipEventRecord(ctx->ev[4], s));
  k_bbox_partial<<<nb_bbox, kBBoxBlock, 0, s>>>(coords, n_src, DIM, bbox);
  k_grid_setup<<<1, 64, 0, s>>>(bbox, (int)nb_bbox, DIM, knn ? 0 : 1, spec.radius, spec.k, n_src, ncell_max, gp);
  GMLS_HIP(fill_zero(cnt, sizeof(int) * (size_t)(ncell_max + 1), s));
  GMLS_HIP(fill_zero(flags, sizeof(int) * 4, s));
  k_cell_keys<DIM><<<grid_for(n_src, 256), 256, 0, s>>>(gp, coords, n_src, key, cnt);
  GMLS_HIP(exclusive_scan<int, int>(cnt, start, ncell_max, (int *)tmp, s));
  GMLS_HIP(fill_zero(cnt, sizeof(int) * (size_t)(ncell_max + 1), s));
  const bool by_index = ctx->opt.row_order != 0;
  if ((!knn && !by_index) || records) {
    // radius rows come out in staging order, which is cell order once each
    // cell's sources are in ascending index (and the records handed out are
    // then the same on every call)
    GMLS_WS(scattered, SPoint, WS_SORTED_TMP, n_src);
    k_cell_scatter<DIM><<<grid_for(n_src, 256), 256, 0, s>>>(coords, n_src, key, start, cnt, scattered);
    k_cell_sort<<<(unsigned)xcd_grid(ctx->cus * 32), 64, 0, s>>>(gp, start, scattered, sorted);
  } else {
    k_cell_scatter<DIM><<<grid_for(n_src, 256), 256, 0, s>>>(coords, n_src, key, start, cnt, sorted);
  }
  GMLS_HIP(hipGetLastError());
  int *pos = nullptr;  // source index -> record position
  if (records) {
    pos = (int *)ctx->ws(WS_SRC_POS, sizeof(int) * (size_t)n_src);
    if (!pos) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed (positions)");
    k_source_records<<<grid_for(n_src, 256), 256, 0, s>>>(sorted, n_src, pos, records);
  }
  const int *tcs = start;  // target ranges per cell in `order`
  if (n_tgt > 0) {
    if (targets == coords && n_tgt == n_src) {
      k_sorted_order<<<grid_for(n_tgt, 256), 256, 0, s>>>(sorted, n_tgt, order);
    } else {
      GMLS_WS(tkey, int, WS_TGT_KEY, n_tgt);
      GMLS_WS(tcnt, int, WS_TGT_COUNT, ncell_max + 1);
      GMLS_WS(tstart, int, WS_TGT_START, ncell_max + 1);
      GMLS_HIP(fill_zero(tcnt, sizeof(int) * (size_t)(ncell_max + 1), s));
      k_cell_keys<DIM><<<grid_for(n_tgt, 256), 256, 0, s>>>(gp, targets, n_tgt, tkey, tcnt);
      GMLS_HIP(exclusive_scan<int, int>(tcnt, tstart, ncell_max, (int *)tmp, s));
      GMLS_HIP(fill_zero(tcnt, sizeof(int) * (size_t)(ncell_max + 1), s));
      k_index_scatter<<<grid_for(n_tgt, 256), 256, 0, s>>>(n_tgt, tkey, tstart, tcnt, order);
      tcs = tstart;
    }
    GMLS_HIP(hipGetLastError());
  }
  if (knn) {
    k_knn_rowptr<<<grid_for(n_tgt + 1, 256), 256, 0, s>>>(n_tgt, spec.k, row_ptr);
    if (n_tgt > 0) {
      // two register passes, then the expanding kernel for what is left;
      // lists[0] and lists[stride] count the targets left by each pass
      const int64_t stride = n_tgt + 1;
      GMLS_WS(lists, int, WS_DEFER, 2 * stride);
      GMLS_HIP(fill_zero(lists, sizeof(int), s));
      GMLS_HIP(fill_zero(lists + stride, sizeof(int), s));
      const unsigned nb = (unsigned)xcd_grid(ctx->cus * 64);
      const int *left = lists + stride;
      if (!launch_knn_reg<DIM>(gp, sorted, start, targets, order, n_tgt, spec.k, spec.eps_mult, col, eps, lists,
                               stride, nb, s))
        left = nullptr;  // k beyond the register path: every target expands
      if (left)
        k_knn_list<DIM><<<4096, 64, 0, s>>>(gp, sorted, start, targets, left + 1, left, n_tgt, spec.k,
                                            spec.eps_mult, col, eps);
      else
        k_knn_list<DIM><<<4096, 64, 0, s>>>(gp, sorted, start, targets, order, nullptr, n_tgt, spec.k,
                                            spec.eps_mult, col, eps);
      if (pcol) k_rows_pos<<<grid_for(n_tgt, 16), 256, 0, s>>>(n_tgt, row_ptr, col, nullptr, pos, pcol, flags);
    }
    GMLS_HIP(hipGetLastError());
    if (sync) {
      GMLS_HIP(hipEventRecord(ctx->ev[5], s));
      GMLS_HIP(hipStreamSynchronize(s));
      search_time(ctx);
    }
    return GMLS_OK;
  }
  GMLS_WS(counts, int64_t, WS_ROW_COUNT, n_tgt > 0 ? n_tgt : 1);
  GMLS_WS(defer, int, WS_DEFER, 2 * (n_tgt > 0 ? n_tgt : 1));
  // flags: [0] error bits, [1] overflow count, [2] deferred (count pass), [3] deferred (fill pass)
  const int cus = ctx->cus;
  const unsigned nb_cells = (unsigned)xcd_grid(cus * 6);
  // one pass with a scratch row per target when that fits the budget,
  // otherwise a count pass and a fill pass
  const bool fused = (double)n_tgt * kSmallCap * sizeof(int32_t) <= (double)ctx->opt.radius_scratch_mb * (1 << 20);
  int32_t *rows = nullptr;
  uint8_t *dflag = nullptr;
  if (fused && n_tgt > 0) {
    rows = (int32_t *)ctx->ws(WS_RADIUS_ROWS, sizeof(int32_t) * (size_t)n_tgt * kSmallCap);
    dflag = (uint8_t *)ctx->ws(WS_TGT_FLAG, (size_t)n_tgt);
    if (!rows || !dflag) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed (rows)");
  }
  // the one-pass search in cell order writes record positions to its scratch
  // rows when they are asked for; the other paths translate finished rows
  const int pos_rows = (pcol && fused && !by_index) ? 1 : 0;
  if (n_tgt > 0) {
    if (fused)
      launch_cells<DIM, kFused>(by_index, nb_cells, s, (const GridParams *)gp, (const SPoint *)sorted, start, tcs,
                                targets, (const int *)order, spec.radius, spec.k_min, counts,
                                (const int64_t *)nullptr, rows, eps, defer, flags + 2, dflag, flags, pos_rows);
    else
      launch_cells<DIM, kCount>(by_index, nb_cells, s, (const GridParams *)gp, (const SPoint *)sorted, start, tcs,
                                targets, (const int *)order, spec.radius, spec.k_min, counts,
                                (const int64_t *)nullptr, (int32_t *)nullptr, (double *)nullptr, defer, flags + 2,
                                (uint8_t *)nullptr, flags, 0);
    k_radius_count_list<DIM><<<4096, 64, 0, s>>>(gp, sorted, start, targets, defer, flags + 2, spec.radius,
                                                 spec.k_min, counts, flags);
  }
  GMLS_HIP(exclusive_scan<int64_t, int64_t>(counts, row_ptr, n_tgt, tmp, s));
  if (sync) {
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
  } else {
    // the size is known on the device only: the kernels that write `col`
    // skip their writes when it exceeds the capacity (flag bit 2)
    *nnz_host = -1;
    k_check_capacity<<<1, 64, 0, s>>>(row_ptr + n_tgt, col_capacity, flags);
  }
  if (n_tgt > 0) {
    int *defer_fill = defer;
    int *n_defer_fill = flags + 2;
    int *overflow = (int *)counts;  // the counts are consumed by the scan
    if (fused) {
      k_rows_copy<<<grid_for(n_tgt, 16), 256, 0, s>>>(n_tgt, row_ptr, rows, dflag, col, flags,
                                                       (const SPoint *)sorted, pos_rows ? pcol : nullptr,
                                                       (const int *)order);
    } else {
      defer_fill = defer + n_tgt;
      n_defer_fill = flags + 3;
      launch_cells<DIM, kFill>(by_index, nb_cells, s, (const GridParams *)gp, (const SPoint *)sorted, start, tcs,
                               targets, (const int *)order, spec.radius, spec.k_min, (int64_t *)nullptr,
                               (const int64_t *)row_ptr, col, eps, defer_fill, n_defer_fill, (uint8_t *)nullptr,
                               flags, 0);
    }
    launch_fill_list<DIM>(by_index, s, (const GridParams *)gp, (const SPoint *)sorted, start, coords, targets,
                          (const int *)defer_fill, (const int *)n_defer_fill, spec.radius, spec.k_min,
                          (const int64_t *)row_ptr, col, eps, overflow, flags + 1, (const int *)flags);
    launch_fill_big<DIM>(by_index, s, (const GridParams *)gp, (const SPoint *)sorted, start, coords, targets,
                         spec.radius, spec.k_min, (const int64_t *)row_ptr, col, eps, (const int *)overflow,
                         (const int *)(flags + 1), (const int *)flags);
    if (pcol)  // rows written with source indices: the deferred ones, or all
      k_rows_pos<<<grid_for(n_tgt, 16), 256, 0, s>>>(n_tgt, row_ptr, col, pos_rows ? dflag : nullptr, pos, pcol,
                                                      flags);
  }
  GMLS_HIP(hipGetLastError());
  if (sync) {
    GMLS_HIP(hipEventRecord(ctx->ev[5], s));
    GMLS_HIP(hipStreamSynchronize(s));
    search_time(ctx);
  } else {
    int *de = (int *)ctx->ws(WS_DEV_ERR, sizeof(int));
    GMLS_HIP(or_error_bit(de, flags, 1, DEV_ERR_RADIUS_ROWS, s));
    GMLS_HIP(or_error_bit(de, flags, 2, DEV_ERR_CAPACITY, s));
  }
  return GMLS_OK;
}

gmls_status run_neighbors(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                          int64_t n_tgt, int dim, const gmls_search &spec, int64_t *row_ptr, int32_t *col,
                          int64_t col_capacity, double *eps, int64_t *nnz_host, double *records, int32_t *pcol) {
  switch (dim) {
    case 1:
      return neighbors_dim<1>(ctx, coords, n_src, targets, n_tgt, spec, row_ptr, col, col_capacity, eps, nnz_host,
                              records, pcol);
    case 2:
      return neighbors_dim<2>(ctx, coords, n_src, targets, n_tgt, spec, row_ptr, col, col_capacity, eps, nnz_host,
                              records, pcol);
    case 3:
      return neighbors_dim<3>(ctx, coords, n_src, targets, n_tgt, spec, row_ptr, col, col_capacity, eps, nnz_host,
                              records, pcol);
    default:
      return gmls_set_error(ctx, GMLS_ERR_ARG, "dim must be 1, 2 or 3");
  }
}

}  // namespace gmls
