// assemble.hip -- the global Stokes operator of Section 3.2 from stencils,
// and a CSR matrix-vector product.
//
// Unknowns and rows: velocity v_(J,c) at J*d + c, pressure phi_J at d*n + J,
// the zero-mean multiplier lambda at d*n + n.  Rows (nu the viscosity):
//   velocity, interior I, component c:
//       -nu sum_j sum_c' L^v_(I,c,j,c') v_(J,c') + sum_j G_(I,c,j) phi_J
//   velocity, boundary I:  v_(I,c)                         (Dirichlet)
//   pressure, interior I:  sum_j L^s_(I,j) phi_J + tau_I phi_I + lambda
//   pressure, boundary I:  nu beta_I sum_j sum_c' (n_I . L^v_(I,.,j,c')) v_(J,c')
//                          + sum_j L^n_(I,j) phi_J + lambda
//   multiplier:            sum_J phi_J
// with L^v the divergence-free vector Laplacian, G the scalar gradient, L^s
// the staggered Laplacian with target weight tau, L^n the Neumann-constrained
// Laplacian with h-weight beta (Section 2.3: Laplacian phi(x_I) =
// sum_j L^n phi_j + beta_I h_I, h_I = n.f + nu n.Laplacian v(x_I)).
// A velocity row holds the K block then the G block, a pressure row the N
// block (boundary), then the L block, then the multiplier; entries follow the
// neighbour order.  One wavefront writes all rows of a particle.
#include <atomic>
#include <mutex>

#include "common.hpp"
#include "gmls_internal.hpp"

namespace gmls {

// entries of the rows of particle I: d velocity rows then its pressure row
__device__ __forceinline__ void stokes_row_lengths(const StokesArgs &s, int64_t I, int N, bool self, int64_t *vlen,
                                                   int64_t *plen) {
  const int d = s.dim;
  if (s.boundary[I]) {
    *vlen = 1;
    *plen = (int64_t)d * N + N + 1;
  } else {
    *vlen = (int64_t)d * N + N;
    *plen = N + (self ? 0 : 1) + 1;
  }
}

// whether particle I is among its own neighbours (wave-uniform)
__device__ __forceinline__ bool self_listed(const StokesArgs &s, int64_t I, int64_t rb, int N) {
  bool hit = false;
  for (int q = lane_id(); q < N; q += 64) hit = hit || s.col[rb + q] == (int32_t)I;
  return __ballot(hit) != 0;
}

__global__ __launch_bounds__(256) void k_stokes_count(StokesArgs s, int64_t *rlen) {
  const int lane = lane_id();
  const int64_t wpb = blockDim.x >> 6;
  const int d = s.dim;
  for (int64_t I = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); I < s.n; I += (int64_t)gridDim.x * wpb) {
    const int64_t rb = s.row_ptr[I];
    const int N = (int)(s.row_ptr[I + 1] - rb);
    const bool self = self_listed(s, I, rb, N);
    int64_t vlen, plen;
    stokes_row_lengths(s, I, N, self, &vlen, &plen);
    if (lane < d) rlen[I * d + lane] = vlen;
    if (lane == 0) rlen[(int64_t)d * s.n + I] = plen;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) rlen[(int64_t)d * s.n + s.n] = s.n;
}

__global__ __launch_bounds__(256) void k_stokes_fill(StokesArgs s, const int64_t *arp, int32_t *acol, double *aval,
                                                     const int *flags) {
  if (*flags) return;  // over capacity: nothing is written
  const int lane = lane_id();
  const int64_t wpb = blockDim.x >> 6;
  const int d = s.dim;
  const int64_t n = s.n;
  const int32_t pcol0 = (int32_t)(d * n);  // column of phi_0
  for (int64_t I = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); I < n; I += (int64_t)gridDim.x * wpb) {
    const int64_t rb = s.row_ptr[I];
    const int N = (int)(s.row_ptr[I + 1] - rb);
    const int32_t *nb = s.col + rb;
    const bool bnd = s.boundary[I] != 0;
    // velocity rows
    for (int c = 0; c < d; ++c) {
      const int64_t o = arp[I * d + c];
      if (bnd) {
        if (lane == 0) {
          acol[o] = (int32_t)(I * d + c);
          aval[o] = 1.0;
        }
        continue;
      }
      // K block: -nu L^v, weights (c*N + j)*d + c' of the particle's d*d*rb block
      const double *lv = s.vlap + (int64_t)d * d * rb + (int64_t)c * N * d;
      for (int q = lane; q < N * d; q += 64) {
        const int j = q / d, cp = q - j * d;
        acol[o + q] = nb[j] * d + cp;
        aval[o + q] = -s.nu * lv[q];
      }
      // G block
      const double *gr = s.grad + (int64_t)d * rb + (int64_t)c * N;
      for (int j = lane; j < N; j += 64) {
        acol[o + (int64_t)N * d + j] = pcol0 + nb[j];
        aval[o + (int64_t)N * d + j] = gr[j];
      }
    }
    // pressure row
    int64_t o = arp[d * n + I];
    if (bnd) {
      // N block: nu beta_I n_I . L^v
      const double beta = s.nlap_h[I];
      double nv[3] = {0.0, 0.0, 0.0};
      for (int c = 0; c < d; ++c) nv[c] = s.normals[I * d + c];
      const double *lv = s.vlap + (int64_t)d * d * rb;
      for (int q = lane; q < N * d; q += 64) {
        const int j = q / d, cp = q - j * d;
        double acc = 0.0;
        for (int c = 0; c < d; ++c) acc += nv[c] * lv[((int64_t)c * N + j) * d + cp];
        acol[o + q] = nb[j] * d + cp;
        aval[o + q] = s.nu * beta * acc;
      }
      o += (int64_t)N * d;
      for (int j = lane; j < N; j += 64) {
        acol[o + j] = pcol0 + nb[j];
        aval[o + j] = s.nlap[rb + j];
      }
      o += N;
    } else {
      const bool self = self_listed(s, I, rb, N);
      const double tau = s.plap_t[I];
      for (int j = lane; j < N; j += 64) {
        acol[o + j] = pcol0 + nb[j];
        aval[o + j] = s.plap[rb + j] + (nb[j] == (int32_t)I ? tau : 0.0);
      }
      o += N;
      if (!self) {
        if (lane == 0) {
          acol[o] = pcol0 + (int32_t)I;
          aval[o] = tau;
        }
        ++o;
      }
    }
    if (lane == 0) {
      acol[o] = (int32_t)(d * n + n);
      aval[o] = 1.0;
    }
  }
  // the multiplier row
  const int64_t o = arp[d * n + n];
  for (int64_t J = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; J < n; J += (int64_t)gridDim.x * blockDim.x) {
    acol[o + J] = pcol0 + (int32_t)J;
    aval[o + J] = 1.0;
  }
}

__global__ void k_stokes_check(const int64_t *arp, int64_t rows, int64_t capacity, int *flags) {
  if (threadIdx.x == 0) *flags = arp[rows] > capacity ? 1 : 0;
}

hipError_t launch_stokes_assembly(const StokesArgs &s, int64_t *rlen, int64_t *arp, int64_t *tmp, int32_t *acol,
                                  double *aval, int64_t capacity, int *flags, int cus, hipStream_t st) {
  const int64_t rows = (int64_t)s.dim * s.n + s.n + 1;
  const unsigned nb = (unsigned)xcd_grid(cus * 16);
  k_stokes_count<<<nb, 256, 0, st>>>(s, rlen);
  hipError_t e = scan_i64_exclusive(rlen, arp, rows, tmp, st);
  if (e != hipSuccess) return e;
  k_stokes_check<<<1, 64, 0, st>>>(arp, rows, capacity, flags);
  k_stokes_fill<<<nb, 256, 0, st>>>(s, arp, acol, aval, flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// y = A x for a CSR matrix: one wavefront per row (lane q takes entries q,
// q + 64, ... in order, then a butterfly sum), rows longer than kLongRow are
// handed to a 1024-thread block each (strided partial sums, then a tree
// reduction in LDS); both orders are fixed, so y is reproducible.
// ---------------------------------------------------------------------------
constexpr int kLongRow = 8192;

__global__ __launch_bounds__(256) void k_spmv(int64_t rows, const int64_t *rp, const int32_t *col, const double *val,
                                              const double *x, double *y, int *long_rows, int *n_long) {
  const int lane = lane_id();
  const int64_t wpb = blockDim.x >> 6;
  for (int64_t r = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); r < rows; r += (int64_t)gridDim.x * wpb) {
    const int64_t b = rp[r], e = rp[r + 1];
    if (e - b > kLongRow) {
      if (lane == 0) long_rows[atomicAdd(n_long, 1)] = (int)r;
      continue;
    }
    double acc = 0.0;
    for (int64_t q = b + lane; q < e; q += 64) acc += val[q] * x[col[q]];
    acc = wave_sum(acc);
    if (lane == 0) y[r] = acc;
  }
}

__global__ __launch_bounds__(1024) void k_spmv_long(const int64_t *rp, const int32_t *col, const double *val,
                                                    const double *x, double *y, const int *long_rows,
                                                    const int *n_long) {
  __shared__ double part[1024];
  const int n = *n_long;
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int64_t r = long_rows[w];
    const int64_t b = rp[r], e = rp[r + 1];
    double acc = 0.0;
    for (int64_t q = b + threadIdx.x; q < e; q += blockDim.x) acc += val[q] * x[col[q]];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = blockDim.x >> 1; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) y[r] = part[0];
    __syncthreads();
  }
}

hipError_t launch_spmv(int64_t rows, const int64_t *rp, const int32_t *col, const double *val, const double *x,
                       double *y, int *long_rows, int *n_long, int cus, hipStream_t s) {
  hipError_t e = fill_zero(n_long, sizeof(int), s);
  if (e != hipSuccess) return e;
  int64_t g = (rows + 3) / 4;
  if (g > (int64_t)cus * 64) g = (int64_t)cus * 64;
  if (g < 1) g = 1;
  k_spmv<<<(unsigned)g, 256, 0, s>>>(rows, rp, col, val, x, y, long_rows, n_long);
  k_spmv_long<<<64, 1024, 0, s>>>(rp, col, val, x, y, long_rows, n_long);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free product (gmls_spmv_noalloc): the long-row
// counter at word 0 and the long-row list from word 64 (256-byte aligned),
// room for every row of a matrix of up to kNoAllocSpmvRows rows.  Each device
// holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) int scratch[64 + kNoAllocSpmvRows];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mutex;
static std::atomic<int *> g_scratch_ptr[kMaxScratchDevices];

hipError_t spmv_scratch_setup(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  if (g_scratch_ptr[device].load(std::memory_order_acquire)) return hipSuccess;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device].load(std::memory_order_relaxed)) return hipSuccess;
  int *p = nullptr;  // the caller has made `device` current
  hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device].store(p, std::memory_order_release);
  return hipSuccess;
}

int *spmv_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  return g_scratch_ptr[device].load(std::memory_order_acquire);
}

}  // namespace gmls
