// apply.hip -- stencil application (Section 3.2: D u(x_I) ~ sum_j alpha_Ij u_j).
// One wavefront per target; each lane takes (neighbour, component) entries,
// which are contiguous in the weight layout, and the wave reduces.
#include "common.hpp"
#include "gmls_internal.hpp"

namespace gmls {

__global__ __launch_bounds__(256) void k_apply(int64_t n_tgt, const int64_t *row_ptr, const int32_t *col,
                                               const double *weights, int F, int C, const double *field,
                                               double *out) {
  const int lane = lane_id();
  const int64_t wpb = blockDim.x / 64;
  for (int64_t t = (int64_t)blockIdx.x * wpb + threadIdx.x / 64; t < n_tgt; t += (int64_t)gridDim.x * wpb) {
    const int64_t base = row_ptr[t];
    const int n = (int)(row_ptr[t + 1] - base);
    const int len = n * C;
    const double *w = weights + (int64_t)F * C * base;
    for (int f = 0; f < F; ++f) {
      double acc = 0.0;
      for (int q = lane; q < len; q += 64) {
        const int j = q / C, c = q - j * C;
        acc += w[(int64_t)f * len + q] * field[(int64_t)col[base + j] * C + c];
      }
      acc = wave_sum(acc);
      if (lane == 0) out[t * F + f] = acc;
    }
  }
}

hipError_t launch_apply(int64_t n_tgt, const int64_t *row_ptr, const int32_t *col, const double *weights, int F,
                        int C, const double *field, double *out, hipStream_t s) {
  if (n_tgt <= 0) return hipSuccess;
  int64_t g = (n_tgt + 3) / 4;
  if (g > 65536) g = 65536;
  k_apply<<<(unsigned)g, 256, 0, s>>>(n_tgt, row_ptr, col, weights, F, C, field, out);
  return hipGetLastError();
}

}  // namespace gmls
