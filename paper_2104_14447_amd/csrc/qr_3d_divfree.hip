// FP64 QR stencil kernels for dim 3, divergence-free basis (instantiations).
#include "stencil_fp64.hpp"

namespace gmls {

template <int DIM, int ORDER, int BASIS>
static hipError_t launch_qr_rpl(int rpl, const StencilArgs &a, const int *list, const int *count,
                                const int *offset, int *cursor, int n_blocks, hipStream_t s) {
  switch (rpl) {
    case 1: k_qr<DIM, ORDER, BASIS, 1><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
    case 2: k_qr<DIM, ORDER, BASIS, 2><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
    case 3: k_qr<DIM, ORDER, BASIS, 3><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
    default: k_qr<DIM, ORDER, BASIS, 4><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
  }
  return hipGetLastError();
}

hipError_t launch_qr_3d_divfree(int order, int rpl, const StencilArgs &a, const int *list, const int *count, const int *offset,
                     int *cursor, int n_blocks, hipStream_t s) {
  switch (order) {
    case 1: return launch_qr_rpl<3, 1, 1>(rpl, a, list, count, offset, cursor, n_blocks, s);
    case 2: return launch_qr_rpl<3, 2, 1>(rpl, a, list, count, offset, cursor, n_blocks, s);
    case 3: return launch_qr_rpl<3, 3, 1>(rpl, a, list, count, offset, cursor, n_blocks, s);
    case 4: return launch_qr_rpl<3, 4, 1>(rpl, a, list, count, offset, cursor, n_blocks, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gmls
