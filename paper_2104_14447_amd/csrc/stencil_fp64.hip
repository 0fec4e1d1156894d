// stencil_fp64.hip -- dispatch of the FP64 QR stencil kernels (instantiated
// per dimension and basis in qr_*.hip).
#include "gmls_internal.hpp"

namespace gmls {

hipError_t launch_qr_2d_scalar(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_3d_scalar(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_2d_divfree(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                                hipStream_t);
hipError_t launch_qr_3d_divfree(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                                hipStream_t);

static hipError_t dispatch_qr(int dim, int order, int basis, int rpl, const StencilArgs &a, const int *list,
                              const int *count, const int *offset, int *cursor, int n_blocks, hipStream_t s) {
  if (dim == 2 && basis == 0) return launch_qr_2d_scalar(order, rpl, a, list, count, offset, cursor, n_blocks, s);
  if (dim == 3 && basis == 0) return launch_qr_3d_scalar(order, rpl, a, list, count, offset, cursor, n_blocks, s);
  if (dim == 2 && basis == 1) return launch_qr_2d_divfree(order, rpl, a, list, count, offset, cursor, n_blocks, s);
  if (dim == 3 && basis == 1) return launch_qr_3d_divfree(order, rpl, a, list, count, offset, cursor, n_blocks, s);
  return hipErrorInvalidValue;
}

bool qr_supported(int dim, int order, int basis) {
  return (dim == 2 || dim == 3) && order >= 1 && order <= 4 && (basis == 0 || basis == 1);
}

hipError_t launch_qr_bin(int dim, int order, int basis, int bin, const StencilArgs &a, const int *list,
                         BinMeta *meta, int n_blocks, hipStream_t s) {
  return dispatch_qr(dim, order, basis, bin, a, list, meta->count + bin, meta->offset + bin, meta->cursor + bin,
                     n_blocks, s);
}

hipError_t launch_qr_fallback(int dim, int order, int basis, const StencilArgs &a, const int *list, BinMeta *meta,
                              int max_bin, int n_blocks, hipStream_t s) {
  return dispatch_qr(dim, order, basis, max_bin, a, list, &meta->fb_count, nullptr, &meta->fb_cursor, n_blocks, s);
}

}  // namespace gmls
