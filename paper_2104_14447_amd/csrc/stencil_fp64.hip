// stencil_fp64.hip -- dispatch of the FP64 QR stencil kernels.  The kernels
// are instantiated per (dim, order, basis) from qr_unit.hip.
#include "gmls_internal.hpp"

namespace gmls {

hipError_t launch_qr_d2_o1_b0(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d2_o1_b1(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d2_o2_b0(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d2_o2_b1(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d2_o3_b0(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d2_o3_b1(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d2_o4_b0(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d2_o4_b1(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o1_b0(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o1_b1(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o2_b0(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o2_b1(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o3_b0(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o3_b1(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o4_b0(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o4_b1(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);

hipError_t launch_qr_d2_o1_b2(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d2_o2_b2(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d2_o3_b2(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d2_o4_b2(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o1_b2(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o2_b2(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o3_b2(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);
hipError_t launch_qr_d3_o4_b2(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int,
                               hipStream_t);

hipError_t launch_qr_kmat_d2_o1(const StencilArgs &, const int *, const int *, int *, int, hipStream_t);
hipError_t launch_qr_kmat_d2_o2(const StencilArgs &, const int *, const int *, int *, int, hipStream_t);
hipError_t launch_qr_kmat_d2_o3(const StencilArgs &, const int *, const int *, int *, int, hipStream_t);
hipError_t launch_qr_kmat_d2_o4(const StencilArgs &, const int *, const int *, int *, int, hipStream_t);
hipError_t launch_qr_kmat_d3_o1(const StencilArgs &, const int *, const int *, int *, int, hipStream_t);
hipError_t launch_qr_kmat_d3_o2(const StencilArgs &, const int *, const int *, int *, int, hipStream_t);
hipError_t launch_qr_kmat_d3_o3(const StencilArgs &, const int *, const int *, int *, int, hipStream_t);
hipError_t launch_qr_kmat_d3_o4(const StencilArgs &, const int *, const int *, int *, int, hipStream_t);

using KmatFn = hipError_t (*)(const StencilArgs &, const int *, const int *, int *, int, hipStream_t);
static const KmatFn kKmat[2][4] = {
    {launch_qr_kmat_d2_o1, launch_qr_kmat_d2_o2, launch_qr_kmat_d2_o3, launch_qr_kmat_d2_o4},
    {launch_qr_kmat_d3_o1, launch_qr_kmat_d3_o2, launch_qr_kmat_d3_o3, launch_qr_kmat_d3_o4}};

hipError_t launch_qr_kmat(int dim, int order, const StencilArgs &a, const int *list, const int *count, int *cursor,
                          int n_blocks, hipStream_t s) {
  if (!qr_supported(dim, order, 1)) return hipErrorInvalidValue;
  return kKmat[dim - 2][order - 1](a, list, count, cursor, n_blocks, s);
}

hipError_t launch_qr_shared_d2_o1(int, int, const StencilArgs &, const StencilArgs &, const int *, const int *,
                                   const int *, int *, int, hipStream_t);
hipError_t launch_qr_shared_d2_o2(int, int, const StencilArgs &, const StencilArgs &, const int *, const int *,
                                   const int *, int *, int, hipStream_t);
hipError_t launch_qr_shared_d2_o3(int, int, const StencilArgs &, const StencilArgs &, const int *, const int *,
                                   const int *, int *, int, hipStream_t);
hipError_t launch_qr_shared_d2_o4(int, int, const StencilArgs &, const StencilArgs &, const int *, const int *,
                                   const int *, int *, int, hipStream_t);
hipError_t launch_qr_shared_d3_o1(int, int, const StencilArgs &, const StencilArgs &, const int *, const int *,
                                   const int *, int *, int, hipStream_t);
hipError_t launch_qr_shared_d3_o2(int, int, const StencilArgs &, const StencilArgs &, const int *, const int *,
                                   const int *, int *, int, hipStream_t);
hipError_t launch_qr_shared_d3_o3(int, int, const StencilArgs &, const StencilArgs &, const int *, const int *,
                                   const int *, int *, int, hipStream_t);
hipError_t launch_qr_shared_d3_o4(int, int, const StencilArgs &, const StencilArgs &, const int *, const int *,
                                   const int *, int *, int, hipStream_t);

using SharedFn = hipError_t (*)(int, int, const StencilArgs &, const StencilArgs &, const int *, const int *, const int *,
                                int *, int, hipStream_t);
static const SharedFn kShared[2][4] = {
    {launch_qr_shared_d2_o1, launch_qr_shared_d2_o2, launch_qr_shared_d2_o3, launch_qr_shared_d2_o4},
    {launch_qr_shared_d3_o1, launch_qr_shared_d3_o2, launch_qr_shared_d3_o3, launch_qr_shared_d3_o4}};

hipError_t launch_qr_shared_bin(int dim, int order, int bin, int rpl, int wpe, const StencilArgs &as,
                                const StencilArgs &av, const int *list, BinMeta *meta, int n_blocks, hipStream_t s) {
  if (!qr_supported(dim, order, 1)) return hipErrorInvalidValue;
  return kShared[dim - 2][order - 1](rpl, wpe, as, av, list, meta->count + bin, meta->offset + bin, meta->cursor + bin,
                                     n_blocks, s);
}

using QrFn = hipError_t (*)(int, int, const StencilArgs &, const int *, const int *, const int *, int *, int, hipStream_t);
// [dim - 2][order - 1][basis]: basis 0 scalar, 1 divergence-free, 2 staggered
static const QrFn kQr[2][4][3] = {
    {{launch_qr_d2_o1_b0, launch_qr_d2_o1_b1, launch_qr_d2_o1_b2}, {launch_qr_d2_o2_b0, launch_qr_d2_o2_b1, launch_qr_d2_o2_b2}, {launch_qr_d2_o3_b0, launch_qr_d2_o3_b1, launch_qr_d2_o3_b2}, {launch_qr_d2_o4_b0, launch_qr_d2_o4_b1, launch_qr_d2_o4_b2}},
    {{launch_qr_d3_o1_b0, launch_qr_d3_o1_b1, launch_qr_d3_o1_b2}, {launch_qr_d3_o2_b0, launch_qr_d3_o2_b1, launch_qr_d3_o2_b2}, {launch_qr_d3_o3_b0, launch_qr_d3_o3_b1, launch_qr_d3_o3_b2}, {launch_qr_d3_o4_b0, launch_qr_d3_o4_b1, launch_qr_d3_o4_b2}}};

bool qr_supported(int dim, int order, int basis) {
  return (dim == 2 || dim == 3) && order >= 1 && order <= 4 && basis >= 0 && basis <= 2;
}

static hipError_t dispatch_qr(int dim, int order, int basis, int rpl, int wpe, const StencilArgs &a, const int *list,
                              const int *count, const int *offset, int *cursor, int n_blocks, hipStream_t s) {
  if (!qr_supported(dim, order, basis)) return hipErrorInvalidValue;
  return kQr[dim - 2][order - 1][basis](rpl, wpe, a, list, count, offset, cursor, n_blocks, s);
}

hipError_t launch_qr_bin(int dim, int order, int basis, int bin, int rpl, int wpe, const StencilArgs &a,
                         const int *list, BinMeta *meta, int n_blocks, hipStream_t s) {
  return dispatch_qr(dim, order, basis, rpl, wpe, a, list, meta->count + bin, meta->offset + bin, meta->cursor + bin,
                     n_blocks, s);
}

hipError_t launch_qr_queue(int dim, int order, int basis, const StencilArgs &a, const int *list, const int *count,
                           int *cursor, int n_blocks, hipStream_t s) {
  return dispatch_qr(dim, order, basis, 4, 0, a, list, count, nullptr, cursor, n_blocks, s);
}

hipError_t launch_qr_fallback(int dim, int order, int basis, const StencilArgs &a, const int *list, BinMeta *meta,
                              int max_bin, int n_blocks, hipStream_t s) {
  return dispatch_qr(dim, order, basis, max_bin, 0, a, list, &meta->fb_count, nullptr, &meta->fb_cursor, n_blocks,
                     s);
}

}  // namespace gmls
