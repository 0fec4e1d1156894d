// qr_unit.hip -- one instantiation of the FP64 QR stencil kernels.
// Compiled once per (GMLS_DIM, GMLS_ORDER, GMLS_BASIS) by the build, each
// object defining launch_qr_d<DIM>_o<ORDER>_b<BASIS>.
#include "qr_kernel.hpp"
#include "stencil_fp64_kmat.hpp"

#if !defined(GMLS_DIM) || !defined(GMLS_ORDER) || !defined(GMLS_BASIS)
#error "compile with -DGMLS_DIM=.. -DGMLS_ORDER=.. -DGMLS_BASIS=.."
#endif
// GMLS_PART 0: the per-basis kernel only; 1: the divergence-free unit's
// queued and shared kernels only; undefined: both (objects build in parallel)
#ifndef GMLS_PART
#define GMLS_PART -1
#endif

#define GMLS_CAT2(a, b, c, d, e, f) a##b##c##d##e##f
#define GMLS_CAT(a, b, c, d, e, f) GMLS_CAT2(a, b, c, d, e, f)
#define GMLS_FN GMLS_CAT(launch_qr_d, GMLS_DIM, _o, GMLS_ORDER, _b, GMLS_BASIS)
#define GMLS_KMAT_FN GMLS_CAT(launch_qr_kmat_d, GMLS_DIM, _o, GMLS_ORDER, , )
#define GMLS_SHARED_FN GMLS_CAT(launch_qr_shared_d, GMLS_DIM, _o, GMLS_ORDER, , )

namespace gmls {

#if GMLS_PART != 1
// one wavefront per target, `rpl` rows per lane (longer rows in chunks);
// wpe 2: the variant compiled for two waves per SIMD
hipError_t GMLS_FN(int rpl, int wpe, const StencilArgs &a, const int *list, const int *count, const int *offset,
                   int *cursor, int n_blocks, hipStream_t s) {
  constexpr int D = GMLS_DIM, O = GMLS_ORDER, B = GMLS_BASIS;
  switch ((rpl < 1 || rpl > 4 ? 4 : rpl) + (wpe == 2 ? 4 : 0)) {
    case 1: k_qr<D, O, B, 1><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
    case 2: k_qr<D, O, B, 2><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
    case 3: k_qr<D, O, B, 3><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
    case 5: k_qr_w2<D, O, B, 1><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
    case 6: k_qr_w2<D, O, B, 2><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
    case 7: k_qr_w2<D, O, B, 3><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
    case 8: k_qr_w2<D, O, B, 4><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
    default: k_qr<D, O, B, 4><<<n_blocks, 64, 0, s>>>(a, list, count, offset, cursor); break;
  }
  return hipGetLastError();
}
#endif

#if GMLS_BASIS == 1 && GMLS_PART != 0
// queued divergence-free targets (any row count up to 256: four rows per lane)
hipError_t GMLS_KMAT_FN(const StencilArgs &a, const int *list, const int *count, int *cursor, int n_blocks,
                        hipStream_t s) {
  k_qr_kmat<GMLS_DIM, GMLS_ORDER, 4><<<n_blocks, 64, 0, s>>>(a, list, count, cursor);
  return hipGetLastError();
}

// a scalar and a divergence-free set from one factor per target
hipError_t GMLS_SHARED_FN(int rpl, int wpe, const StencilArgs &as, const StencilArgs &av, const int *list,
                          const int *count, const int *offset, int *cursor, int n_blocks, hipStream_t s) {
  constexpr int D = GMLS_DIM, O = GMLS_ORDER;
  switch ((rpl < 1 || rpl > 4 ? 4 : rpl) + (wpe == 2 ? 4 : 0)) {
    case 1: k_qr_shared<D, O, 1><<<n_blocks, 64, 0, s>>>(as, av, list, count, offset, cursor); break;
    case 2: k_qr_shared<D, O, 2><<<n_blocks, 64, 0, s>>>(as, av, list, count, offset, cursor); break;
    case 3: k_qr_shared<D, O, 3><<<n_blocks, 64, 0, s>>>(as, av, list, count, offset, cursor); break;
    case 5: k_qr_shared_w2<D, O, 1><<<n_blocks, 64, 0, s>>>(as, av, list, count, offset, cursor); break;
    case 6: k_qr_shared_w2<D, O, 2><<<n_blocks, 64, 0, s>>>(as, av, list, count, offset, cursor); break;
    case 7: k_qr_shared_w2<D, O, 3><<<n_blocks, 64, 0, s>>>(as, av, list, count, offset, cursor); break;
    case 8: k_qr_shared_w2<D, O, 4><<<n_blocks, 64, 0, s>>>(as, av, list, count, offset, cursor); break;
    default: k_qr_shared<D, O, 4><<<n_blocks, 64, 0, s>>>(as, av, list, count, offset, cursor); break;
  }
  return hipGetLastError();
}
#endif

}  // namespace gmls
