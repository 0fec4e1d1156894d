#pragma once
// qr_kernel.hpp -- the FP64 QR stencil kernels: a persistent wavefront per
// target for the scalar (and staggered) basis and for the divergence-free
// basis, their LDS size, and the kernel that serves a scalar and a
// divergence-free set on the same rows from one factor.
#include "stencil_fp64.hpp"
#include "stencil_fp64_div.hpp"

namespace gmls {

template <int DIM, int ORDER, int BASIS>
constexpr int qr_lds_doubles() {
  constexpr int Q = num_mono(DIM, ORDER);
  // the solves' buffers, or the factor's column sums if larger (the factor
  // runs before the solves, so they share the array)
  constexpr int SOLVE = BASIS != 1 ? 2 * Q * Q + 8 * Q : qr_divfree_lds_doubles<DIM, ORDER>();
  return SOLVE > kSumBufDoubles ? SOLVE : kSumBufDoubles;
}

// Persistent kernel: waves take targets from list[0 .. *count) in turn.
template <int DIM, int ORDER, int BASIS, int RPL>
__device__ __forceinline__ void qr_loop(const StencilArgs &a, const int *list, const int *count, const int *offset,
                                        int *cursor) {
  __shared__ __align__(16) double lds[qr_lds_doubles<DIM, ORDER, BASIS>()];
  const RowKinds rk = row_kinds(DIM, BASIS == 1 ? 1 : 0, a.mask);
  const int n = readfirstlane_i(*count);
  const int off = readfirstlane_i(offset ? *offset : 0);
  for (;;) {
    int i = 0;
    if (lane_id() == 0) i = atomicAdd(cursor, 1);
    i = __builtin_amdgcn_readfirstlane(i);
    if (i >= n) break;
    const int t = readfirstlane_i(list[off + i]);
    if constexpr (BASIS == 0)
      qr_scalar_target<DIM, ORDER, RPL>(a, rk, t, lds);
    else if constexpr (BASIS == 2)
      qr_scalar_target<DIM, ORDER, RPL, 1>(a, rk, t, lds);
    else
      qr_divfree_target<DIM, ORDER, RPL>(a, rk, t, lds);
  }
}

template <int DIM, int ORDER, int BASIS, int RPL>
__global__ __launch_bounds__(64) void k_qr(StencilArgs a, const int *list, const int *count, const int *offset,
                                           int *cursor) {
  qr_loop<DIM, ORDER, BASIS, RPL>(a, list, count, offset, cursor);
}

// The same kernel compiled for two waves per SIMD (at most 256 registers):
// an autotuner candidate for the instantiations that the compiler gives
// slightly more than 256 registers, and so one wave per SIMD.
template <int DIM, int ORDER, int BASIS, int RPL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_qr_w2(
    StencilArgs a, const int *list, const int *count, const int *offset, int *cursor) {
  qr_loop<DIM, ORDER, BASIS, RPL>(a, list, count, offset, cursor);
}

// A scalar set (as) and a divergence-free set (av) of the same order on the
// same neighbour rows: both fits are taken through the Householder factor R
// of the scalar sample matrix sqrt(W) P, which is computed once per target
// (the divergence-free set's Gram I (x) G has G = R^T R as its blocks).  The
// per-set steps are those of k_qr, so the weights equal those of two k_qr
// calls bit for bit.
template <int DIM, int ORDER, int RPL>
__device__ __forceinline__ void qr_shared_loop(const StencilArgs &as, const StencilArgs &av, const int *list,
                                               const int *count, const int *offset, int *cursor) {
  constexpr int Q = num_mono(DIM, ORDER);
  constexpr int LS = qr_lds_doubles<DIM, ORDER, 0>(), LV = qr_lds_doubles<DIM, ORDER, 1>();
  __shared__ __align__(16) double lds[LS > LV ? LS : LV];
  const RowKinds rks = row_kinds(DIM, 0, as.mask);
  const RowKinds rkv = row_kinds(DIM, 1, av.mask);
  const int n = readfirstlane_i(*count);
  const int off = readfirstlane_i(offset ? *offset : 0);
  for (;;) {
    int i = 0;
    if (lane_id() == 0) i = atomicAdd(cursor, 1);
    i = __builtin_amdgcn_readfirstlane(i);
    if (i >= n) break;
    const int t = readfirstlane_i(list[off + i]);
    Rows<DIM, RPL> r;
    double M[RPL][Q];
    double rdiag;
    qr_factor<DIM, ORDER, RPL>(as, t, r, M, rdiag, lane_id(), lds);  // lds is free until the solves
    // the scalar solve leaves R row-major in lds[0 .. Q*Q) (the divergence-free
    // solve's layout) unless R fails the rank test, after which the
    // divergence-free solve does not read it; it ends with a barrier
    qr_scalar_solve<DIM, ORDER, RPL>(as, rks, t, r, M[0], rdiag, lds);
    qr_divfree_solve<DIM, ORDER, RPL, true>(av, rkv, t, r, M[0], rdiag, lds);
  }
}

template <int DIM, int ORDER, int RPL>
__global__ __launch_bounds__(64) void k_qr_shared(StencilArgs as, StencilArgs av, const int *list, const int *count,
                                                  const int *offset, int *cursor) {
  qr_shared_loop<DIM, ORDER, RPL>(as, av, list, count, offset, cursor);
}

template <int DIM, int ORDER, int RPL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_qr_shared_w2(
    StencilArgs as, StencilArgs av, const int *list, const int *count, const int *offset, int *cursor) {
  qr_shared_loop<DIM, ORDER, RPL>(as, av, list, count, offset, cursor);
}

}  // namespace gmls
