#pragma once
// qr_kernel.hpp -- the FP64 QR stencil kernel: a persistent wavefront per
// target for the scalar (and staggered) basis and for the divergence-free
// basis, and its LDS size.
#include "stencil_fp64.hpp"
#include "stencil_fp64_div.hpp"

namespace gmls {

template <int DIM, int ORDER, int BASIS>
constexpr int qr_lds_doubles() {
  constexpr int Q = num_mono(DIM, ORDER);
  if (BASIS != 1) return 2 * Q * Q + 8 * Q;
  return qr_divfree_lds_doubles<DIM, ORDER>();
}

// Persistent kernel: waves take targets from list[0 .. *count) in turn.
template <int DIM, int ORDER, int BASIS, int RPL>
__global__ __launch_bounds__(64) void k_qr(StencilArgs a, const int *list, const int *count, const int *offset,
                                           int *cursor) {
  __shared__ double lds[qr_lds_doubles<DIM, ORDER, BASIS>()];
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

}  // namespace gmls
