// stencil_mixed.hip -- dispatch of the mixed-precision stencil kernels.  The
// kernels are instantiated per (dim, order, basis) from mixed_unit.hip.
#include "gmls_internal.hpp"

namespace gmls {

hipError_t launch_mixed_d2_o1_b0(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d2_o1_b1(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d2_o2_b0(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d2_o2_b1(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d2_o3_b0(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d2_o3_b1(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d2_o4_b0(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d2_o4_b1(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d3_o1_b0(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d3_o1_b1(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d3_o2_b0(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d3_o2_b1(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d3_o3_b0(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d3_o3_b1(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d3_o4_b0(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);
hipError_t launch_mixed_d3_o4_b1(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                                  const Options &, int, int, hipStream_t);

using MixedFn = hipError_t (*)(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *, const Options &, int,
                               int, hipStream_t);
static const MixedFn kMixed[2][4][2] = {
    {{launch_mixed_d2_o1_b0, launch_mixed_d2_o1_b1}, {launch_mixed_d2_o2_b0, launch_mixed_d2_o2_b1}, {launch_mixed_d2_o3_b0, launch_mixed_d2_o3_b1}, {launch_mixed_d2_o4_b0, launch_mixed_d2_o4_b1}},
    {{launch_mixed_d3_o1_b0, launch_mixed_d3_o1_b1}, {launch_mixed_d3_o2_b0, launch_mixed_d3_o2_b1}, {launch_mixed_d3_o3_b0, launch_mixed_d3_o3_b1}, {launch_mixed_d3_o4_b0, launch_mixed_d3_o4_b1}}};

bool mixed_supported(int dim, int order, int basis) {
  return (dim == 2 || dim == 3) && order >= 1 && order <= 4 && (basis == 0 || basis == 1);
}

hipError_t launch_mixed_bin(int dim, int order, int basis, int bin, const StencilArgs &a, const int *list,
                            BinMeta *meta, int *fb, Stats *stats, const Options &opt, int count, int cus,
                            hipStream_t s) {
  if (!mixed_supported(dim, order, basis)) return hipErrorInvalidValue;
  return kMixed[dim - 2][order - 1][basis](bin, a, list, meta, fb, stats, opt, count, cus, s);
}

}  // namespace gmls
