// stencil_mixed.hip -- mixed-precision stencils (placeholder until the mixed
// kernels are built; every launch reports "unsupported").
#include "gmls_internal.hpp"

namespace gmls {

bool mixed_supported(int, int, int) { return false; }

hipError_t launch_mixed_bin(int, int, int, int, const StencilArgs &, const int *, BinMeta *, int *, Stats *,
                            const Options &, int, hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace gmls
