// wave_unit.hip -- one instantiation of the mixed-path kernels that give each
// target a whole wavefront.  Compiled once per (GMLS_DIM, GMLS_ORDER,
// GMLS_BASIS) by the build, each object defining
// launch_wave_d<DIM>_o<ORDER>_b<BASIS>.
#include "stencil_wave.hpp"

#if !defined(GMLS_DIM) || !defined(GMLS_ORDER) || !defined(GMLS_BASIS)
#error "compile with -DGMLS_DIM=.. -DGMLS_ORDER=.. -DGMLS_BASIS=.."
#endif

#define GMLS_CAT2(a, b, c, d, e, f) a##b##c##d##e##f
#define GMLS_CAT(a, b, c, d, e, f) GMLS_CAT2(a, b, c, d, e, f)
#define GMLS_WAVE_FN GMLS_CAT(launch_wave_d, GMLS_DIM, _o, GMLS_ORDER, _b, GMLS_BASIS)

namespace gmls {

hipError_t GMLS_WAVE_FN(const StencilArgs &a, const int *list, const BinMeta *hm, BinMeta *meta, int *fb,
                        Stats *stats, const Options &opt, int n_max, int cus, hipStream_t s) {
  return launch_wave<GMLS_DIM, GMLS_ORDER, GMLS_BASIS>(a, list, hm, meta, fb, stats, opt, n_max, cus, s);
}

}  // namespace gmls
