// wave_unit.hip -- one instantiation of the mixed-path kernels that give each
// target a whole wavefront.  Compiled once per (GMLS_DIM, GMLS_ORDER,
// GMLS_BASIS) by the build, each object defining
// launch_wave_d<DIM>_o<ORDER>_b<BASIS> (and, with the divergence-free basis,
// launch_wave_shared_d<DIM>_o<ORDER>: a scalar and a divergence-free set).
#include "stencil_wave.hpp"

#if !defined(GMLS_DIM) || !defined(GMLS_ORDER) || !defined(GMLS_BASIS)
#error "compile with -DGMLS_DIM=.. -DGMLS_ORDER=.. -DGMLS_BASIS=.."
#endif
// GMLS_PART 0: the per-basis launcher only; 1: the shared launcher only;
// undefined: both (objects build in parallel)
#ifndef GMLS_PART
#define GMLS_PART -1
#endif

#define GMLS_CAT2(a, b, c, d, e, f) a##b##c##d##e##f
#define GMLS_CAT(a, b, c, d, e, f) GMLS_CAT2(a, b, c, d, e, f)
#define GMLS_WAVE_FN GMLS_CAT(launch_wave_d, GMLS_DIM, _o, GMLS_ORDER, _b, GMLS_BASIS)
#define GMLS_SHARED_FN GMLS_CAT(launch_wave_shared_d, GMLS_DIM, _o, GMLS_ORDER, , )

namespace gmls {

#if GMLS_PART != 1
hipError_t GMLS_WAVE_FN(const StencilArgs &a, const int *list, const BinMeta *hm, BinMeta *meta, int *fb,
                        Stats *stats, const Options &opt, int n_max, int cus, PipeTimer *timer, hipStream_t s) {
  const WaveSet one{a, fb, &meta->fb_count};
  return launch_wave<GMLS_DIM, GMLS_ORDER, GMLS_BASIS>(one, one, list, hm, meta, stats, opt, n_max, cus, timer, s);
}
#endif

#if GMLS_BASIS == 1 && GMLS_PART != 0
// a scalar and a divergence-free set on the same neighbour lists, one pass
hipError_t GMLS_SHARED_FN(const StencilArgs &as, int *fbs, int *fbs_count, const StencilArgs &av, int *fbv,
                          int *fbv_count, const int *list, const BinMeta *hm, BinMeta *meta, Stats *stats,
                          const Options &opt, int n_max, int cus, PipeTimer *timer, hipStream_t s) {
  const WaveSet ss{as, fbs, fbs_count}, sv{av, fbv, fbv_count};
  return launch_wave<GMLS_DIM, GMLS_ORDER, 3>(ss, sv, list, hm, meta, stats, opt, n_max, cus, timer, s);
}
#endif

}  // namespace gmls
