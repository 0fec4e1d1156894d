// mixed_unit.hip -- one instantiation of the mixed-precision stencil kernels.
// Compiled once per (GMLS_DIM, GMLS_ORDER, GMLS_BASIS) by the build, each
// object defining launch_mixed_d<DIM>_o<ORDER>_b<BASIS> (the per-bin fused
// kernels) and launch_pipe_d<DIM>_o<ORDER>_b<BASIS> (the three-kernel pipeline,
// scalar bases with at most 20 functions).
#include "stencil_mixed64.hpp"
#include "stencil_pipe.hpp"

#if !defined(GMLS_DIM) || !defined(GMLS_ORDER) || !defined(GMLS_BASIS)
#error "compile with -DGMLS_DIM=.. -DGMLS_ORDER=.. -DGMLS_BASIS=.."
#endif

#define GMLS_CAT2(a, b, c, d, e, f) a##b##c##d##e##f
#define GMLS_CAT(a, b, c, d, e, f) GMLS_CAT2(a, b, c, d, e, f)
#define GMLS_FN GMLS_CAT(launch_mixed_d, GMLS_DIM, _o, GMLS_ORDER, _b, GMLS_BASIS)
#define GMLS_PIPE_FN GMLS_CAT(launch_pipe_d, GMLS_DIM, _o, GMLS_ORDER, _b, GMLS_BASIS)

namespace gmls {

template <int DIM, int ORDER, int BASIS, int G>
static hipError_t launch_one(const StencilArgs &a, const int *list, BinMeta *meta, int bin, int *fb, Stats *stats,
                             const Options &opt, int count, int cus, hipStream_t s) {
  constexpr int TPW = 64 / G;
  int nb = (count + TPW - 1) / TPW;
  if (nb > cus * 16) nb = cus * 16;
  if (nb < 1) nb = 1;
  if constexpr (has_gram64<DIM, ORDER>()) {
    if (opt.scheme == MIXED_GRAM) {
      k_mixed64<DIM, ORDER, BASIS, G><<<nb, 64, 0, s>>>(a, list, meta->count + bin, meta->offset + bin,
                                                         meta->cursor + bin, fb, meta, stats, opt);
      return hipGetLastError();
    }
  }
  k_mixed<DIM, ORDER, BASIS, G><<<nb, 64, 0, s>>>(a, list, meta->count + bin, meta->offset + bin,
                                                   meta->cursor + bin, fb, meta, stats, opt);
  return hipGetLastError();
}

// Rows per target: bin 1 <= 64, bin 2 <= 128, bins 3-4 <= 256, eight rows per
// lane; systems larger than 48 unknowns take a whole wavefront per target.
hipError_t GMLS_FN(int bin, const StencilArgs &a, const int *list, BinMeta *meta, int *fb, Stats *stats,
                   const Options &opt, int count, int cus, hipStream_t s) {
  constexpr int D = GMLS_DIM, O = GMLS_ORDER, B = GMLS_BASIS;
  if constexpr (MixedCfg<D, O, B, 64>::QA > 48) {
    return launch_one<D, O, B, 64>(a, list, meta, bin, fb, stats, opt, count, cus, s);
  } else {
    switch (bin) {
      case 1: return launch_one<D, O, B, 8>(a, list, meta, bin, fb, stats, opt, count, cus, s);
      case 2: return launch_one<D, O, B, 16>(a, list, meta, bin, fb, stats, opt, count, cus, s);
      default: return launch_one<D, O, B, 32>(a, list, meta, bin, fb, stats, opt, count, cus, s);
    }
  }
}

hipError_t GMLS_PIPE_FN(const StencilArgs &a, const int *list, const BinMeta *hm, BinMeta *meta, int *fb,
                        Stats *stats, const Options &opt, double *mom, double *y, void *rec, int64_t chunk,
                        int n_max, int cus, PipeTimer *timer, hipStream_t s) {
  constexpr int D = GMLS_DIM, O = GMLS_ORDER, B = GMLS_BASIS;
  PipeRec *r = (PipeRec *)rec;
  if constexpr (B == 0 && has_pipe<D, O>()) {
    if (a.skip_const)  // staggered stencils
      return launch_pipe<D, O, 1>(a, list, hm, meta, fb, stats, opt, mom, y, r, chunk, n_max, cus, timer, s);
    return launch_pipe<D, O>(a, list, hm, meta, fb, stats, opt, mom, y, r, chunk, n_max, cus, timer, s);
  } else if constexpr (B == 1 && has_pipe_div<D, O>()) {
    return launch_pipe<D, O, 0, 1>(a, list, hm, meta, fb, stats, opt, mom, y, r, chunk, n_max, cus, timer, s);
  } else {
    return hipErrorInvalidValue;
  }
}

}  // namespace gmls
