// stencil_mixed.hip -- dispatch of the mixed-precision stencil kernels.  The
// kernels are instantiated per (dim, order, basis) from mixed_unit.hip (fused
// kernels and pipeline) and wave_unit.hip (one wavefront per target).
#include "common.hpp"
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

hipError_t launch_pipe_d2_o1_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d2_o1_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d2_o2_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d2_o2_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d2_o3_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d2_o3_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d2_o4_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d2_o4_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d3_o1_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d3_o1_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d3_o2_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d3_o2_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d3_o3_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d3_o3_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d3_o4_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);
hipError_t launch_pipe_d3_o4_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *, hipStream_t);

using PipeFn = hipError_t (*)(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                              const Options &, double *, double *, void *, int64_t, int, int, PipeTimer *,
                              hipStream_t);
static const PipeFn kPipe[2][4][2] = {
    {{launch_pipe_d2_o1_b0, launch_pipe_d2_o1_b1}, {launch_pipe_d2_o2_b0, launch_pipe_d2_o2_b1}, {launch_pipe_d2_o3_b0, launch_pipe_d2_o3_b1}, {launch_pipe_d2_o4_b0, launch_pipe_d2_o4_b1}},
    {{launch_pipe_d3_o1_b0, launch_pipe_d3_o1_b1}, {launch_pipe_d3_o2_b0, launch_pipe_d3_o2_b1}, {launch_pipe_d3_o3_b0, launch_pipe_d3_o3_b1}, {launch_pipe_d3_o4_b0, launch_pipe_d3_o4_b1}}};

hipError_t launch_wave_d2_o1_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d2_o1_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d2_o2_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d2_o2_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d2_o3_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d2_o3_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d2_o4_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d2_o4_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d3_o1_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d3_o1_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d3_o2_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d3_o2_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d3_o3_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d3_o3_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d3_o4_b0(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);
hipError_t launch_wave_d3_o4_b1(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                                const Options &, int, int, PipeTimer *, hipStream_t);

using WaveFn = hipError_t (*)(const StencilArgs &, const int *, const BinMeta *, BinMeta *, int *, Stats *,
                              const Options &, int, int, PipeTimer *, hipStream_t);
static const WaveFn kWave[2][4][2] = {
    {{launch_wave_d2_o1_b0, launch_wave_d2_o1_b1}, {launch_wave_d2_o2_b0, launch_wave_d2_o2_b1}, {launch_wave_d2_o3_b0, launch_wave_d2_o3_b1}, {launch_wave_d2_o4_b0, launch_wave_d2_o4_b1}},
    {{launch_wave_d3_o1_b0, launch_wave_d3_o1_b1}, {launch_wave_d3_o2_b0, launch_wave_d3_o2_b1}, {launch_wave_d3_o3_b0, launch_wave_d3_o3_b1}, {launch_wave_d3_o4_b0, launch_wave_d3_o4_b1}}};

hipError_t launch_wave_shared_d2_o1(const StencilArgs &, int *, int *, const StencilArgs &, int *, int *,
                                 const int *, const BinMeta *, BinMeta *, Stats *, const Options &, int, int,
                                 PipeTimer *, hipStream_t);
hipError_t launch_wave_shared_d2_o2(const StencilArgs &, int *, int *, const StencilArgs &, int *, int *,
                                 const int *, const BinMeta *, BinMeta *, Stats *, const Options &, int, int,
                                 PipeTimer *, hipStream_t);
hipError_t launch_wave_shared_d2_o3(const StencilArgs &, int *, int *, const StencilArgs &, int *, int *,
                                 const int *, const BinMeta *, BinMeta *, Stats *, const Options &, int, int,
                                 PipeTimer *, hipStream_t);
hipError_t launch_wave_shared_d2_o4(const StencilArgs &, int *, int *, const StencilArgs &, int *, int *,
                                 const int *, const BinMeta *, BinMeta *, Stats *, const Options &, int, int,
                                 PipeTimer *, hipStream_t);
hipError_t launch_wave_shared_d3_o1(const StencilArgs &, int *, int *, const StencilArgs &, int *, int *,
                                 const int *, const BinMeta *, BinMeta *, Stats *, const Options &, int, int,
                                 PipeTimer *, hipStream_t);
hipError_t launch_wave_shared_d3_o2(const StencilArgs &, int *, int *, const StencilArgs &, int *, int *,
                                 const int *, const BinMeta *, BinMeta *, Stats *, const Options &, int, int,
                                 PipeTimer *, hipStream_t);
hipError_t launch_wave_shared_d3_o3(const StencilArgs &, int *, int *, const StencilArgs &, int *, int *,
                                 const int *, const BinMeta *, BinMeta *, Stats *, const Options &, int, int,
                                 PipeTimer *, hipStream_t);
hipError_t launch_wave_shared_d3_o4(const StencilArgs &, int *, int *, const StencilArgs &, int *, int *,
                                 const int *, const BinMeta *, BinMeta *, Stats *, const Options &, int, int,
                                 PipeTimer *, hipStream_t);
using SharedFn = hipError_t (*)(const StencilArgs &, int *, int *, const StencilArgs &, int *, int *, const int *,
                                const BinMeta *, BinMeta *, Stats *, const Options &, int, int, PipeTimer *, hipStream_t);
static const SharedFn kShared[2][4] = {
    {launch_wave_shared_d2_o1, launch_wave_shared_d2_o2, launch_wave_shared_d2_o3, launch_wave_shared_d2_o4},
    {launch_wave_shared_d3_o1, launch_wave_shared_d3_o2, launch_wave_shared_d3_o3, launch_wave_shared_d3_o4}};

using MixedFn = hipError_t (*)(int, const StencilArgs &, const int *, BinMeta *, int *, Stats *, const Options &, int,
                               int, hipStream_t);
static const MixedFn kMixed[2][4][2] = {
    {{launch_mixed_d2_o1_b0, launch_mixed_d2_o1_b1}, {launch_mixed_d2_o2_b0, launch_mixed_d2_o2_b1}, {launch_mixed_d2_o3_b0, launch_mixed_d2_o3_b1}, {launch_mixed_d2_o4_b0, launch_mixed_d2_o4_b1}},
    {{launch_mixed_d3_o1_b0, launch_mixed_d3_o1_b1}, {launch_mixed_d3_o2_b0, launch_mixed_d3_o2_b1}, {launch_mixed_d3_o3_b0, launch_mixed_d3_o3_b1}, {launch_mixed_d3_o4_b0, launch_mixed_d3_o4_b1}}};

bool mixed_supported(int dim, int order, int basis) {
  return (dim == 2 || dim == 3) && order >= 1 && order <= 4 && (basis == 0 || basis == 1);
}

int mixed_scheme(int dim, int order, int basis, int requested) {
  if (!mixed_supported(dim, order, basis)) return -1;
  const bool pipe = (basis == 0 && num_mono(dim, order) <= 20) || (basis == 1 && num_mono(dim, order) <= 10);
  const bool gram = num_mono(dim, 2 * order) <= 96;
  const bool wave = num_mono(dim, order) <= 35;
  switch (requested) {
    case MIXED_AUTO: return pipe ? MIXED_PIPE : wave ? MIXED_WAVE : gram ? MIXED_GRAM : MIXED_ROWS;
    case MIXED_ROWS: return MIXED_ROWS;
    case MIXED_GRAM: return gram ? MIXED_GRAM : -1;
    case MIXED_PIPE: return pipe ? MIXED_PIPE : -1;
    case MIXED_WAVE: return wave ? MIXED_WAVE : -1;
    default: return -1;
  }
}

int pipe_num_moments(int dim, int order) { return num_mono(dim, 2 * order); }

hipError_t launch_mixed_pipe(int dim, int order, int basis, const StencilArgs &a, const int *list,
                             const BinMeta *hm, BinMeta *meta, int *fb, Stats *stats, const Options &opt,
                             double *mom, double *y, void *rec, int64_t chunk, int n_max, int cus,
                             PipeTimer *timer, hipStream_t s) {
  if (mixed_scheme(dim, order, basis, MIXED_PIPE) != MIXED_PIPE) return hipErrorInvalidValue;
  return kPipe[dim - 2][order - 1][basis](a, list, hm, meta, fb, stats, opt, mom, y, rec, chunk, n_max, cus, timer,
                                          s);
}

hipError_t launch_mixed_wave(int dim, int order, int basis, const StencilArgs &a, const int *list,
                             const BinMeta *hm, BinMeta *meta, int *fb, Stats *stats, const Options &opt, int n_max,
                             int cus, PipeTimer *timer, hipStream_t s) {
  if (mixed_scheme(dim, order, basis, MIXED_WAVE) != MIXED_WAVE) return hipErrorInvalidValue;
  return kWave[dim - 2][order - 1][basis](a, list, hm, meta, fb, stats, opt, n_max, cus, timer, s);
}

hipError_t launch_mixed_wave_shared(int dim, int order, const StencilArgs &as, int *fbs, int *fbs_count,
                                    const StencilArgs &av, int *fbv, int *fbv_count, const int *list,
                                    const BinMeta *hm, BinMeta *meta, Stats *stats, const Options &opt, int n_max,
                                    int cus, PipeTimer *timer, hipStream_t s) {
  if (mixed_scheme(dim, order, 0, MIXED_WAVE) != MIXED_WAVE || mixed_scheme(dim, order, 1, MIXED_WAVE) != MIXED_WAVE)
    return hipErrorInvalidValue;
  return kShared[dim - 2][order - 1](as, fbs, fbs_count, av, fbv, fbv_count, list, hm, meta, stats, opt, n_max, cus,
                                     timer, s);
}

hipError_t launch_mixed_bin(int dim, int order, int basis, int bin, const StencilArgs &a, const int *list,
                            BinMeta *meta, int *fb, Stats *stats, const Options &opt, int count, int cus,
                            hipStream_t s) {
  if (!mixed_supported(dim, order, basis)) return hipErrorInvalidValue;
  return kMixed[dim - 2][order - 1][basis](bin, a, list, meta, fb, stats, opt, count, cus, s);
}

}  // namespace gmls
