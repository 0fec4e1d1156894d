// gmls_internal.hpp -- context, workspace and the launch interfaces shared by
// the translation units of libgmls (host side only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <map>
#include <string>
#include <vector>

#include "../../include/libgmls.h"

namespace gmls {

// Workspace slots owned by a context (device memory, grown on demand).
enum Slot {
  WS_BBOX = 0,
  WS_GRID,
  WS_CELL_KEY,
  WS_CELL_COUNT,
  WS_CELL_START,
  WS_SORTED,
  WS_SORTED_TMP,
  WS_TGT_KEY,
  WS_TGT_COUNT,
  WS_TGT_START,
  WS_TGT_ORDER,
  WS_ROW_COUNT,
  WS_DEFER,
  WS_RADIUS_ROWS,
  WS_TGT_FLAG,
  WS_DEV_ERR,
  WS_SCAN_TMP,
  WS_FLAGS,
  WS_BIN_META,
  WS_BIN_LIST,
  WS_FALLBACK,
  WS_STATS,
  WS_STATUS_TMP,
  WS_BIN_TEMP,
  WS_PIPE_MOM,
  WS_PIPE_Y,
  WS_PIPE_REC,
  WS_STOKES_LEN,
  WS_STOKES_TMP,
  WS_STOKES_FLAG,
  WS_SPMV_LONG,
  WS_AUX_LIST,
  WS_FALLBACK2,
  WS_STATUS_TMP2,
  WS_PIPE_Y2,
  WS_COND,
  WS_REPORT,
  WS_SRC_POS,
  WS_TUNE_AUX,
  WS_NUM_SLOTS
};

// internal basis id of the staggered scheme: scalar monomials of degree
// 1..order without the constant, FP64 QR only (gmls_stencils_staggered)
constexpr int kBasisStaggered = 2;

// mixed-precision schemes (GMLS_OPT_MIXED_SCHEME)
enum MixedScheme { MIXED_AUTO = 0, MIXED_ROWS = 1, MIXED_GRAM = 2, MIXED_PIPE = 3, MIXED_WAVE = 4 };

struct Options {
  double cond_threshold = 1e6;
  int max_sweeps = 8;
  double refine_tol = 1e-11;
  int force_fallback = 0;
  int scheme = MIXED_AUTO;  // resolved to ROWS, GRAM, PIPE or WAVE before any launch
  int64_t pipe_chunk = 0;   // list slots per pipeline chunk (0: the whole call)
  int64_t radius_scratch_mb = 8192;  // scratch rows of the one-pass radius search (MiB)
  int capture_safe = 0;              // nonzero: no call waits for the device (see libgmls.h)
  int row_order = 0;                 // radius rows: 0 cell order, 1 ascending source index
  int pipe_force = -1;               // pipeline row shape: -1 the tuned table, else this candidate
  int wave_force = -1;               // wavefront-kernel variant: -1 the tuned table, else this candidate
  int qr_force = -1;                 // FP64 QR shape: -1 the tuned table, else this candidate
  int source_stride = 0;             // doubles per source record of the stencil calls (0: dim)
  int reuse_moments = 0;             // per call: the pipeline's moments and records are already in place
  // per call: pipeline row-shape candidate of [kernel: 0 moments, 1 weights][bin]
  signed char pipe_shape[2][8] = {};
  // per call: wavefront-kernel variant and FP64 QR shape of [bin]
  signed char wave_shape[8] = {};
  signed char qr_shape[8] = {};
};

// HIP events around every per-bin launch of the tunable kernels (the
// autotuner's measurement: [0 pipeline moments, 1 pipeline weights,
// 2 wavefront kernel, 3 FP64 QR][bin]); used[k][b] is set for each launch
// recorded
struct PipeTimer {
  hipEvent_t ev[4][8][2] = {};
  int used[4][8] = {};
};

// Device error bits accumulated for gmls_check (capture-safe mode).
enum DevErr { DEV_ERR_RADIUS_ROWS = 1, DEV_ERR_CAPACITY = 2, DEV_ERR_STENCIL_ROWS = 4 };

}  // namespace gmls

struct gmls_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<std::pair<void *, size_t>> slots;
  gmls::Options opt;
  hipEvent_t ev[8] = {};
  int cus = 256;  // compute units of the device
  // autotuned pipeline row shapes: key (dim * 8 + order) * 4 + basis ->
  // candidate of [kernel * 8 + bin], -1 where not tuned
  // autotune table: (dim, order, basis) -> candidate of [kernel * 8 + bin]
  // (kernels: 0 pipeline moments, 1 pipeline weights, 2 wavefront, 3 FP64 QR;
  // -1 where nothing was tuned)
  std::map<int, std::array<signed char, 32>> tune;
  gmls::PipeTimer *timer = nullptr;  // set by the autotuner around its runs
  double t_search_ms = 0.0;           // GPU time of the last synchronising gmls_neighbors call

  // Device buffer of at least `bytes` for `slot`; nullptr on failure (and,
  // in capture-safe mode, when the slot would have to grow).
  void *ws(int slot, size_t bytes);
  ~gmls_ctx_s();
};

namespace gmls {

// Source point after the cell sort: coordinates, original index.
struct SPoint {
  double x, y, z;
  int idx;
  int pad;
};

// Uniform cell grid over the sources (cells numbered x fastest).
struct GridParams {
  double lo[3];
  double c, inv_c;
  int nc[3];
  int ncell;
};

// Bin bookkeeping of the stencil scheduler (device memory).
struct BinMeta {
  int count[8];    // targets per bin
  int offset[8];   // start of the bin in the packed list
  int cursor[8];   // fill cursor (binning) / work counter (stencils)
  int fb_count;    // targets queued for the FP64 fallback
  int fb_cursor;   // fallback work counter
  int err;         // nonzero: a row longer than the compiled maximum
  int pad;
  int aux_count;   // divergence-free targets queued for the factorisation of
  int aux_cursor;  // their own sample matrix (scalar basis not unisolvent)
  int fb2_count;   // second set of a shared call (gmls_stencils_multi):
  int fb2_cursor;  // its FP64 fallback queue
};

// Per-call statistics accumulated on the device (mixed path).
struct Stats {
  unsigned long long n_fallback;
  unsigned long long n_not_converged;
  unsigned long long n_rank_def;
  unsigned long long sweep_hist[16];
  unsigned long long cond_max_bits;  // max of a non-negative double, as bits
};

// ---- search (search.hip) ----
gmls_status run_neighbors(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                          int64_t n_tgt, int dim, const gmls_search &spec, int64_t *row_ptr, int32_t *col,
                          int64_t col_capacity, double *eps, int64_t *nnz_host, double *records, int32_t *pcol);

// ---- stencils (stencil_*.hip) ----
struct StencilArgs {
  const double *coords;  // source j at coords[j * cstride .. + dim)
  int cstride;
  const double *targets;
  const double *eps;
  const int64_t *row_ptr;
  const int32_t *col;
  double *weights;
  uint8_t *status;  // never null inside kernels (a workspace stands in)
  unsigned mask;
  int F;            // functional rows of this basis/mask
  int p;            // kernel power
  int n_tgt;
  int ok_status;    // status written on success (-1: leave the status as it is)
  // Neumann-constrained stencils (scalar basis): per-target normals [n][dim]
  // and the weight of the boundary value h per functional row [n][F];
  // both null for plain stencils
  const double *normals = nullptr;
  double *hweights = nullptr;
  // staggered stencils on the mixed pipeline: the constant monomial is not a
  // column, and hweights receives the target weight -sum_j alpha_j
  int skip_const = 0;
  // divergence-free FP64 kernel: targets whose scalar basis is not unisolvent
  // go to aux_list[atomicAdd(aux_count, 1)] (null: they are rank deficient)
  int *aux_list = nullptr;
  int *aux_count = nullptr;
  // when non-null (a report was requested): the mixed kernels write the
  // condition number (estimate) of each target's equilibrated Gram here
  float *cond_out = nullptr;
};

// Per-bin stencil launches.  The FP64 QR kernel of bin `bin` runs with `rpl`
// rows per lane (a row longer than 64 * rpl is factored in chunks); wpe 2
// selects its variant compiled for two waves per SIMD.
hipError_t launch_qr_bin(int dim, int order, int basis, int bin, int rpl, int wpe, const StencilArgs &a,
                         const int *list, BinMeta *meta, int n_blocks, hipStream_t s);
hipError_t launch_qr_fallback(int dim, int order, int basis, const StencilArgs &a, const int *list,
                              BinMeta *meta, int max_bin, int n_blocks, hipStream_t s);
hipError_t launch_mixed_bin(int dim, int order, int basis, int bin, const StencilArgs &a, const int *list,
                            BinMeta *meta, int *fb_list, Stats *stats, const Options &opt, int count, int cus,
                            hipStream_t s);
// bytes of the pipeline's per-target record
constexpr size_t kPipeRecBytes = 64;
// hm: host copy of the bin table, or nullptr when the launches may not
// depend on it (every bound then comes from `meta` on the device)
// timer: nullptr, or events to record around each per-bin launch
hipError_t launch_mixed_pipe(int dim, int order, int basis, const StencilArgs &a, const int *list,
                             const BinMeta *hm, BinMeta *meta, int *fb, Stats *stats, const Options &opt,
                             double *mom, double *y, void *rec, int64_t chunk, int n_max, int cus,
                             PipeTimer *timer, hipStream_t s);
// one wavefront per target (bins launched as in launch_mixed_pipe)
hipError_t launch_mixed_wave(int dim, int order, int basis, const StencilArgs &a, const int *list,
                             const BinMeta *hm, BinMeta *meta, int *fb, Stats *stats, const Options &opt, int n_max,
                             int cus, PipeTimer *timer, hipStream_t s);
// FP64 QR of the targets list[0 .. *count) (work counter *cursor), any row count
hipError_t launch_qr_queue(int dim, int order, int basis, const StencilArgs &a, const int *list, const int *count,
                           int *cursor, int n_blocks, hipStream_t s);
// one wavefront per target for a scalar set (as) and a divergence-free set
// (av) on the same neighbour lists: moments and swept Gram formed once
hipError_t launch_mixed_wave_shared(int dim, int order, const StencilArgs &as, int *fbs, int *fbs_count,
                                    const StencilArgs &av, int *fbv, int *fbv_count, const int *list,
                                    const BinMeta *hm, BinMeta *meta, Stats *stats, const Options &opt, int n_max,
                                    int cus, PipeTimer *timer, hipStream_t s);
// FP64 QR of bin `bin` for a scalar set (as) and a divergence-free set (av)
// on the same neighbour lists: one Householder factor per target for both
hipError_t launch_qr_shared_bin(int dim, int order, int bin, int rpl, int wpe, const StencilArgs &as,
                                const StencilArgs &av, const int *list, BinMeta *meta, int n_blocks, hipStream_t s);
// the queued divergence-free targets of aux_list[0 .. *count)
hipError_t launch_qr_kmat(int dim, int order, const StencilArgs &a, const int *list, const int *count,
                          int *cursor, int n_blocks, hipStream_t s);
bool qr_supported(int dim, int order, int basis);
bool mixed_supported(int dim, int order, int basis);
// the scheme a request resolves to (MIXED_AUTO picks the fastest compiled
// one); -1 when the requested scheme is not compiled for this shape
int mixed_scheme(int dim, int order, int basis, int requested);
// FP64 moments of the pipeline per target (num_mono(dim, 2*order))
int pipe_num_moments(int dim, int order);

// device-side helpers (stencil_bins.hip): zero a buffer with a kernel (no
// memset node in captured graphs); OR (src & mask) != 0 ? bit : 0 into *dst
hipError_t fill_zero(void *p, size_t bytes, hipStream_t s);
hipError_t or_error_bit(int *dst, const int *src, int mask, int bit, hipStream_t s);

// Report counters (stencil_bins.hip): per-status target counts of a status
// array, and the smallest value and a log2 histogram (kCondBinsPerOctave
// bins per factor of 2 over [1, 2^64)) of per-target condition numbers
// (non-finite entries are skipped).
constexpr int kCondBinsPerOctave = 16;
constexpr int kCondBins = 64 * kCondBinsPerOctave;
struct ReportCounts {
  unsigned long long status[4];      // targets with status 0..3 (summed over the arrays counted)
  unsigned long long n_cond;         // finite condition numbers seen
  unsigned int cond_min_inv;         // ~(float bits) of the smallest one (non-negative floats order as
                                     // their bits, so the largest complement is the smallest value)
  unsigned int pad;
  unsigned int cond_hist[kCondBins];
};
hipError_t fill_f32(float *p, float v, int64_t n, hipStream_t s);
hipError_t launch_status_count(const uint8_t *status, int n, ReportCounts *rc, hipStream_t s);
hipError_t launch_cond_stats(const float *cond, int n, ReportCounts *rc, hipStream_t s);

// exclusive scan of n ints (search.hip): out[0..n], tmp of scan_i32_tmp_words(n)
int64_t scan_i32_tmp_words(int64_t n);
hipError_t scan_i32_exclusive(const int *in, int *out, int64_t n, int *tmp, hipStream_t s);
// the same for int64 (tmp of scan_i32_tmp_words(n) int64 entries)
hipError_t scan_i64_exclusive(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s);

// binning (stencil_bins.hip)
// temporary device bytes launch_binning needs for n_tgt targets
size_t binning_temp_bytes(int n_tgt);
hipError_t launch_binning(const int64_t *row_ptr, const double *targets, int n_tgt, int dim, int Q,
                          int rows_per_nbr, BinMeta *meta, int *list, void *temp, size_t temp_bytes, hipStream_t s);
hipError_t launch_rank_deficient(const StencilArgs &a, int C, const int *list, BinMeta *meta, hipStream_t s);
// every target of `bin` to the FP64 fallback queue fb_list / *fb_count with
// status FALLBACK (stats: counted there unless null)
hipError_t launch_defer_bin(uint8_t *status, const int *list, const BinMeta *meta, int bin, int *fb_list,
                            int *fb_count, Stats *stats, hipStream_t s);

// apply (apply.hip)
// global Stokes operator (assemble.hip)
struct StokesArgs {
  int64_t n = 0;
  int dim = 0;
  double nu = 1.0;
  const int64_t *row_ptr = nullptr;
  const int32_t *col = nullptr;
  const uint8_t *boundary = nullptr;
  const double *normals = nullptr;
  const double *vlap = nullptr, *grad = nullptr, *plap = nullptr, *plap_t = nullptr, *nlap = nullptr,
               *nlap_h = nullptr;
};
hipError_t launch_stokes_assembly(const StokesArgs &s, int64_t *rlen, int64_t *arp, int64_t *tmp, int32_t *acol,
                                  double *aval, int64_t capacity, int *flags, int cus, hipStream_t st);
hipError_t launch_spmv(int64_t rows, const int64_t *rp, const int32_t *col, const double *val, const double *x,
                       double *y, int *long_rows, int *n_long, int cus, hipStream_t s);
// allocation-free product: rows of at most kNoAllocSpmvRows, the long-row
// list in the file-scope device array of assemble.hip, whose address on a
// device spmv_scratch_setup (called with that device current, once per
// device) looks up and spmv_scratch returns (nullptr before the set-up)
constexpr int64_t kNoAllocSpmvRows = (int64_t)1 << 23;
hipError_t spmv_scratch_setup(int device);
int *spmv_scratch(int device);

hipError_t launch_apply(int64_t n_tgt, const int64_t *row_ptr, const int32_t *col, const double *weights, int F,
                        int C, const double *field, double *out, hipStream_t s);

// number of bins: 0 = rank deficient (N*C < Q), b = 1..4: 64(b-1) < N <=
// 64b, b = 5 (kLongBin): 256 < N <= kMaxRows, rows taken in chunks; a longer
// row (bin 7 of the binning) fails the call
constexpr int kNumBins = 6;
constexpr int kLongBin = 5;
constexpr int kMaxRows = 1 << 24;

// Row shapes of the pipeline's row-parallel kernels (moments, weights):
// G lanes per target, RPL rows per lane, G * RPL >= 64 b for bin b (the long
// bin loops over chunks of G * RPL rows).  All three are compiled for every
// bin; candidate 0 is the untuned default and the autotuner keeps the
// fastest per (dimension, order, basis, kernel, bin).
constexpr int kPipeCands = 3;
struct PipeShape {
  int g, rpl;
};
// FP64 QR shapes per bin: rows per lane (a row count above 64 * rpl is
// factored in chunks by the tall-skinny QR), persistent wavefronts per
// compute unit, and the occupancy the kernel is compiled for (0: the
// compiler's choice; 2: at most 256 registers, two waves per SIMD)
struct QrShape {
  int rpl, per_cu, wpe;
};
constexpr QrShape kQrShapes[kNumBins][kPipeCands] = {
    {{4, 8, 0}, {4, 8, 0}, {4, 8, 0}},  // bin 0: divergence-free targets whose scalar basis is rank deficient
    {{1, 16, 0}, {1, 8, 0}, {1, 16, 2}},
    {{2, 16, 0}, {1, 16, 0}, {2, 16, 2}},
    {{3, 16, 0}, {2, 16, 0}, {3, 16, 2}},
    {{4, 16, 0}, {3, 16, 0}, {4, 16, 2}},
    {{4, 16, 0}, {3, 16, 0}, {2, 16, 0}}};
// Compiled variants of the wavefront kernel (mixed scheme 4), selected per
// row-count bin: the occupancy it is compiled for (waves per SIMD) and the
// moments per LDS reduction round.
struct WaveCand {
  int wpe, rs;
};
constexpr int kWaveCands = 3;
constexpr WaveCand kWaveCand[kWaveCands] = {{2, 16}, {1, 16}, {2, 8}};
// key basis of the tuned shapes of gmls_stencils_multi's shared kernels
constexpr int kTuneShared = 3;
constexpr PipeShape kPipeShapes[kNumBins][kPipeCands] = {
    {{0, 0}, {0, 0}, {0, 0}},  // bin 0: rank deficient, never launched
    {{8, 8}, {16, 4}, {4, 16}},
    {{16, 8}, {32, 4}, {8, 16}},
    {{32, 6}, {16, 12}, {64, 3}},
    {{32, 8}, {64, 4}, {16, 16}},
    {{64, 4}, {64, 2}, {32, 8}}};

}  // namespace gmls

gmls_status gmls_set_error(gmls_ctx ctx, gmls_status st, const std::string &msg);
