// api.cpp -- the C ABI of libgmls (include/libgmls.h): argument validation,
// workspace management and the launch sequence of each call.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>

#include "gmls_internal.hpp"

using namespace gmls;

void *gmls_ctx_s::ws(int slot, size_t bytes) {
  if (slot < 0 || slot >= WS_NUM_SLOTS) return nullptr;
  if ((int)slots.size() < WS_NUM_SLOTS) slots.resize(WS_NUM_SLOTS, {nullptr, 0});
  auto &e = slots[slot];
  if (bytes == 0) bytes = 1;
  if (e.second >= bytes) return e.first;
  if (opt.capture_safe) return nullptr;  // no allocation while a stream may be captured
  if (e.first) {
    hipStreamSynchronize(stream);
    hipFree(e.first);
    e.first = nullptr;
    e.second = 0;
  }
  size_t want = std::max(bytes, e.second + e.second / 4);
  void *p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    want = bytes;
  }
  e.first = p;
  e.second = want;
  return p;
}

gmls_ctx_s::~gmls_ctx_s() {
  hipStreamSynchronize(stream);
  for (auto &e : slots)
    if (e.first) hipFree(e.first);
  for (auto &e : ev)
    if (e) hipEventDestroy(e);
}

gmls_status gmls_set_error(gmls_ctx ctx, gmls_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return st;
}

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
  }
};

int shape_rows(int dim, int basis, unsigned mask) {
  if (basis == GMLS_BASIS_SCALAR) {
    if (mask & GMLS_F_DIV) return -1;
    return ((mask & GMLS_F_VALUE) ? 1 : 0) + ((mask & GMLS_F_GRAD) ? dim : 0) + ((mask & GMLS_F_LAPLACIAN) ? 1 : 0);
  }
  if (mask & GMLS_F_GRAD) return -1;
  return ((mask & GMLS_F_VALUE) ? dim : 0) + ((mask & GMLS_F_LAPLACIAN) ? dim : 0) + ((mask & GMLS_F_DIV) ? 1 : 0);
}

long binom_l(int n, int k) {
  if (k < 0 || k > n) return 0;
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

}  // namespace

#define GMLS_HIP(...)                                                                                     \
  do {                                                                                                     \
    hipError_t e_ = (__VA_ARGS__);                                                                                \
    if (e_ != hipSuccess)                                                                                  \
      return gmls_set_error(ctx, GMLS_ERR_HIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));        \
  } while (0)

extern "C" {

gmls_status gmls_create(gmls_ctx *out, int device, void *hip_stream) {
  if (!out) return GMLS_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return GMLS_ERR_ARG;
  }
  gmls_ctx ctx = new (std::nothrow) gmls_ctx_s();
  if (!ctx) return GMLS_ERR_NOMEM;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->slots.resize(WS_NUM_SLOTS, {nullptr, 0});
  DeviceGuard g(device);
  for (auto &e : ctx->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete ctx;
      return GMLS_ERR_HIP;
    }
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
      ctx->cus = prop.multiProcessorCount;
  }
  void *de = ctx->ws(WS_DEV_ERR, sizeof(int));
  if (!de || fill_zero(de, sizeof(int), ctx->stream) != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess) {
    delete ctx;
    return GMLS_ERR_HIP;
  }
  // the allocation-free product's scratch address on this device (current here)
  if (spmv_scratch_setup(device) != hipSuccess) {
    (void)hipGetLastError();
    delete ctx;
    return GMLS_ERR_HIP;
  }
  *out = ctx;
  return GMLS_OK;
}

void gmls_destroy(gmls_ctx ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  delete ctx;
}

const char *gmls_last_error(gmls_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gmls_status gmls_set_option(gmls_ctx ctx, int option, double value) {
  if (!ctx) return GMLS_ERR_ARG;
  switch (option) {
    case GMLS_OPT_COND_THRESHOLD:
      if (!(value > 0)) return gmls_set_error(ctx, GMLS_ERR_ARG, "condition threshold must be > 0");
      ctx->opt.cond_threshold = value;
      return GMLS_OK;
    case GMLS_OPT_MAX_SWEEPS:
      if (!(value >= 1 && value <= 15)) return gmls_set_error(ctx, GMLS_ERR_ARG, "max sweeps must be 1..15");
      ctx->opt.max_sweeps = (int)value;
      return GMLS_OK;
    case GMLS_OPT_REFINE_TOL:
      if (!(value > 0 && value < 1)) return gmls_set_error(ctx, GMLS_ERR_ARG, "refine tol must be in (0, 1)");
      ctx->opt.refine_tol = value;
      return GMLS_OK;
    case GMLS_OPT_FORCE_FALLBACK:
      ctx->opt.force_fallback = value != 0;
      return GMLS_OK;
    case GMLS_OPT_MIXED_SCHEME:
      if (value != 0 && value != 1 && value != 2 && value != 3 && value != 4)
        return gmls_set_error(ctx, GMLS_ERR_ARG, "mixed scheme must be 0 (auto), 1, 2, 3 or 4");
      ctx->opt.scheme = (int)value;
      return GMLS_OK;
    case GMLS_OPT_PIPE_CHUNK:
      if (!(value >= 0 && value <= 2147483647.0 && value == (double)(int64_t)value))
        return gmls_set_error(ctx, GMLS_ERR_ARG, "pipeline chunk must be an integer in [0, 2^31)");
      if (value != 0 && value < 64) return gmls_set_error(ctx, GMLS_ERR_ARG, "pipeline chunk must be 0 or >= 64");
      ctx->opt.pipe_chunk = (int64_t)value;
      return GMLS_OK;
    case GMLS_OPT_CAPTURE_SAFE:
      ctx->opt.capture_safe = value != 0;
      return GMLS_OK;
    case GMLS_OPT_ROW_ORDER:
      if (value != 0 && value != 1) return gmls_set_error(ctx, GMLS_ERR_ARG, "row order must be 0 (cell) or 1 (index)");
      ctx->opt.row_order = (int)value;
      return GMLS_OK;
    case GMLS_OPT_PIPE_SHAPE:
      if (!(value == (double)(int)value && value >= -1 && value < kPipeCands))
        return gmls_set_error(ctx, GMLS_ERR_ARG, "pipeline shape must be -1 (tuned) or a candidate 0..2");
      ctx->opt.pipe_force = (int)value;
      return GMLS_OK;
    case GMLS_OPT_WAVE_SHAPE:
    case GMLS_OPT_QR_SHAPE:
      if (!(value == (double)(int)value && value >= -1 && value < kPipeCands))
        return gmls_set_error(ctx, GMLS_ERR_ARG, "shape must be -1 (tuned) or a candidate 0..2");
      (option == GMLS_OPT_WAVE_SHAPE ? ctx->opt.wave_force : ctx->opt.qr_force) = (int)value;
      return GMLS_OK;
    case GMLS_OPT_SOURCE_STRIDE:
      if (!(value == (double)(int)value && value >= 0 && value <= 64))
        return gmls_set_error(ctx, GMLS_ERR_ARG, "source stride must be an integer in [0, 64]");
      ctx->opt.source_stride = (int)value;
      return GMLS_OK;
    case GMLS_OPT_RADIUS_SCRATCH_MB:
      if (!(value >= 0 && value <= 1048576.0 && value == (double)(int64_t)value))
        return gmls_set_error(ctx, GMLS_ERR_ARG, "radius scratch must be an integer number of MiB in [0, 2^20]");
      ctx->opt.radius_scratch_mb = (int64_t)value;
      return GMLS_OK;
    default:
      return gmls_set_error(ctx, GMLS_ERR_ARG, "unknown option");
  }
}

gmls_status gmls_stencil_shape(int dim, int order, int basis, unsigned functional_mask, int *F, int *C_in,
                               int *Q) {
  if (dim < 1 || dim > 3 || order < 0 || order > 8 || (basis != GMLS_BASIS_SCALAR && basis != GMLS_BASIS_DIVFREE))
    return GMLS_ERR_ARG;
  if (functional_mask == 0 || (functional_mask & ~15u)) return GMLS_ERR_ARG;
  const int f = shape_rows(dim, basis, functional_mask);
  if (f < 0) return GMLS_ERR_UNSUPPORTED;
  const long qs = binom_l(order + dim, dim);
  const long q = basis == GMLS_BASIS_SCALAR ? qs : dim * qs - (order >= 1 ? binom_l(order - 1 + dim, dim) : 0);
  if (F) *F = f;
  if (C_in) *C_in = basis == GMLS_BASIS_SCALAR ? 1 : dim;
  if (Q) *Q = (int)q;
  return GMLS_OK;
}

static gmls_status neighbors(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                             int64_t n_tgt, int dim, const gmls_search *spec, int64_t *row_ptr, int32_t *col,
                             int64_t col_capacity, double *eps, int64_t *nnz_host, double *records,
                             int32_t *pcol) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  if (!spec || !nnz_host) return gmls_set_error(ctx, GMLS_ERR_ARG, "spec and nnz_host must be non-null");
  if (dim < 1 || dim > 3) return gmls_set_error(ctx, GMLS_ERR_ARG, "dim must be 1, 2 or 3");
  if (n_src < 1 || n_src > (1ll << 28)) return gmls_set_error(ctx, GMLS_ERR_ARG, "n_src must be in [1, 2^28]");
  if (n_tgt < 0 || n_tgt > (1ll << 31) - 1) return gmls_set_error(ctx, GMLS_ERR_ARG, "n_tgt out of range");
  if (!coords || !row_ptr || (n_tgt > 0 && (!targets || !eps)))
    return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer");
  if (col_capacity < 0) return gmls_set_error(ctx, GMLS_ERR_ARG, "col_capacity must be >= 0");
  if (col_capacity > 0 && !col) return gmls_set_error(ctx, GMLS_ERR_ARG, "col is null");
  if (spec->mode == GMLS_SEARCH_KNN) {
    if (spec->k < 1 || spec->k > 1024 || spec->k > n_src)
      return gmls_set_error(ctx, GMLS_ERR_ARG, "knn: k must be in [1, min(1024, n_src)]");
    if (!(spec->eps_mult > 0) || !isfinite(spec->eps_mult))
      return gmls_set_error(ctx, GMLS_ERR_ARG, "knn: eps_mult must be finite and > 0");
    if ((double)n_tgt * spec->k > 2147483647.0 * 4)
      return gmls_set_error(ctx, GMLS_ERR_ARG, "knn: output too large");
  } else if (spec->mode == GMLS_SEARCH_RADIUS) {
    if (!(spec->radius > 0) || !isfinite(spec->radius))
      return gmls_set_error(ctx, GMLS_ERR_ARG, "radius must be finite and > 0");
    if (spec->k_min < 0 || spec->k_min > 1024 || spec->k_min + 1 > n_src)
      return gmls_set_error(ctx, GMLS_ERR_ARG, "radius: k_min must be in [0, min(1024, n_src - 1)]");
  } else {
    return gmls_set_error(ctx, GMLS_ERR_ARG, "unknown search mode");
  }
  DeviceGuard g(ctx->device);
  return run_neighbors(ctx, coords, n_src, targets, n_tgt, dim, *spec, row_ptr, col, col_capacity, eps, nnz_host,
                       records, pcol);
}

gmls_status gmls_neighbors(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                           int64_t n_tgt, int dim, const gmls_search *spec, int64_t *row_ptr, int32_t *col,
                           int64_t col_capacity, double *eps, int64_t *nnz_host) {
  return neighbors(ctx, coords, n_src, targets, n_tgt, dim, spec, row_ptr, col, col_capacity, eps, nnz_host, nullptr,
                   nullptr);
}

gmls_status gmls_neighbors_sorted(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                                  int64_t n_tgt, int dim, const gmls_search *spec, int64_t *row_ptr, int32_t *col,
                                  int64_t col_capacity, double *eps, int64_t *nnz_host, double *sources_sorted,
                                  int32_t *col_sorted) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  if (!sources_sorted || (col_capacity > 0 && !col_sorted))
    return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer (sources_sorted, col_sorted)");
  if (col_sorted && col_sorted == col) return gmls_set_error(ctx, GMLS_ERR_ARG, "col_sorted must not alias col");
  return neighbors(ctx, coords, n_src, targets, n_tgt, dim, spec, row_ptr, col, col_capacity, eps, nnz_host,
                   sources_sorted, col_sorted);
}

}  // extern "C"


// Device buffers of a report: the per-target condition numbers of the mixed
// kernels (NaN where none was computed) and the counters, both cleared.
static gmls_status report_begin(gmls_ctx ctx, int n, float **cond, ReportCounts **rc) {
  *cond = (float *)ctx->ws(WS_COND, sizeof(float) * (size_t)n);
  *rc = (ReportCounts *)ctx->ws(WS_REPORT, sizeof(ReportCounts));
  if (!*cond || !*rc) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed (report)");
  GMLS_HIP(fill_f32(*cond, NAN, n, ctx->stream));
  GMLS_HIP(fill_zero(*rc, sizeof(ReportCounts), ctx->stream));
  return GMLS_OK;
}

// The report of a stencil call (synchronises): target counts by status over
// the call's status arrays (one per stencil set), the refinement histogram
// and largest condition number from the mixed kernels' statistics (n_stats
// records), the smallest and median condition number over the targets whose
// Gram the mixed kernels factored, the phase times between events 0..3, and
// the time of the context's last search.
static gmls_status report_end(gmls_ctx ctx, gmls_report *report, int n, const uint8_t *const *status, int n_sets,
                              const Stats *stats, int n_stats, const float *cond, ReportCounts *rc) {
  hipStream_t s = ctx->stream;
  for (int k = 0; k < n_sets; ++k) GMLS_HIP(launch_status_count(status[k], n, rc, s));
  GMLS_HIP(launch_cond_stats(cond, n, rc, s));
  Stats hs[2];
  ReportCounts hr;
  GMLS_HIP(hipMemcpyAsync(hs, stats, sizeof(Stats) * (size_t)n_stats, hipMemcpyDeviceToHost, s));
  GMLS_HIP(hipMemcpyAsync(&hr, rc, sizeof(ReportCounts), hipMemcpyDeviceToHost, s));
  GMLS_HIP(hipStreamSynchronize(s));
  float t01 = 0, t12 = 0, t23 = 0;
  hipEventElapsedTime(&t01, ctx->ev[0], ctx->ev[1]);
  hipEventElapsedTime(&t12, ctx->ev[1], ctx->ev[2]);
  hipEventElapsedTime(&t23, ctx->ev[2], ctx->ev[3]);
  memset(report, 0, sizeof(*report));
  report->n_targets = (int64_t)n * n_sets;
  report->n_rank_deficient = (int64_t)hr.status[GMLS_TARGET_RANK_DEFICIENT];
  report->n_fallback = (int64_t)hr.status[GMLS_TARGET_FALLBACK];
  report->n_not_converged = (int64_t)hr.status[GMLS_TARGET_NOT_CONVERGED];
  report->n_ok = report->n_targets - report->n_rank_deficient;
  double cmax = 0.0;
  for (int k = 0; k < n_stats; ++k) {
    for (int i = 0; i < 16; ++i) report->sweep_hist[i] += (int32_t)hs[k].sweep_hist[i];
    double c;
    memcpy(&c, &hs[k].cond_max_bits, sizeof(double));
    cmax = std::max(cmax, c);
  }
  report->cond_max = cmax;
  if (hr.n_cond > 0) {
    const unsigned int bits = ~hr.cond_min_inv;
    float cmin;
    memcpy(&cmin, &bits, sizeof(float));
    report->cond_min = cmin;
    const unsigned long long half = (hr.n_cond + 1) / 2;
    unsigned long long cum = 0;
    for (int b = 0; b < kCondBins; ++b) {
      cum += hr.cond_hist[b];
      if (cum >= half) {
        report->cond_med = exp2((b + 0.5) / kCondBinsPerOctave);
        break;
      }
    }
  }
  report->t_bin_ms = t01;
  report->t_stencil_ms = t12;
  report->t_fallback_ms = t23;
  report->t_search_ms = ctx->t_search_ms;
  return report->n_rank_deficient > 0 ? GMLS_WARN_TARGET_FLAGS : GMLS_OK;
}

// plain (normals == nullptr), Neumann-constrained and staggered
// (basis == kBasisStaggered) stencils
// key of the autotune table
static int tune_key(int dim, int order, int basis) { return (dim * 8 + order) * 4 + basis; }

// The per-bin candidates of one call: forced by an option, else the tuned
// table's entry under `key`, else candidate 0.  pipe_key: the key of the
// pipeline's shapes (a shared call runs each set's own pipeline).
static void resolve_shapes(gmls_ctx ctx, int key, int pipe_key, Options &o) {
  const auto it = ctx->tune.find(key), ip = ctx->tune.find(pipe_key);
  auto pick = [&](decltype(it) e, int k, int b, int force) -> signed char {
    if (force >= 0) return (signed char)force;
    if (e != ctx->tune.end() && e->second[k * 8 + b] >= 0) return e->second[k * 8 + b];
    return 0;
  };
  for (int b = 0; b < 8; ++b) {
    o.pipe_shape[0][b] = pick(ip, 0, b, o.pipe_force);
    o.pipe_shape[1][b] = pick(ip, 1, b, o.pipe_force);
    o.wave_shape[b] = pick(it, 2, b, o.wave_force);
    o.qr_shape[b] = pick(it, 3, b, o.qr_force);
  }
}

// The FP64 QR kernel on row-count bin b (scalar, divergence-free or
// staggered; or, with av, both sets of a shared call) in the bin's shape,
// bracketed by the autotuner's events when it is timing.
static hipError_t qr_bin(gmls_ctx ctx, const Options &o, int dim, int order, int basis, int b, int cnt,
                         const StencilArgs &a, const StencilArgs *av, const int *list, BinMeta *meta,
                         hipStream_t s) {
  const QrShape q = kQrShapes[b][o.qr_shape[b]];
  const int nb = std::min(cnt, ctx->cus * q.per_cu);
  PipeTimer *tm = ctx->timer;
  hipError_t e = tm ? hipEventRecord(tm->ev[3][b][0], s) : hipSuccess;
  if (e == hipSuccess)
    e = av ? launch_qr_shared_bin(dim, order, b, q.rpl, q.wpe, a, *av, list, meta, nb, s)
           : launch_qr_bin(dim, order, basis, b, q.rpl, q.wpe, a, list, meta, nb, s);
  if (e == hipSuccess && tm) {
    e = hipEventRecord(tm->ev[3][b][1], s);
    tm->used[3][b] = 1;
  }
  return e;
}

static gmls_status run_stencils(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                                int64_t n_tgt, int dim, int order, int basis, unsigned functional_mask, int weight_p,
                                const double *eps, const int64_t *row_ptr, const int32_t *col,
                                const double *normals, int prec, double *weights, double *hweights,
                                uint8_t *target_status, gmls_report *report) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  int F = 0, C = 0, Q = 0;
  const bool stag = basis == kBasisStaggered;
  gmls_status st = gmls_stencil_shape(dim, order, stag ? GMLS_BASIS_SCALAR : basis, functional_mask, &F, &C, &Q);
  if (st != GMLS_OK) return gmls_set_error(ctx, st, "functional/basis combination not supported or bad shape");
  // the mixed kernels of a staggered call are the scalar pipeline's with
  // the constant column dropped; its FP64 QR kernels (and fallback) are basis 2
  const int mbasis = stag ? (int)GMLS_BASIS_SCALAR : basis;
  if (stag) {
    Q -= 1;  // no constant monomial
    if (n_tgt > 0 && !hweights) return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer (target_weights)");
  }
  if (!qr_supported(dim, order, basis))
    return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "compiled kernels cover dim 2-3 and order 1-4");
  if (prec != GMLS_PREC_FP64 && prec != GMLS_PREC_MIXED) return gmls_set_error(ctx, GMLS_ERR_ARG, "bad precision");
  if (prec == GMLS_PREC_MIXED && !mixed_supported(dim, order, mbasis))
    return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "mixed precision not compiled for this basis/order");
  Options opt = ctx->opt;
  if (prec == GMLS_PREC_MIXED) {
    opt.scheme = mixed_scheme(dim, order, mbasis, stag ? (int)MIXED_PIPE : ctx->opt.scheme);
    if (opt.scheme < 0)
      return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED,
                            stag ? "mixed staggered stencils need the pipeline (at most 20 monomials of degree "
                                   "order + 1)"
                                 : "the selected mixed scheme is not compiled for this shape");
  }
  if (weight_p < 1 || weight_p > 12) return gmls_set_error(ctx, GMLS_ERR_ARG, "weight power must be 1..12");
  if (n_src < 1 || n_tgt < 0 || n_tgt > (1ll << 31) - 1)
    return gmls_set_error(ctx, GMLS_ERR_ARG, "n_src must be >= 1 and n_tgt in [0, 2^31)");
  if (n_tgt > 0 && (!coords || !targets || !eps || !row_ptr || !col || !weights))
    return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer");
  const int cstride = ctx->opt.source_stride ? ctx->opt.source_stride : dim;
  if (cstride < dim) return gmls_set_error(ctx, GMLS_ERR_ARG, "source stride is smaller than dim");
  if (normals) {
    if (basis != GMLS_BASIS_SCALAR)
      return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "the Neumann constraint is implemented for the scalar basis");
    if (prec != GMLS_PREC_FP64)
      return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "constrained stencils are computed in FP64 (GMLS_PREC_FP64)");
    if (n_tgt > 0 && !hweights) return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer (h_weights)");
  }
  if (report) memset(report, 0, sizeof(*report));
  if (n_tgt == 0) return GMLS_OK;
  DeviceGuard g(ctx->device);
  hipStream_t s = ctx->stream;
  const int n = (int)n_tgt;
  BinMeta *meta = (BinMeta *)ctx->ws(WS_BIN_META, sizeof(BinMeta));
  int *list = (int *)ctx->ws(WS_BIN_LIST, sizeof(int) * (size_t)n);
  int *fb = (int *)ctx->ws(WS_FALLBACK, sizeof(int) * (size_t)n);
  Stats *stats = (Stats *)ctx->ws(WS_STATS, sizeof(Stats));
  uint8_t *status = target_status ? target_status : (uint8_t *)ctx->ws(WS_STATUS_TMP, (size_t)n);
  if (!meta || !list || !fb || !stats || !status)
    return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed");

  StencilArgs a;
  a.coords = coords;
  a.cstride = cstride;
  a.targets = targets;
  a.eps = eps;
  a.row_ptr = row_ptr;
  a.col = col;
  a.weights = weights;
  a.status = status;
  a.mask = functional_mask;
  a.F = F;
  a.p = weight_p;
  a.n_tgt = n;
  a.ok_status = GMLS_TARGET_OK;
  a.normals = normals;
  a.hweights = hweights;
  a.skip_const = stag ? 1 : 0;
  if (basis == GMLS_BASIS_DIVFREE) {  // queue of targets whose scalar basis is not unisolvent
    a.aux_list = (int *)ctx->ws(WS_AUX_LIST, sizeof(int) * (size_t)n);
    if (!a.aux_list) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed");
    a.aux_count = &meta->aux_count;  // cleared with the bin table
  }

  const bool sync = !opt.capture_safe;  // capture-safe: nothing below waits for the device
  if (!sync && report)
    return gmls_set_error(ctx, GMLS_ERR_ARG, "a report synchronises: pass NULL in capture-safe mode");
  float *cond = nullptr;
  ReportCounts *rc = nullptr;
  if (report) {
    st = report_begin(ctx, n, &cond, &rc);
    if (st != GMLS_OK) return st;
    a.cond_out = cond;
  }
  if (report) GMLS_HIP(hipEventRecord(ctx->ev[0], s));
  const size_t bin_bytes = binning_temp_bytes(n);
  void *bin_tmp = ctx->ws(WS_BIN_TEMP, bin_bytes);
  if (!bin_tmp) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed");
  GMLS_HIP(launch_binning(row_ptr, targets, n, dim, Q, C, meta, list, bin_tmp, bin_bytes, s));
  BinMeta hm;
  if (sync) {
    GMLS_HIP(hipMemcpyAsync(&hm, meta, sizeof(BinMeta), hipMemcpyDeviceToHost, s));
    GMLS_HIP(hipStreamSynchronize(s));
    if (hm.err) return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "a target has more than 2^24 neighbours");
  } else {
    // rows over the compiled maximum stay in bin 7 (never processed) and are
    // reported by gmls_check
    GMLS_HIP(or_error_bit((int *)ctx->ws(WS_DEV_ERR, sizeof(int)), &meta->err, 1, DEV_ERR_STENCIL_ROWS, s));
  }
  GMLS_HIP(fill_zero(stats, sizeof(Stats), s));
  if (report) GMLS_HIP(hipEventRecord(ctx->ev[1], s));
  if (!sync || hm.count[0] > 0) GMLS_HIP(launch_rank_deficient(a, C, list, meta, s));
  const int cus = ctx->cus;
  // shapes of the pipeline, wavefront and QR kernels: forced, tuned or default
  resolve_shapes(ctx, tune_key(dim, order, basis), tune_key(dim, order, mbasis), opt);
  if (prec == GMLS_PREC_MIXED && opt.scheme == MIXED_PIPE) {
    // moments [chunk][NM], solutions [chunk][F][Q] and records of one chunk of targets
    // (sized for every target, so that a capture-safe call finds the
    // workspace of an earlier call of the same size)
    const int64_t n_work = sync ? (int64_t)n - hm.count[0] : (int64_t)n;
    const int64_t chunk =
        std::max<int64_t>(1, sync && opt.pipe_chunk > 0 ? std::min<int64_t>(opt.pipe_chunk, n_work) : n_work);
    const size_t cap = (size_t)(sync && opt.pipe_chunk > 0 ? chunk : (int64_t)n);
    double *mom = (double *)ctx->ws(WS_PIPE_MOM, sizeof(double) * (size_t)pipe_num_moments(dim, order) * cap);
    // per target: F*Q solution values (scalar), F*C*Q_s coefficients (divergence-free)
    const int qy = basis == GMLS_BASIS_DIVFREE ? C * (int)binom_l(order + dim, dim) : Q;
    double *yb = (double *)ctx->ws(WS_PIPE_Y, sizeof(double) * (size_t)F * qy * cap);
    void *rec = ctx->ws(WS_PIPE_REC, kPipeRecBytes * cap);
    if (!mom || !yb || !rec) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed");
    if (n_work > 0)
      GMLS_HIP(launch_mixed_pipe(dim, order, mbasis, a, list, sync ? &hm : nullptr, meta, fb, stats, opt, mom, yb,
                                 rec, chunk, n, cus, ctx->timer, s));
  } else if (prec == GMLS_PREC_MIXED && opt.scheme == MIXED_WAVE) {
    if (!sync || hm.count[0] < n)
      GMLS_HIP(launch_mixed_wave(dim, order, mbasis, a, list, sync ? &hm : nullptr, meta, fb, stats, opt, n, cus,
                                 ctx->timer, s));
  } else {
    for (int b = 1; b < kNumBins; ++b) {
      if (sync && hm.count[b] == 0) continue;
      const int cnt = sync ? hm.count[b] : n;  // sizes the grid; the kernels read the count on the device
      if (prec == GMLS_PREC_FP64) {
        GMLS_HIP(qr_bin(ctx, opt, dim, order, basis, b, cnt, a, nullptr, list, meta, s));
      } else if (b == kLongBin) {  // the fused kernels hold at most 256 rows: FP64 QR in chunks
        GMLS_HIP(launch_defer_bin(a.status, list, meta, b, fb, &meta->fb_count, stats, s));
      } else {
        GMLS_HIP(launch_mixed_bin(dim, order, basis, b, a, list, meta, fb, stats, opt, cnt, cus, s));
      }
    }
  }
  if (report) GMLS_HIP(hipEventRecord(ctx->ev[2], s));
  StencilArgs af = a;
  if (prec == GMLS_PREC_MIXED) {
    af.ok_status = -1;  // keep the fallback/not-converged status set by the mixed kernel
    GMLS_HIP(launch_qr_fallback(dim, order, basis, af, fb, meta, 4, cus * 8, s));
  }
  if (basis == GMLS_BASIS_DIVFREE)  // the queue is usually empty: a small persistent grid
    GMLS_HIP(launch_qr_kmat(dim, order, af, a.aux_list, &meta->aux_count, &meta->aux_cursor, 64, s));
  if (report) GMLS_HIP(hipEventRecord(ctx->ev[3], s));
  if (!report) return GMLS_OK;
  const uint8_t *sts[1] = {status};
  return report_end(ctx, report, n, sts, 1, stats, 1, cond, rc);
}

// A scalar set (ss) and a divergence-free set (sv) on the same neighbour
// lists.  FP64 (scheme < 0): one QR kernel takes the Householder factor of
// each target once for both sets.  Mixed precision, the same scheme for both:
// with the wavefront scheme one kernel forms the moments and the swept Gram
// of each target once for both; with the pipeline the moments (and
// per-target records) of the scalar set's run are taken by the
// divergence-free set's solve and weights.  Bins follow the scalar basis
// (bin 0: N < Q_s); the divergence-free set's bin-0 targets, which its own
// call would have handled through the FP64 kernel's queue, go to that kernel
// directly.
static gmls_status run_shared(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                              int64_t n_tgt, int dim, int order, int weight_p, const double *eps,
                              const int64_t *row_ptr, const int32_t *col, const gmls_stencil_set &ss,
                              const gmls_stencil_set &sv, int scheme, gmls_report *report) {
  int Fs = 0, Cs = 0, Qs = 0, Fv = 0, Cv = 0, Qv = 0;
  gmls_status st = gmls_stencil_shape(dim, order, GMLS_BASIS_SCALAR, ss.functional_mask, &Fs, &Cs, &Qs);
  if (st == GMLS_OK) st = gmls_stencil_shape(dim, order, GMLS_BASIS_DIVFREE, sv.functional_mask, &Fv, &Cv, &Qv);
  if (st != GMLS_OK) return gmls_set_error(ctx, st, "functional/basis combination not supported or bad shape");
  if (weight_p < 1 || weight_p > 12) return gmls_set_error(ctx, GMLS_ERR_ARG, "weight power must be 1..12");
  if (n_src < 1 || n_tgt < 0 || n_tgt > (1ll << 31) - 1)
    return gmls_set_error(ctx, GMLS_ERR_ARG, "n_src must be >= 1 and n_tgt in [0, 2^31)");
  if (n_tgt > 0 && (!coords || !targets || !eps || !row_ptr || !col || !ss.weights || !sv.weights))
    return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer");
  const int cstride = ctx->opt.source_stride ? ctx->opt.source_stride : dim;
  if (cstride < dim) return gmls_set_error(ctx, GMLS_ERR_ARG, "source stride is smaller than dim");
  if (report) memset(report, 0, sizeof(*report));
  if (n_tgt == 0) return GMLS_OK;
  DeviceGuard g(ctx->device);
  hipStream_t s = ctx->stream;
  const int n = (int)n_tgt;
  Options opt = ctx->opt;
  opt.scheme = scheme;
  // the shared kernels' shapes (wavefront, QR) are tuned under their own key
  resolve_shapes(ctx, tune_key(dim, order, kTuneShared), tune_key(dim, order, 0), opt);
  BinMeta *meta = (BinMeta *)ctx->ws(WS_BIN_META, sizeof(BinMeta));
  int *list = (int *)ctx->ws(WS_BIN_LIST, sizeof(int) * (size_t)n);
  int *fbs = (int *)ctx->ws(WS_FALLBACK, sizeof(int) * (size_t)n);
  int *fbv = (int *)ctx->ws(WS_FALLBACK2, sizeof(int) * (size_t)n);
  int *aux = (int *)ctx->ws(WS_AUX_LIST, sizeof(int) * (size_t)n);
  Stats *stats = (Stats *)ctx->ws(WS_STATS, 2 * sizeof(Stats));  // [0] scalar set (reported), [1] the other
  uint8_t *sts = ss.target_status ? ss.target_status : (uint8_t *)ctx->ws(WS_STATUS_TMP, (size_t)n);
  uint8_t *stv = sv.target_status ? sv.target_status : (uint8_t *)ctx->ws(WS_STATUS_TMP2, (size_t)n);
  if (!meta || !list || !fbs || !fbv || !aux || !stats || !sts || !stv)
    return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed");
  StencilArgs as;
  as.coords = coords;
  as.cstride = cstride;
  as.targets = targets;
  as.eps = eps;
  as.row_ptr = row_ptr;
  as.col = col;
  as.weights = ss.weights;
  as.status = sts;
  as.mask = ss.functional_mask;
  as.F = Fs;
  as.p = weight_p;
  as.n_tgt = n;
  as.ok_status = GMLS_TARGET_OK;
  StencilArgs av = as;
  av.weights = sv.weights;
  av.status = stv;
  av.mask = sv.functional_mask;
  av.F = Fv;
  av.aux_list = aux;
  av.aux_count = &meta->aux_count;

  const bool sync = !opt.capture_safe;
  if (!sync && report)
    return gmls_set_error(ctx, GMLS_ERR_ARG, "a report synchronises: pass NULL in capture-safe mode");
  float *cond = nullptr;
  ReportCounts *rc = nullptr;
  if (report) {  // the condition numbers of the shared scalar Gram
    st = report_begin(ctx, n, &cond, &rc);
    if (st != GMLS_OK) return st;
    as.cond_out = cond;
  }
  if (report) GMLS_HIP(hipEventRecord(ctx->ev[0], s));
  const size_t bin_bytes = binning_temp_bytes(n);
  void *bin_tmp = ctx->ws(WS_BIN_TEMP, bin_bytes);
  if (!bin_tmp) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed");
  GMLS_HIP(launch_binning(row_ptr, targets, n, dim, Qs, 1, meta, list, bin_tmp, bin_bytes, s));
  BinMeta hm;
  if (sync) {
    GMLS_HIP(hipMemcpyAsync(&hm, meta, sizeof(BinMeta), hipMemcpyDeviceToHost, s));
    GMLS_HIP(hipStreamSynchronize(s));
    if (hm.err) return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "a target has more than 2^24 neighbours");
  } else {
    GMLS_HIP(or_error_bit((int *)ctx->ws(WS_DEV_ERR, sizeof(int)), &meta->err, 1, DEV_ERR_STENCIL_ROWS, s));
  }
  GMLS_HIP(fill_zero(stats, 2 * sizeof(Stats), s));
  if (report) GMLS_HIP(hipEventRecord(ctx->ev[1], s));
  // the FP64 kernels' targets were computed outside the mixed path: status 2
  StencilArgs afv = av;
  afv.ok_status = scheme < 0 ? GMLS_TARGET_OK : GMLS_TARGET_FALLBACK;
  if (!sync || hm.count[0] > 0) {
    GMLS_HIP(launch_rank_deficient(as, 1, list, meta, s));
    GMLS_HIP(launch_qr_bin(dim, order, GMLS_BASIS_DIVFREE, 0, 4, 0, afv, list, meta, ctx->cus * 8, s));
  }
  StencilArgs afs = as;
  afs.ok_status = -1;  // keep the fallback status set by the mixed kernel
  StencilArgs afv2 = av;
  afv2.ok_status = -1;
  if (scheme < 0) {
    for (int b = 1; b < kNumBins; ++b) {
      if (sync && hm.count[b] == 0) continue;
      const int cnt = sync ? hm.count[b] : n;  // sizes the grid; the kernel reads the count on the device
      GMLS_HIP(qr_bin(ctx, opt, dim, order, 0, b, cnt, as, &av, list, meta, s));
    }
    if (report) GMLS_HIP(hipEventRecord(ctx->ev[2], s));
  } else if (scheme == MIXED_WAVE) {
    GMLS_HIP(launch_mixed_wave_shared(dim, order, as, fbs, &meta->fb_count, av, fbv, &meta->fb2_count, list,
                                      sync ? &hm : nullptr, meta, stats, opt, n, ctx->cus, ctx->timer, s));
    if (report) GMLS_HIP(hipEventRecord(ctx->ev[2], s));
    GMLS_HIP(launch_qr_fallback(dim, order, GMLS_BASIS_SCALAR, afs, fbs, meta, 4, ctx->cus * 8, s));
  } else {
    // pipeline: the whole list in one window; the scalar set (prep, moments,
    // solve, weights) and its fallback, then the divergence-free set's solve
    // and weights on the same records and moments, with the fallback queue
    // cleared in between
    const int qs = (int)binom_l(order + dim, dim);
    double *mom = (double *)ctx->ws(WS_PIPE_MOM, sizeof(double) * (size_t)pipe_num_moments(dim, order) * n);
    double *ys = (double *)ctx->ws(WS_PIPE_Y, sizeof(double) * (size_t)as.F * qs * n);
    double *yv = (double *)ctx->ws(WS_PIPE_Y2, sizeof(double) * (size_t)av.F * dim * qs * n);
    void *rec = ctx->ws(WS_PIPE_REC, kPipeRecBytes * (size_t)n);
    if (!mom || !ys || !yv || !rec) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed");
    Options os = opt, ov = opt;  // each set's own pipeline shapes
    resolve_shapes(ctx, tune_key(dim, order, kTuneShared), tune_key(dim, order, 0), os);
    resolve_shapes(ctx, tune_key(dim, order, kTuneShared), tune_key(dim, order, 1), ov);
    ov.reuse_moments = 1;
    GMLS_HIP(launch_mixed_pipe(dim, order, GMLS_BASIS_SCALAR, as, list, sync ? &hm : nullptr, meta, fbs, stats, os,
                               mom, ys, rec, n, n, ctx->cus, nullptr, s));
    GMLS_HIP(launch_qr_fallback(dim, order, GMLS_BASIS_SCALAR, afs, fbs, meta, 4, ctx->cus * 8, s));
    GMLS_HIP(fill_zero(&meta->fb_count, 2 * sizeof(int), s));  // fb_count, fb_cursor
    GMLS_HIP(launch_mixed_pipe(dim, order, GMLS_BASIS_DIVFREE, av, list, sync ? &hm : nullptr, meta, fbv, stats + 1, ov,
                               mom, yv, rec, n, n, ctx->cus, nullptr, s));
    if (report) GMLS_HIP(hipEventRecord(ctx->ev[2], s));
    GMLS_HIP(launch_qr_fallback(dim, order, GMLS_BASIS_DIVFREE, afv2, fbv, meta, 4, ctx->cus * 8, s));
  }
  if (scheme == MIXED_WAVE)
    GMLS_HIP(launch_qr_queue(dim, order, GMLS_BASIS_DIVFREE, afv2, fbv, &meta->fb2_count, &meta->fb2_cursor,
                             ctx->cus * 8, s));
  GMLS_HIP(launch_qr_kmat(dim, order, afv, aux, &meta->aux_count, &meta->aux_cursor, 64, s));
  if (report) GMLS_HIP(hipEventRecord(ctx->ev[3], s));
  if (!report) return GMLS_OK;
  const uint8_t *stl[2] = {sts, stv};
  return report_end(ctx, report, n, stl, 2, stats, scheme < 0 ? 1 : 2, cond, rc);
}

extern "C" {

gmls_status gmls_stencils(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                          int64_t n_tgt, int dim, int order, int basis, unsigned functional_mask, int weight_p,
                          const double *eps, const int64_t *row_ptr, const int32_t *col, int prec,
                          double *weights, uint8_t *target_status, gmls_report *report) {
  return run_stencils(ctx, coords, n_src, targets, n_tgt, dim, order, basis, functional_mask, weight_p, eps, row_ptr,
                      col, nullptr, prec, weights, nullptr, target_status, report);
}

gmls_status gmls_stencils_multi(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                                int64_t n_tgt, int dim, int order, int weight_p, const double *eps,
                                const int64_t *row_ptr, const int32_t *col, int prec, int n_sets,
                                const gmls_stencil_set *sets, gmls_report *report) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  if (!sets || n_sets < 1 || n_sets > 8)
    return gmls_set_error(ctx, GMLS_ERR_ARG, "n_sets must be in 1..8, with a host array of sets");
  int is = -1, iv = -1;
  for (int k = 0; k < n_sets; ++k) {
    if (sets[k].basis != GMLS_BASIS_SCALAR && sets[k].basis != GMLS_BASIS_DIVFREE)
      return gmls_set_error(ctx, GMLS_ERR_ARG, "a set's basis must be GMLS_BASIS_SCALAR or GMLS_BASIS_DIVFREE");
    (sets[k].basis == GMLS_BASIS_SCALAR ? is : iv) = k;
  }
  const bool pair = n_sets == 2 && is >= 0 && iv >= 0 && (dim == 2 || dim == 3) && order >= 1 && order <= 4;
  int scheme = -2;  // -1: FP64, shared factor
  if (pair && prec == GMLS_PREC_FP64) {
    scheme = -1;
  } else if (pair && prec == GMLS_PREC_MIXED) {
    const int s0 = mixed_scheme(dim, order, GMLS_BASIS_SCALAR, ctx->opt.scheme);
    const int s1 = mixed_scheme(dim, order, GMLS_BASIS_DIVFREE, ctx->opt.scheme);
    if (s0 == s1 && (s0 == MIXED_WAVE || s0 == MIXED_PIPE)) scheme = s0;
  }
  if (scheme >= -1)
    return run_shared(ctx, coords, n_src, targets, n_tgt, dim, order, weight_p, eps, row_ptr, col, sets[is],
                      sets[iv], scheme, report);
  gmls_status ret = GMLS_OK;
  gmls_report acc;
  for (int k = 0; k < n_sets; ++k) {
    gmls_report r;
    const gmls_status st = run_stencils(ctx, coords, n_src, targets, n_tgt, dim, order, sets[k].basis,
                                        sets[k].functional_mask, weight_p, eps, row_ptr, col, nullptr, prec,
                                        sets[k].weights, nullptr, sets[k].target_status, report ? &r : nullptr);
    if (st != GMLS_OK && st != GMLS_WARN_TARGET_FLAGS) return st;
    if (st == GMLS_WARN_TARGET_FLAGS) ret = st;
    if (k == 0) {
      if (report) acc = r;
    } else if (report) {  // counts summed over the sets; condition figures: min, max, sets[0]'s median
      acc.n_targets += r.n_targets;
      acc.n_ok += r.n_ok;
      acc.n_rank_deficient += r.n_rank_deficient;
      acc.n_fallback += r.n_fallback;
      acc.n_not_converged += r.n_not_converged;
      for (int i = 0; i < 16; ++i) acc.sweep_hist[i] += r.sweep_hist[i];
      acc.cond_max = std::max(acc.cond_max, r.cond_max);
      if (r.cond_min > 0 && (acc.cond_min == 0 || r.cond_min < acc.cond_min)) acc.cond_min = r.cond_min;
      acc.t_bin_ms += r.t_bin_ms;
      acc.t_stencil_ms += r.t_stencil_ms;
      acc.t_fallback_ms += r.t_fallback_ms;
    }
  }
  if (report) *report = acc;
  return ret;
}

gmls_status gmls_stencils_constrained(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                                      int64_t n_tgt, int dim, int order, unsigned functional_mask, int weight_p,
                                      const double *eps, const int64_t *row_ptr, const int32_t *col,
                                      const double *normals, int prec, double *weights, double *h_weights,
                                      uint8_t *target_status, gmls_report *report) {
  if (!ctx) return GMLS_ERR_ARG;
  if (n_tgt > 0 && !normals) return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer (normals)");
  static const double kNoNormal = 0.0;
  return run_stencils(ctx, coords, n_src, targets, n_tgt, dim, order, GMLS_BASIS_SCALAR, functional_mask, weight_p,
                      eps, row_ptr, col, n_tgt > 0 ? normals : &kNoNormal, prec, weights, h_weights, target_status,
                      report);
}

gmls_status gmls_stencils_staggered(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                                    int64_t n_tgt, int dim, int order, unsigned functional_mask, int weight_p,
                                    const double *eps, const int64_t *row_ptr, const int32_t *col, int prec,
                                    double *weights, double *target_weights, uint8_t *target_status,
                                    gmls_report *report) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  if (functional_mask == 0 || (functional_mask & ~(unsigned)(GMLS_F_GRAD | GMLS_F_LAPLACIAN)))
    return gmls_set_error(ctx, GMLS_ERR_ARG, "staggered stencils provide GMLS_F_GRAD and GMLS_F_LAPLACIAN only");
  if (order < 0 || order > 3)
    return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "staggered vector order must be 0..3");
  return run_stencils(ctx, coords, n_src, targets, n_tgt, dim, order + 1, kBasisStaggered, functional_mask, weight_p,
                      eps, row_ptr, col, nullptr, prec, weights, target_weights, target_status, report);
}

gmls_status gmls_assemble_stokes(gmls_ctx ctx, const gmls_stokes_stencils *st, double nu, int64_t *a_row_ptr,
                                 int32_t *a_col, double *a_val, int64_t capacity, int64_t *nnz_host) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  if (!st || !nnz_host) return gmls_set_error(ctx, GMLS_ERR_ARG, "null host pointer");
  if (ctx->opt.capture_safe) return gmls_set_error(ctx, GMLS_ERR_ARG, "the assembly synchronises (capture-safe mode)");
  if (st->dim != 2 && st->dim != 3) return gmls_set_error(ctx, GMLS_ERR_ARG, "dim must be 2 or 3");
  if (st->n < 1 || (int64_t)st->dim * st->n + st->n + 1 >= (1ll << 31))
    return gmls_set_error(ctx, GMLS_ERR_ARG, "n must be >= 1 with dim*n + n + 1 < 2^31");
  if (!st->row_ptr || !st->col || !st->boundary || !st->normals || !st->vlap || !st->grad || !st->plap ||
      !st->plap_t || !st->nlap || !st->nlap_h || !a_row_ptr || (capacity > 0 && (!a_col || !a_val)))
    return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer");
  if (!(nu > 0)) return gmls_set_error(ctx, GMLS_ERR_ARG, "nu must be > 0");
  DeviceGuard g(ctx->device);
  hipStream_t s = ctx->stream;
  StokesArgs a;
  a.n = st->n;
  a.dim = st->dim;
  a.nu = nu;
  a.row_ptr = st->row_ptr;
  a.col = st->col;
  a.boundary = st->boundary;
  a.normals = st->normals;
  a.vlap = st->vlap;
  a.grad = st->grad;
  a.plap = st->plap;
  a.plap_t = st->plap_t;
  a.nlap = st->nlap;
  a.nlap_h = st->nlap_h;
  const int64_t rows = (int64_t)st->dim * st->n + st->n + 1;
  int64_t *rlen = (int64_t *)ctx->ws(WS_STOKES_LEN, sizeof(int64_t) * (size_t)(rows + 1));
  int64_t *tmp = (int64_t *)ctx->ws(WS_STOKES_TMP, sizeof(int64_t) * (size_t)scan_i32_tmp_words(rows + 1));
  int *flags = (int *)ctx->ws(WS_STOKES_FLAG, sizeof(int));
  if (!rlen || !tmp || !flags) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed");
  GMLS_HIP(launch_stokes_assembly(a, rlen, a_row_ptr, tmp, a_col, a_val, capacity, flags, ctx->cus, s));
  int64_t nnz = 0;
  GMLS_HIP(hipMemcpyAsync(&nnz, a_row_ptr + rows, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  GMLS_HIP(hipStreamSynchronize(s));
  *nnz_host = nnz;
  if (nnz > capacity)
    return gmls_set_error(ctx, GMLS_ERR_CAPACITY,
                          "capacity " + std::to_string(capacity) + " < required " + std::to_string(nnz));
  return GMLS_OK;
}

gmls_status gmls_spmv(gmls_ctx ctx, int64_t n_rows, const int64_t *row_ptr, const int32_t *col, const double *val,
                      const double *x, double *y) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  if (n_rows < 0 || n_rows >= (1ll << 31)) return gmls_set_error(ctx, GMLS_ERR_ARG, "n_rows must be in [0, 2^31)");
  if (n_rows == 0) return GMLS_OK;
  if (!row_ptr || !col || !val || !x || !y) return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer");
  DeviceGuard g(ctx->device);
  int *lr = (int *)ctx->ws(WS_SPMV_LONG, sizeof(int) * (size_t)(n_rows + 1));
  if (!lr) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed");
  GMLS_HIP(launch_spmv(n_rows, row_ptr, col, val, x, y, lr + 1, lr, ctx->cus, ctx->stream));
  return GMLS_OK;
}

gmls_status gmls_spmv_noalloc(gmls_ctx ctx, int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                              const double *val, const double *x, double *y) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  if (n_rows < 0 || n_rows > kNoAllocSpmvRows)
    return gmls_set_error(ctx, GMLS_ERR_ARG,
                          "gmls_spmv_noalloc takes 0 .. " + std::to_string(kNoAllocSpmvRows) + " rows");
  if (n_rows == 0) return GMLS_OK;
  if (!row_ptr || !col || !val || !x || !y) return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer");
  int *sp = spmv_scratch(ctx->device);
  if (!sp) return gmls_set_error(ctx, GMLS_ERR_HIP, "the scratch of gmls_spmv_noalloc was not set up on this device");
  DeviceGuard g(ctx->device);
  // the counter at word 0 is cleared by a kernel of launch_spmv; the list
  // starts at word 64
  GMLS_HIP(launch_spmv(n_rows, row_ptr, col, val, x, y, sp + 64, sp, ctx->cus, ctx->stream));
  return GMLS_OK;
}

gmls_status gmls_check(gmls_ctx ctx) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  DeviceGuard g(ctx->device);
  int *de = (int *)ctx->ws(WS_DEV_ERR, sizeof(int));
  if (!de) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device error word missing");
  int bits = 0;
  GMLS_HIP(hipMemcpyAsync(&bits, de, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  GMLS_HIP(hipStreamSynchronize(ctx->stream));
  if (!bits) return GMLS_OK;
  GMLS_HIP(fill_zero(de, sizeof(int), ctx->stream));
  GMLS_HIP(hipStreamSynchronize(ctx->stream));
  if (bits & DEV_ERR_CAPACITY)
    return gmls_set_error(ctx, GMLS_ERR_CAPACITY, "a neighbour search needed more than col_capacity entries");
  if (bits & DEV_ERR_RADIUS_ROWS)
    return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "a target had more than 2048 sources inside the radius");
  return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "a stencil call had a target with more than 2^24 neighbours");
}

gmls_status gmls_apply(gmls_ctx ctx, int64_t n_tgt, const int64_t *row_ptr, const int32_t *col,
                       const double *weights, int F, int C_in, const double *field, double *out) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  if (n_tgt < 0 || F < 1 || F > 16 || C_in < 1 || C_in > 3)
    return gmls_set_error(ctx, GMLS_ERR_ARG, "bad n_tgt, F or C_in");
  if (n_tgt > 0 && (!row_ptr || !col || !weights || !field || !out))
    return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer");
  DeviceGuard g(ctx->device);
  GMLS_HIP(launch_apply(n_tgt, row_ptr, col, weights, F, C_in, field, out, ctx->stream));
  return GMLS_OK;
}

// ---------------------------------------------------------------------------
// autotuner of the pipeline's row shapes
// ---------------------------------------------------------------------------
// Candidates of every tunable kernel, as reported in gmls_tune_result.
static void tune_candidates(gmls_tune_result *out) {
  memset(out, 0, sizeof(*out));
  for (int k = 0; k < GMLS_TUNE_KERNELS; ++k)
    for (int b = 0; b < kNumBins; ++b) {
      out->chosen[k][b] = -1;
      if (b == 0) continue;
      for (int c = 0; c < kPipeCands; ++c) {
        int lanes = 64, rows = b, wps = 0, round = 0, per_cu = 0;
        if (k < 2) {
          lanes = kPipeShapes[b][c].g;
          rows = kPipeShapes[b][c].rpl;
          wps = k == 0 ? 2 : 0;
          round = k == 0 ? 32 : 0;
        } else if (k == 2) {
          rows = b == kLongBin ? 0 : b;  // the long bin goes to the FP64 QR
          wps = kWaveCand[c].wpe;
          round = kWaveCand[c].rs;
        } else {
          rows = kQrShapes[b][c].rpl;
          per_cu = kQrShapes[b][c].per_cu;
          wps = kQrShapes[b][c].wpe;
        }
        out->lanes[k][b][c] = lanes;
        out->rows[k][b][c] = rows;
        out->waves_per_simd[k][b][c] = wps;
        out->lds_round[k][b][c] = round;
        out->waves_per_cu[k][b][c] = per_cu;
      }
    }
}

gmls_status gmls_autotune(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets, int64_t n_tgt,
                          int dim, int order, int basis, unsigned functional_mask, int weight_p, const double *eps,
                          const int64_t *row_ptr, const int32_t *col, int reps, double *weights,
                          uint8_t *target_status, gmls_tune_result *out) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  if (reps < 1 || reps > 100) return gmls_set_error(ctx, GMLS_ERR_ARG, "reps must be in 1..100");
  if (ctx->opt.capture_safe)
    return gmls_set_error(ctx, GMLS_ERR_ARG, "the autotuner times its runs: not available in capture-safe mode");
  const bool shared = basis == GMLS_TUNE_SHARED, stag = basis == GMLS_TUNE_STAGGERED;
  if (basis != GMLS_BASIS_SCALAR && basis != GMLS_BASIS_DIVFREE && !shared && !stag)
    return gmls_set_error(ctx, GMLS_ERR_ARG,
                          "basis must be GMLS_BASIS_SCALAR, GMLS_BASIS_DIVFREE, GMLS_TUNE_SHARED or GMLS_TUNE_STAGGERED");
  if (stag && (functional_mask == 0 || (functional_mask & ~(unsigned)(GMLS_F_GRAD | GMLS_F_LAPLACIAN))))
    return gmls_set_error(ctx, GMLS_ERR_ARG, "staggered tuning: GMLS_F_GRAD and/or GMLS_F_LAPLACIAN");
  if (stag && (order < 0 || order > 3))
    return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "staggered vector order must be 0..3");
  if (!qr_supported(dim, stag ? order + 1 : order, shared ? 1 : stag ? kBasisStaggered : basis))
    return gmls_set_error(ctx, GMLS_ERR_UNSUPPORTED, "compiled kernels cover dim 2-3 and order 1-4");
  // staggered: the target weights go to a workspace
  double *hw = nullptr;
  if (stag && n_tgt > 0) {
    const int F = (functional_mask & GMLS_F_GRAD ? dim : 0) + (functional_mask & GMLS_F_LAPLACIAN ? 1 : 0);
    hw = (double *)ctx->ws(WS_TUNE_AUX, sizeof(double) * (size_t)F * (size_t)n_tgt);
    if (!hw) return gmls_set_error(ctx, GMLS_ERR_NOMEM, "device workspace allocation failed");
  }
  // what each precision runs for this shape
  int mixed = -1;  // the mixed scheme, when it is a tuned one
  if (shared) {
    const int s0 = mixed_scheme(dim, order, 0, ctx->opt.scheme), s1 = mixed_scheme(dim, order, 1, ctx->opt.scheme);
    if (s0 == s1 && s0 == MIXED_WAVE) mixed = MIXED_WAVE;  // the shared pipeline runs each set's own shapes
  } else if (!stag) {  // a staggered call's pipeline is tuned as the scalar basis of order + 1
    const int sc = mixed_scheme(dim, order, basis, ctx->opt.scheme);
    if (sc == MIXED_PIPE || sc == MIXED_WAVE) mixed = sc;
  }
  gmls_stencil_set sets[2] = {};
  if (shared) {
    int Fs = 0, Fv = 0, Cv = 0;
    const unsigned ms = functional_mask & 15u, mv = (functional_mask >> 4) & 15u;
    if (gmls_stencil_shape(dim, order, GMLS_BASIS_SCALAR, ms, &Fs, nullptr, nullptr) != GMLS_OK ||
        gmls_stencil_shape(dim, order, GMLS_BASIS_DIVFREE, mv, &Fv, &Cv, nullptr) != GMLS_OK ||
        (functional_mask >> 8) != 0)
      return gmls_set_error(ctx, GMLS_ERR_ARG, "shared tuning: scalar mask in bits 0-3, divergence-free in 4-7");
    // the divergence-free set's weights follow the scalar set's F_s * nnz
    int64_t tot = 0;
    if (n_tgt > 0) {
      if (!row_ptr) return gmls_set_error(ctx, GMLS_ERR_ARG, "null device pointer");
      DeviceGuard g(ctx->device);
      if (hipMemcpyAsync(&tot, row_ptr + n_tgt, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
          hipStreamSynchronize(ctx->stream) != hipSuccess)
        return gmls_set_error(ctx, GMLS_ERR_HIP, "reading row_ptr[n_tgt]");
    }
    sets[0] = {GMLS_BASIS_SCALAR, ms, weights, target_status};
    sets[1] = {GMLS_BASIS_DIVFREE, mv, weights ? weights + (int64_t)Fs * tot : nullptr,
               target_status ? target_status + n_tgt : nullptr};
  }
  if (out) tune_candidates(out);
  DeviceGuard g(ctx->device);
  PipeTimer tm;
  hipError_t he = hipSuccess;
  for (int k = 0; k < 4 && he == hipSuccess; ++k)
    for (int b = 0; b < 8 && he == hipSuccess; ++b)
      for (int e = 0; e < 2 && he == hipSuccess; ++e) he = hipEventCreate(&tm.ev[k][b][e]);
  auto destroy = [&]() {
    for (int k = 0; k < 4; ++k)
      for (int b = 0; b < 8; ++b)
        for (int e = 0; e < 2; ++e)
          if (tm.ev[k][b][e]) hipEventDestroy(tm.ev[k][b][e]);
  };
  if (he != hipSuccess) {
    destroy();
    return gmls_set_error(ctx, GMLS_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(he));
  }
  const Options saved = ctx->opt;
  ctx->opt.pipe_chunk = 0;  // one launch per bin
  float best[4][8][kPipeCands];
  bool seen[4][8] = {};
  for (auto &x : best)
    for (auto &y : x)
      for (auto &z : y) z = INFINITY;
  // groups of kernels timed together: the pipeline's two (mixed), the
  // wavefront kernel (mixed), the QR kernel (FP64)
  struct Group {
    int k0, k1, prec;
  };
  Group groups[2];
  int ng = 0;
  if (mixed == MIXED_PIPE) groups[ng++] = {0, 1, GMLS_PREC_MIXED};
  if (mixed == MIXED_WAVE) groups[ng++] = {2, 2, GMLS_PREC_MIXED};
  groups[ng++] = {3, 3, GMLS_PREC_FP64};
  gmls_status st = GMLS_OK;
  for (int gi = 0; gi < ng && st == GMLS_OK; ++gi) {
    const Group &gr = groups[gi];
    for (int c = 0; c < kPipeCands && st == GMLS_OK; ++c) {
      ctx->opt.pipe_force = gr.k0 == 0 ? c : -1;
      ctx->opt.wave_force = gr.k0 == 2 ? c : -1;
      ctx->opt.qr_force = gr.k0 == 3 ? c : -1;
      for (int r = 0; r < reps && st == GMLS_OK; ++r) {
        memset(tm.used, 0, sizeof(tm.used));
        ctx->timer = &tm;
        if (shared)
          st = run_shared(ctx, coords, n_src, targets, n_tgt, dim, order, weight_p, eps, row_ptr, col, sets[0],
                          sets[1], gr.prec == GMLS_PREC_FP64 ? -1 : mixed, nullptr);
        else if (stag)
          st = run_stencils(ctx, coords, n_src, targets, n_tgt, dim, order + 1, kBasisStaggered, functional_mask,
                            weight_p, eps, row_ptr, col, nullptr, GMLS_PREC_FP64, weights, hw, target_status, nullptr);
        else
          st = run_stencils(ctx, coords, n_src, targets, n_tgt, dim, order, basis, functional_mask, weight_p, eps,
                            row_ptr, col, nullptr, gr.prec, weights, nullptr, target_status, nullptr);
        ctx->timer = nullptr;
        if (st == GMLS_WARN_TARGET_FLAGS) st = GMLS_OK;
        if (st != GMLS_OK) break;
        he = hipStreamSynchronize(ctx->stream);
        if (he != hipSuccess) {
          st = gmls_set_error(ctx, GMLS_ERR_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(he));
          break;
        }
        for (int k = gr.k0; k <= gr.k1; ++k)
          for (int b = 1; b < kNumBins; ++b) {
            if (!tm.used[k][b]) continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, tm.ev[k][b][0], tm.ev[k][b][1]) != hipSuccess) continue;
            best[k][b][c] = std::min(best[k][b][c], ms);
            seen[k][b] = true;
          }
      }
    }
  }
  ctx->opt = saved;
  destroy();
  if (st != GMLS_OK) return st;
  const int key = stag ? tune_key(dim, order + 1, kBasisStaggered) : tune_key(dim, order, shared ? kTuneShared : basis);
  auto ins = ctx->tune.emplace(key, std::array<signed char, 32>{});
  if (ins.second) ins.first->second.fill(-1);
  auto &ent = ins.first->second;
  for (int k = 0; k < 4; ++k)
    for (int b = 1; b < kNumBins; ++b) {
      if (!seen[k][b]) continue;
      int arg = 0;
      for (int c = 1; c < kPipeCands; ++c)
        if (best[k][b][c] < best[k][b][arg]) arg = c;
      ent[k * 8 + b] = (signed char)arg;
      if (out) {
        out->chosen[k][b] = arg;
        for (int c = 0; c < kPipeCands; ++c) out->ms[k][b][c] = isfinite(best[k][b][c]) ? best[k][b][c] : 0.f;
      }
    }
  return GMLS_OK;
}

static const char *kTuneKernel[4] = {"moments", "weights", "wave", "qr"};

gmls_status gmls_autotune_save(gmls_ctx ctx, const char *path) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  if (!path) return gmls_set_error(ctx, GMLS_ERR_ARG, "null path");
  FILE *f = fopen(path, "w");
  if (!f) return gmls_set_error(ctx, GMLS_ERR_ARG, std::string("cannot open ") + path + " for writing");
  fprintf(f, "{\"libgmls_autotune\": 1,\n \"entries\": [");
  bool first = true;
  for (const auto &kv : ctx->tune) {
    const int basis = kv.first % 4, order = (kv.first / 4) % 8, dim = kv.first / 32;
    for (int k = 0; k < 4; ++k)
      for (int b = 1; b < kNumBins; ++b) {
        const int c = kv.second[k * 8 + b];
        if (c < 0) continue;
        const int lanes = k < 2 ? kPipeShapes[b][c].g : 64;
        const int rows = k < 2 ? kPipeShapes[b][c].rpl : k == 2 ? b : kQrShapes[b][c].rpl;
        fprintf(f,
                "%s\n  {\"dim\": %d, \"order\": %d, \"basis\": %d, \"kernel\": \"%s\", \"bin\": %d, \"lanes\": %d, "
                "\"rows_per_lane\": %d",
                first ? "" : ",", dim, order, basis, kTuneKernel[k], b, lanes, rows);
        if (k == 2) fprintf(f, ", \"waves_per_simd\": %d, \"lds_round\": %d", kWaveCand[c].wpe, kWaveCand[c].rs);
        if (k == 3)
          fprintf(f, ", \"waves_per_simd\": %d, \"waves_per_cu\": %d", kQrShapes[b][c].wpe, kQrShapes[b][c].per_cu);
        fprintf(f, "}");
        first = false;
      }
  }
  fprintf(f, "\n ]}\n");
  const bool bad = ferror(f) != 0;
  if (fclose(f) != 0 || bad) return gmls_set_error(ctx, GMLS_ERR_ARG, std::string("write error on ") + path);
  return GMLS_OK;
}

gmls_status gmls_autotune_load(gmls_ctx ctx, const char *path) {
  if (!ctx) return GMLS_ERR_ARG;
  ctx->err.clear();
  if (!path) return gmls_set_error(ctx, GMLS_ERR_ARG, "null path");
  FILE *f = fopen(path, "r");
  if (!f) return gmls_set_error(ctx, GMLS_ERR_ARG, std::string("cannot open ") + path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0 && text.size() < (1u << 20)) text.append(buf, got);
  fclose(f);
  if (text.find("\"libgmls_autotune\": 1") == std::string::npos)
    return gmls_set_error(ctx, GMLS_ERR_ARG, "not a libgmls autotune file (version 1)");
  std::map<int, std::array<signed char, 32>> add;
  size_t pos = 0;
  const std::string tag = "{\"dim\":";
  while ((pos = text.find(tag, pos)) != std::string::npos) {
    int dim = 0, order = 0, basis = 0, bin = 0, lanes = 0, rows = 0, used = 0;
    char kernel[16] = {0};
    const char *at = text.c_str() + pos;
    const int n = sscanf(at,
                         "{\"dim\": %d, \"order\": %d, \"basis\": %d, \"kernel\": \"%15[a-z]\", \"bin\": %d, "
                         "\"lanes\": %d, \"rows_per_lane\": %d%n",
                         &dim, &order, &basis, kernel, &bin, &lanes, &rows, &used);
    if (n != 7 || used == 0) return gmls_set_error(ctx, GMLS_ERR_ARG, "malformed autotune entry");
    int k = -1;
    for (int q = 0; q < 4; ++q)
      if (strcmp(kernel, kTuneKernel[q]) == 0) k = q;
    int wps = 0, round = 0, per_cu = 0, more = 0;
    int m = -1;
    if (k == 2)
      m = sscanf(at + used, ", \"waves_per_simd\": %d, \"lds_round\": %d}%n", &wps, &round, &more) == 2 ? 0 : -1;
    else if (k == 3)
      m = sscanf(at + used, ", \"waves_per_simd\": %d, \"waves_per_cu\": %d}%n", &wps, &per_cu, &more) == 2 ? 0
                                                                                                         : -1;
    else if (k >= 0)
      m = sscanf(at + used, "}%n", &more) == 0 ? 0 : -1;
    if (k < 0 || m < 0 || more == 0) return gmls_set_error(ctx, GMLS_ERR_ARG, "malformed autotune entry");
    // the bases each kernel runs for: 0 scalar, 1 divergence-free, 2 staggered (QR), 3 shared
    const bool basis_ok = k < 2 ? basis <= 1 : k == 2 ? basis != 2 : true;
    if (dim < 2 || dim > 3 || order < 1 || order > 4 || basis < 0 || basis > 3 || !basis_ok || bin < 1 ||
        bin >= kNumBins || (k == 2 && bin == kLongBin))
      return gmls_set_error(ctx, GMLS_ERR_ARG, "autotune entry out of range");
    int cand = -1;
    for (int c = 0; c < kPipeCands; ++c) {
      if (k < 2 && kPipeShapes[bin][c].g == lanes && kPipeShapes[bin][c].rpl == rows) cand = c;
      if (k == 2 && lanes == 64 && rows == bin && kWaveCand[c].wpe == wps && kWaveCand[c].rs == round) cand = c;
      if (k == 3 && lanes == 64 && kQrShapes[bin][c].rpl == rows && kQrShapes[bin][c].per_cu == per_cu &&
          kQrShapes[bin][c].wpe == wps)
        cand = c;
    }
    if (cand < 0) return gmls_set_error(ctx, GMLS_ERR_ARG, "autotune entry names a shape that is not compiled");
    auto ins = add.emplace(tune_key(dim, order, basis), std::array<signed char, 32>{});
    if (ins.second) ins.first->second.fill(-1);
    ins.first->second[k * 8 + bin] = (signed char)cand;
    pos += (size_t)(used + more);
  }
  for (const auto &kv : add) {
    auto ins = ctx->tune.emplace(kv.first, kv.second);
    if (!ins.second)
      for (int q = 0; q < 32; ++q)
        if (kv.second[q] >= 0) ins.first->second[q] = kv.second[q];
  }
  return GMLS_OK;
}

}  // extern "C"
