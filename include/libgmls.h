/*
 * libgmls.h -- C ABI of the MI355X (gfx950) GMLS stencil generator.
 *
 * Generalized moving least squares (Ha, Kuberry, Trask, Ryan, "Parallel
 * implementation of a compatible high-order meshless method for the Stokes'
 * equations"): for every target x_T the library finds the neighbours inside
 * the kernel support (Section 2.1), builds the kernel-weighted polynomial
 * sample matrix of an eps-scaled Taylor basis (Section 2.1, basis equations)
 * or of a divergence-free vector basis (Section 2.2), solves the local
 * least-squares problem (Section 2.1, normal equations A c = B u) and applies
 * a target functional to the basis at x_T (Section 2.5) to give stencil
 * weights alpha with  D u(x_T) ~ sum_j alpha_j u(x_j)  (Section 3.2).
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers owned by the caller unless marked
 *    "host".  The library owns only the opaque context (its stream, a
 *    workspace that grows on demand, tuning options).
 *  - Work is enqueued on the context's HIP stream.  Calls return without
 *    waiting for the GPU except where a result must reach the host (marked
 *    "synchronises").
 *  - Arguments are validated before anything is enqueued; a failure returns
 *    GMLS_ERR_ARG and leaves outputs untouched.  HIP runtime failures return
 *    GMLS_ERR_HIP.  gmls_last_error() gives a message for the last non-OK
 *    status of that context.  No C++ exception crosses this boundary.
 *  - Floating point data are IEEE double; indices are int32 (source ids)
 *    and int64 (CSR offsets).
 *  - A context may be used by one host thread at a time.
 */
#ifndef LIBGMLS_H
#define LIBGMLS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmls_ctx_s *gmls_ctx;

typedef enum {
  GMLS_OK = 0,
  GMLS_ERR_ARG = 1,         /* invalid argument (nothing enqueued)              */
  GMLS_ERR_HIP = 2,         /* HIP runtime error                                */
  GMLS_ERR_NOMEM = 3,       /* device workspace allocation failed               */
  GMLS_ERR_CAPACITY = 4,    /* col_capacity too small; required size returned   */
  GMLS_ERR_UNSUPPORTED = 5, /* shape outside the compiled kernels' range        */
  GMLS_WARN_TARGET_FLAGS = 6 /* finished; some targets are rank deficient       */
} gmls_status;

/* basis of the local polynomial space */
enum {
  GMLS_BASIS_SCALAR = 0, /* eps-scaled Taylor monomials of total degree <= m (Section 2.1)      */
  GMLS_BASIS_DIVFREE = 1 /* divergence-free vector polynomials of degree <= m (Section 2.2)     */
};

/* functional bit mask; output rows appear in the order value, gradient,
 * Laplacian, divergence.  Scalar basis: value (1 row), gradient (dim rows),
 * Laplacian (1 row).  Divergence-free basis: value (dim rows, one per output
 * component), vector Laplacian (dim rows), divergence (1 row, identically
 * zero on this basis).  Gradient on the vector basis and divergence on the
 * scalar basis return GMLS_ERR_UNSUPPORTED. */
enum { GMLS_F_VALUE = 1, GMLS_F_GRAD = 2, GMLS_F_LAPLACIAN = 4, GMLS_F_DIV = 8 };

/* arithmetic of the local solve */
enum {
  GMLS_PREC_FP64 = 0, /* Householder QR of sqrt(W) P in FP64                                 */
  GMLS_PREC_MIXED = 1 /* normal equations of the moment Gram (GMLS_OPT_MIXED_SCHEME): FP32
                         Cholesky with FP64 residual refinement for small scalar bases, an
                         FP64 factorisation or inverse of the equilibrated moment Gram
                         otherwise; FP64 weights; FP64 QR fallback for ill-conditioned targets */
};

/* neighbour search rule */
enum {
  GMLS_SEARCH_KNN = 0,   /* the k nearest sources, ties broken by smaller index;
                            eps_T = eps_mult * (distance to the k-th)                       */
  GMLS_SEARCH_RADIUS = 1 /* every source with distance < radius (eps_T = radius); when fewer
                            than k_min, the k_min nearest with eps_T = (d_kmin + d_kmin+1)/2 */
};

/* per-target status codes written to target_status */
enum {
  GMLS_TARGET_OK = 0,
  GMLS_TARGET_RANK_DEFICIENT = 1, /* fewer rows than basis functions, or the QR rank test
                                     failed; weights are NaN                               */
  GMLS_TARGET_FALLBACK = 2,       /* mixed path handed the target to the FP64 QR path       */
  GMLS_TARGET_NOT_CONVERGED = 3   /* mixed refinement did not converge; FP64 QR result      */
};

typedef struct {
  int32_t mode;    /* GMLS_SEARCH_KNN or GMLS_SEARCH_RADIUS                  */
  int32_t k;       /* kNN: neighbour count (1 <= k <= n_src)                  */
  double eps_mult; /* kNN: eps_T = eps_mult * d_k (must be > 1 for d_k < eps)  */
  double radius;   /* radius mode: search radius (> 0)                         */
  int32_t k_min;   /* radius mode: floor on the neighbour count (<= n_src - 1) */
  int32_t reserved;
} gmls_search;

/* filled (host memory) when a non-NULL report is passed to a stencil call;
 * that call then synchronises the stream.  The target counts are those of
 * the statuses written (GMLS_TARGET_*); gmls_stencils_multi sums them over
 * its sets, counting (target, set) pairs. */
typedef struct {
  int64_t n_targets;       /* targets (times the number of sets of a multi call)           */
  int64_t n_ok;            /* targets with weights: n_targets - n_rank_deficient            */
  int64_t n_rank_deficient;/* status GMLS_TARGET_RANK_DEFICIENT                            */
  int64_t n_fallback;      /* status GMLS_TARGET_FALLBACK: the mixed path handed the target
                              to the FP64 QR path (condition or breakdown)                  */
  int64_t n_not_converged; /* status GMLS_TARGET_NOT_CONVERGED (also recomputed by QR)      */
  int32_t sweep_hist[16];  /* mixed: targets by number of refinement sweeps used            */
  double cond_max;         /* mixed: largest 1-norm condition number (estimate) of the
                              equilibrated Gram over the targets the mixed kernels factored */
  double t_bin_ms;         /* GPU time of the binning kernels                                */
  double t_stencil_ms;     /* GPU time of the stencil kernels (all bins)                     */
  double t_fallback_ms;    /* GPU time of the FP64 fallback kernel                           */
  double cond_min;         /* mixed: smallest of those condition numbers (0 when none)       */
  double cond_med;         /* mixed: their median, to within a factor 2^(1/32) (the centre of
                              a log2 histogram bin of width 2^(1/16)); 0 when none.  A multi
                              call reports the scalar Gram's (sets in turn: sets[0]'s)       */
  double t_search_ms;      /* GPU time of the context's last gmls_neighbors call that
                              synchronised (0 if none, or if it failed)                      */
} gmls_report;

/* Options for gmls_set_option. */
enum {
  GMLS_OPT_COND_THRESHOLD = 0, /* fallback when the Gram condition estimate exceeds it (1e6) */
  GMLS_OPT_MAX_SWEEPS = 1,     /* refinement sweeps before giving up (8)                      */
  GMLS_OPT_REFINE_TOL = 2,     /* stop when the predicted relative error after a correction,
                                  rho*|dy|/|y| with rho = 2 n cond 2^-24, is <= tol (1e-11)   */
  GMLS_OPT_FORCE_FALLBACK = 3, /* nonzero: every mixed target takes the FP64 fallback (0)      */
  GMLS_OPT_MIXED_SCHEME = 4,   /* organisation of the mixed path (0):
                                  0 = automatic: 3 where compiled, else 4;
                                  1 = one fused kernel per row-count bin, FP64 residual recomputed
                                      over the rows every sweep (corrected semi-normal equations);
                                  2 = one fused kernel per bin, FP64 weighted moments formed once
                                      and the residual taken against the FP64 moment Gram
                                      (3D order <= 3, 2D order <= 4);
                                  3 = three-kernel pipeline: FP64 moments to device memory, one
                                      thread per target for factorisation and refinement, then the
                                      weights (scalar basis with at most 20 functions: 3D order
                                      <= 3, 2D order <= 4; divergence-free basis whose scalar
                                      basis has at most 10: order <= 2);
                                  4 = one wavefront per target, fused: FP64 moments summed over
                                      the wavefront, the equilibrated moment Gram inverted in FP64
                                      by symmetric sweeps, then the weights (every compiled shape:
                                      scalar bases of up to 35 functions, divergence-free bases
                                      whose scalar basis has up to 35).
                                  A scheme not compiled for the shape makes gmls_stencils return
                                  GMLS_ERR_UNSUPPORTED.                                         */
  GMLS_OPT_PIPE_CHUNK = 5,     /* scheme 3: targets per pipeline chunk, 0 = all at once (0); the
                                  workspace holds (moments + F*Q) doubles per chunk target       */
  GMLS_OPT_RADIUS_SCRATCH_MB = 6, /* radius search: device scratch (MiB) allowed for the one-pass
                                  search, 1 KiB per target; above it (or at 0) the search
                                  counts and fills in two passes (8192)                          */
  GMLS_OPT_CAPTURE_SAFE = 7,   /* nonzero: no call waits for the device or allocates, so that a
                                  sequence of calls can be captured into a HIP graph on the
                                  context's stream and replayed (0).  In this mode:
                                  - workspaces are not grown: run each call once with the mode off
                                    (same sizes) first, else GMLS_ERR_NOMEM;
                                  - gmls_neighbors writes -1 to *nnz_host (the total is
                                    row_ptr[n_tgt] on the device); a total over col_capacity leaves
                                    col unwritten and is reported by gmls_check;
                                  - gmls_stencils takes no report (GMLS_ERR_ARG otherwise); a row
                                    longer than 2^24 leaves its target unwritten and is reported by
                                    gmls_check.                                                  */
  GMLS_OPT_ROW_ORDER = 8,      /* order of the entries of a radius row (a set) (0):
                                  0 = cell order: by (cell of the source in the search's uniform
                                      grid, source index); deterministic for given inputs, no sort;
                                  1 = ascending source index (a sort per row).                   */
  GMLS_OPT_PIPE_SHAPE = 9,     /* row shape of the pipeline's moment and weight kernels (-1):
                                  -1 = the autotuned choice (gmls_autotune) for the call's
                                       (dim, order, basis), kernel and row-count bin; candidate 0
                                       where nothing was tuned;
                                  0, 1, 2 = this candidate in every bin (gmls_tune_result lists
                                       the lanes per target and rows per lane of each).          */
  GMLS_OPT_SOURCE_STRIDE = 10, /* layout of `coords` in the stencil calls (gmls_stencils, _multi,
                                  _constrained, _staggered) (0): source j is at coords[j*stride ..
                                  j*stride + dim); 0 means stride = dim; otherwise an integer in
                                  [dim, 64].  Use 4 with the records of gmls_neighbors_sorted.
                                  The search calls always read [n][dim].                         */
  GMLS_OPT_WAVE_SHAPE = 11,    /* variant of the wavefront kernel (mixed scheme 4) (-1): -1 the
                                  autotuned choice per bin, else this candidate in every bin      */
  GMLS_OPT_QR_SHAPE = 12       /* shape of the FP64 QR kernel per bin (-1): -1 the autotuned
                                  choice, else this candidate in every bin (gmls_tune_result)    */
};

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL means the null stream).  *out receives the handle. */
gmls_status gmls_create(gmls_ctx *out, int device, void *hip_stream);

/* Release the context and its device workspace (synchronises its stream). */
void gmls_destroy(gmls_ctx ctx);

/* Message for the last non-OK status on this context ("" if none).  The
 * string stays valid until the next call on the context. */
const char *gmls_last_error(gmls_ctx ctx);

/* Set a tuning option (see GMLS_OPT_*). */
gmls_status gmls_set_option(gmls_ctx ctx, int option, double value);

/* Neighbour search (Section 2.1: the neighbours of x_T are the particles
 * within distance eps of it).
 *   coords   [n_src][dim] sources;  targets [n_tgt][dim]  (may alias coords)
 *   dim      1, 2 or 3
 *   spec     host pointer to the search rule
 *   row_ptr  out: int64 [n_tgt + 1] CSR offsets (row_ptr[0] = 0)
 *   col      out: int32 [col_capacity] source indices.  kNN rows are sorted by
 *            (squared distance, index).  Radius rows are sets; their order is
 *            set by GMLS_OPT_ROW_ORDER (cell order by default, or ascending
 *            index), the same for every call with the same inputs.  Squared
 *            distances are evaluated as (dx*dx + dy*dy) + dz*dz in IEEE double
 *            without fused multiply-add
 *   eps      out: [n_tgt] support radius of every target
 *   nnz_host host out: total neighbour count
 * kNN rows hold exactly k entries.  Radius rows hold between k_min and
 * 2048 entries (more returns GMLS_ERR_UNSUPPORTED).  If the total exceeds
 * col_capacity nothing is written to col, *nnz_host gets the size needed and
 * GMLS_ERR_CAPACITY is returned.  Synchronises (to return nnz). */
gmls_status gmls_neighbors(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                           int64_t n_tgt, int dim, const gmls_search *spec, int64_t *row_ptr, int32_t *col,
                           int64_t col_capacity, double *eps, int64_t *nnz_host);

/* gmls_neighbors, also handing out the search's cell-ordered copy of the
 * sources and every row as positions in that copy (Section 2.1: a target's
 * neighbours lie in the few cells around it, so in this copy a row is a few
 * runs of nearby records).  A stencil depends only on the coordinates of its
 * row entries, in row order, so gmls_stencils on (sources_sorted, col_sorted)
 * with GMLS_OPT_SOURCE_STRIDE = 4 gives the weights of (coords, col) bit for
 * bit, gathering each row from nearby memory instead of from the sources'
 * own order.
 *   sources_sorted  out: FP64 [n_src][4] records (x, y, z, source index): the
 *                   coordinates (0 beyond dim) and the index as a double, by
 *                   cell of the search's uniform grid, then by source index;
 *                   the same on every call with the same inputs
 *   col_sorted      out: int32 [col_capacity], must not alias col: entry j of
 *                   a row is the position of the record of source col[j]
 *                   (sources_sorted[4*col_sorted[j] + 3] == col[j])
 * Other arguments, errors and capacity rules as for gmls_neighbors; col and
 * col_sorted are both written, or (over capacity) neither.  The one-pass
 * radius search in cell order (GMLS_OPT_ROW_ORDER 0, scratch within
 * GMLS_OPT_RADIUS_SCRATCH_MB) writes the positions as it finds the rows;
 * the other paths translate the finished rows, one more pass over them. */
gmls_status gmls_neighbors_sorted(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                                  int64_t n_tgt, int dim, const gmls_search *spec, int64_t *row_ptr, int32_t *col,
                                  int64_t col_capacity, double *eps, int64_t *nnz_host, double *sources_sorted,
                                  int32_t *col_sorted);

/* Output shape (host only): number of functional rows F, input components
 * C_in (1 scalar, dim vector) and basis size Q for a basis/order/mask. */
gmls_status gmls_stencil_shape(int dim, int order, int basis, unsigned functional_mask, int *F, int *C_in,
                               int *Q);

/* Stencil weights (Section 2.1 normal equations and Section 2.5 functionals:
 * alpha = W P (P^T W P)^{-1} lambda, with W(r) = (1 - r/eps)^p for r < eps).
 *   coords, targets, dim  as for gmls_neighbors
 *   order     polynomial order m (scalar: 0..4 in 2D/3D; divergence-free: 1..4)
 *   basis     GMLS_BASIS_*; functional_mask GMLS_F_*
 *   weight_p  kernel power p (1..12)
 *   eps, row_ptr, col   support radii and CSR neighbour lists (any row order)
 *   prec      GMLS_PREC_FP64 or GMLS_PREC_MIXED
 *   weights   out: target t owns F*C_in*row_ptr[t] ... ; inside, the entry
 *             (f*N_t + j)*C_in + c is the weight of input component c of
 *             neighbour j (the j-th entry of the row) in functional row f
 *   target_status  out (nullable): uint8 [n_tgt], GMLS_TARGET_*
 *   report    host out (nullable): summary; a non-NULL report synchronises
 * Rows must satisfy 0 <= N_t <= 2^24 (N_t * C_in < Q gives a rank-deficient
 * target).  Rows of more than 256 neighbours are taken in chunks: the FP64
 * QR factors them by a tall-skinny QR (the factor of 64 RPL rows stacked
 * with the next rows), the mixed pipeline loops its moment and weight
 * kernels over them, and the other mixed schemes hand them to the FP64 QR
 * path (status GMLS_TARGET_FALLBACK).
 * Returns GMLS_WARN_TARGET_FLAGS when a report is requested and some targets
 * are rank deficient. */
gmls_status gmls_stencils(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                          int64_t n_tgt, int dim, int order, int basis, unsigned functional_mask, int weight_p,
                          const double *eps, const int64_t *row_ptr, const int32_t *col, int prec,
                          double *weights, uint8_t *target_status, gmls_report *report);

/* Staggered stencils (Section 2.4) for the pressure: grad p and Laplacian p
 * at x_T from a vector polynomial fit of grad p of order `order` (0..3),
 * sampled by integrals along the segments x_T -> x_j of the neighbour rows,
 * with data p_j - p(x_T).  The result is exact for p of degree <= order + 1.
 *   functional_mask  GMLS_F_GRAD and/or GMLS_F_LAPLACIAN (others: GMLS_ERR_ARG);
 *                    rows in the order gradient (dim rows), Laplacian
 *   weights          out: as for gmls_stencils with C_in = 1: the weight of
 *                    p_j (the j-th entry of the row) in functional row f
 *   target_weights   out: FP64 [n_tgt][F], the weight of p(x_T) in row f
 *                    (-sum_j of the row's weights); NaN for rank-deficient
 *                    targets.  A target listed among its own neighbours adds
 *                    its target weight to that entry, or is given p(x_T) apart
 *   prec             GMLS_PREC_FP64, or GMLS_PREC_MIXED where the degree-(order+1)
 *                    monomials number at most 20 (3D order <= 2, 2D order <= 3):
 *                    the mixed pipeline of gmls_stencils (FP64 moments, FP32
 *                    factor, FP64 refinement, FP64 QR fallback); otherwise
 *                    GMLS_ERR_UNSUPPORTED
 * Other arguments, statuses and errors as for gmls_stencils (the Gram has
 * (order+2 choose dim) - 1 columns: the circulating vector fields, which
 * integrate to zero on every segment from x_T, are not fitted). */
gmls_status gmls_stencils_staggered(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                                    int64_t n_tgt, int dim, int order, unsigned functional_mask, int weight_p,
                                    const double *eps, const int64_t *row_ptr, const int32_t *col, int prec,
                                    double *weights, double *target_weights, uint8_t *target_status,
                                    gmls_report *report);

/* Stencils of the Stokes system (Section 3.2) for n particles, every one
 * computed on the same neighbour rows (row_ptr, col) for every particle, in
 * the gmls_stencils layouts.  All pointers are device pointers. */
typedef struct {
  int64_t n;              /* particles */
  int32_t dim;            /* 2 or 3 */
  int32_t reserved;
  const int64_t *row_ptr; /* [n + 1] neighbour rows */
  const int32_t *col;     /* [row_ptr[n]] */
  const uint8_t *boundary;/* [n] nonzero for a boundary particle */
  const double *normals;  /* [n][dim] outward unit normals (read for boundary particles) */
  const double *vlap;     /* divergence-free vector Laplacian (gmls_stencils, GMLS_F_LAPLACIAN,
                             F = C_in = dim) */
  const double *grad;     /* scalar gradient (GMLS_F_GRAD, F = dim); interior rows */
  const double *plap;     /* staggered Laplacian (gmls_stencils_staggered, GMLS_F_LAPLACIAN);
                             interior rows */
  const double *plap_t;   /* its target weights [n] */
  const double *nlap;     /* Neumann-constrained Laplacian (gmls_stencils_constrained,
                             GMLS_F_LAPLACIAN); boundary rows */
  const double *nlap_h;   /* its h-weights [n] */
} gmls_stokes_stencils;

/* Global Stokes operator of Section 3.2 (the block system [K G 0; N L 1;
 * 0 1 0]) as one CSR matrix of R = dim*n + n + 1 rows.  Unknown and row
 * order: velocity v_(J,c) at J*dim + c, pressure phi_J at dim*n + J, the
 * zero-mean multiplier at dim*n + n.  Rows, nu the viscosity:
 *   interior velocity (I, c): -nu sum_j vlap v + sum_j grad phi      (K, G)
 *   boundary velocity (I, c): v_(I,c)                                 (K = identity)
 *   interior pressure I:      sum_j plap phi + plap_t[I] phi_I + lambda          (L)
 *   boundary pressure I:      nu nlap_h[I] sum_j n_I . vlap v + sum_j nlap phi + lambda
 *                                                                    (N, L)
 *   multiplier:               sum_J phi_J
 * so that the right-hand side is (f or the boundary velocity w; div f, or
 * div f - nlap_h[I] n_I . f on the boundary; 0).  Entries of a row follow
 * the neighbour order (velocity block, then pressure, then multiplier).
 *   a_row_ptr out: int64 [R + 1];  a_col out: int32 [capacity];
 *   a_val out: FP64 [capacity];    nnz_host out: entries needed
 * If they exceed capacity nothing is written to a_col/a_val and
 * GMLS_ERR_CAPACITY is returned.  Synchronises; not available in
 * capture-safe mode (GMLS_ERR_ARG). */
gmls_status gmls_assemble_stokes(gmls_ctx ctx, const gmls_stokes_stencils *stencils, double nu, int64_t *a_row_ptr,
                                 int32_t *a_col, double *a_val, int64_t capacity, int64_t *nnz_host);

/* y = A x for a CSR matrix of n_rows rows (device pointers; col int32, values
 * and vectors FP64).  Each row is summed in a fixed order, so y is the same on
 * every call.  Does not synchronise. */
gmls_status gmls_spmv(gmls_ctx ctx, int64_t n_rows, const int64_t *row_ptr, const int32_t *col, const double *val,
                      const double *x, double *y);

/* gmls_spmv without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  The same kernels and summation order as gmls_spmv, so
 * y is bit for bit the one gmls_spmv gives.  Its scratch (the list of rows
 * longer than 8192 entries) is a file-scope device array of the library of
 * 4 * (64 + 2^23) bytes (32 MiB), one per GPU, held until the process ends;
 * its address on a device is looked up when a context is created there.
 *   n_rows  0 .. 8388608 (2^23); more returns GMLS_ERR_ARG and enqueues nothing
 * Other arguments as for gmls_spmv.  Every call on one GPU uses that GPU's
 * scratch: calls that overlap in time on one GPU (different streams or
 * contexts) race and must not be made; calls in one stream order are safe.
 * Does not synchronise; no allocation, no memset (the counter is cleared by
 * a kernel). */
gmls_status gmls_spmv_noalloc(gmls_ctx ctx, int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                              const double *val, const double *x, double *y);

/* Errors of capture-safe calls found on the device since the last check
 * (GMLS_OPT_CAPTURE_SAFE): GMLS_OK, GMLS_ERR_CAPACITY or GMLS_ERR_UNSUPPORTED
 * with a message in gmls_last_error.  Synchronises; clears the record. */
gmls_status gmls_check(gmls_ctx ctx);

/* Neumann-constrained stencils (Section 2.3): for boundary targets the local
 * weighted least-squares fit is solved subject to n . grad u(x_T) = h(x_T),
 * with the outward normal n of target T, through the bordered system
 *   [P^T W P   F] [c]   [P^T W u]
 *   [F^T       0] [mu] = [h      ],   F = grad p(x_T)^T n.
 * A functional lambda of the constrained fit is then
 *   lambda^T c = sum_j alpha_j u_j + beta h(x_T),
 * the stencil alpha (layout as in gmls_stencils) plus one boundary weight
 * beta per target and functional row.
 *   normals   [n_tgt][dim] FP64 (need not be unit vectors: the constraint is
 *             on n . grad u; a zero vector leaves that target unconstrained,
 *             beta = 0)
 *   h_weights out: [n_tgt][F] FP64, beta of each functional row
 * Scalar basis only; prec must be GMLS_PREC_FP64 (else
 * GMLS_ERR_UNSUPPORTED).  Other arguments, statuses and errors as for
 * gmls_stencils; rank-deficient targets get NaN in both outputs. */
gmls_status gmls_stencils_constrained(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                                      int64_t n_tgt, int dim, int order, unsigned functional_mask, int weight_p,
                                      const double *eps, const int64_t *row_ptr, const int32_t *col,
                                      const double *normals, int prec, double *weights, double *h_weights,
                                      uint8_t *target_status, gmls_report *report);

/* Apply stencils to a field (Section 3.2, the stencil sum over neighbours):
 *   out[t*F + f] = sum_j sum_c weights[F*C_in*row_ptr[t] + (f*N_t + j)*C_in + c]
 *                               * field[col[row_ptr[t] + j]*C_in + c]
 * field [n_src][C_in], out [n_tgt][F]. */
gmls_status gmls_apply(gmls_ctx ctx, int64_t n_tgt, const int64_t *row_ptr, const int32_t *col,
                       const double *weights, int F, int C_in, const double *field, double *out);

/* Several stencil sets on the same neighbour lists and order: the scalar
 * Gram G = P^T W P of the weighted Taylor basis (Section 2.1) depends only on
 * the neighbours, eps and the weight, and the divergence-free fit of
 * Section 2.2 is the vector fit with Gram I (x) G under the constraint
 * D c = 0, so a scalar set and a divergence-free set can share it.  The
 * result of each set is that of gmls_stencils with the same arguments (bit
 * for bit where nothing is shared, within the precision's gate otherwise).
 * Shared, for exactly one scalar and one divergence-free set: with
 * prec = GMLS_PREC_FP64 one QR kernel takes the Householder factor R of a
 * target's weighted sample matrix once for both sets (G = R^T R; the weights
 * equal those of separate calls bit for bit); with prec = GMLS_PREC_MIXED and
 * the same scheme for both, the wavefront scheme (GMLS_OPT_MIXED_SCHEME 4,
 * automatic for order 4 in 3D), where one kernel forms the moments and the
 * swept Gram of a target once for both sets, or the pipeline (scheme 3,
 * automatic for order 2 in 3D), where the divergence-free set's solve takes
 * the scalar set's moments.  Other combinations run the sets in turn.
 *   sets, n_sets  host array of 1..8 sets: basis (GMLS_BASIS_SCALAR or
 *                 GMLS_BASIS_DIVFREE), functional_mask, weights (device,
 *                 F*C_in*nnz doubles, layout of gmls_stencils) and
 *                 target_status (device uint8[n_tgt], nullable)
 *   report        host, nullable: the times of the whole call and the counts
 *                 of one set (the scalar set where the Gram is shared, else
 *                 sets[0]); synchronises
 * Errors: those of gmls_stencils for any set; GMLS_ERR_ARG for n_sets outside
 * 1..8 or a null sets array. */
typedef struct {
  int32_t basis;
  uint32_t functional_mask;
  double *weights;
  uint8_t *target_status;
} gmls_stencil_set;

gmls_status gmls_stencils_multi(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets,
                                int64_t n_tgt, int dim, int order, int weight_p, const double *eps,
                                const int64_t *row_ptr, const int32_t *col, int prec, int n_sets,
                                const gmls_stencil_set *sets, gmls_report *report);

/* ---------------------------------------------------------------------------
 * Autotuner of the per-bin kernel shapes.  Targets are binned by row count
 * (bin b: 64(b-1) < N <= 64b neighbours; bin 5: N > 256), and each tunable
 * kernel is compiled in GMLS_TUNE_CANDIDATES shapes per bin, listed in
 * gmls_tune_result.  How fast a shape runs depends on the neighbour counts,
 * the cloud's order in memory and the functional count, so it is measured
 * rather than modelled.  The kernels (index k of the result):
 *   0 pipeline moments, 1 pipeline weights (mixed scheme 3): G lanes per
 *     target and R rows per lane, G*R >= 64b (bin 5: chunks of G*R rows);
 *   2 wavefront kernel (mixed scheme 4, one wavefront per target, b rows per
 *     lane): the occupancy it is compiled for (waves per SIMD; 1 lifts the
 *     register cap that 2 imposes) and the moments per LDS reduction round;
 *   3 FP64 Householder QR (one persistent wavefront per target): rows per lane
 *     R (a row of N > 64R is factored in chunks of 64R rows by the tall-skinny
 *     QR), persistent wavefronts per compute unit, and the occupancy it is
 *     compiled for (the compiler's choice, or two waves per SIMD).
 *
 * gmls_autotune runs the call's stencil computation `reps` times per
 * candidate (every bin in the same candidate) for each kernel the shape runs:
 * the mixed scheme's (0 and 1, or 2, where it resolves to scheme 3 or 4) in
 * GMLS_PREC_MIXED, and kernel 3 in GMLS_PREC_FP64.  It brackets every per-bin
 * launch with HIP events and keeps for each (kernel, bin) the candidate with
 * the smallest time (minimum over the repetitions) in the context's table,
 * keyed by (dim, order, basis); later calls with that key use it unless
 * GMLS_OPT_PIPE_SHAPE, GMLS_OPT_WAVE_SHAPE or GMLS_OPT_QR_SHAPE force a
 * candidate.  Bins without targets keep their previous entry.
 *   basis     GMLS_BASIS_SCALAR, GMLS_BASIS_DIVFREE, or GMLS_TUNE_SHARED: the
 *             kernels that gmls_stencils_multi runs for a scalar and a
 *             divergence-free set of one order on the same rows (kernels 2
 *             and 3; each set's pipeline is tuned under its own basis);
 *             functional_mask then holds the scalar set's mask in bits 0-3
 *             and the divergence-free set's in bits 4-7; or
 *             GMLS_TUNE_STAGGERED: the FP64 QR kernel of
 *             gmls_stencils_staggered (kernel 3 only; its mixed pipeline
 *             takes the shapes tuned for the scalar basis of order + 1), with
 *             `order` and functional_mask as that call takes them
 *   weights   F*C_in*nnz doubles (shared: the scalar set's F_s*nnz, then the
 *             divergence-free set's F_v*dim*nnz; staggered: F*nnz, the target
 *             weights go to a workspace); target_status uint8[n_tgt]
 *             (shared: 2*n_tgt), nullable: the last run's result
 * Other arguments are those of gmls_stencils.  Synchronises the context's
 * stream.  Errors: GMLS_ERR_ARG for reps outside 1..100, a bad basis or mask,
 * or capture-safe mode; GMLS_ERR_UNSUPPORTED when no kernel is compiled for
 * the shape; otherwise those of gmls_stencils.  `out` (host, nullable)
 * receives the candidates, their times and the choice.
 * -------------------------------------------------------------------------*/
enum {
  GMLS_TUNE_BINS = 6,
  GMLS_TUNE_CANDIDATES = 3,
  GMLS_TUNE_KERNELS = 4,
  GMLS_TUNE_STAGGERED = 2,
  GMLS_TUNE_SHARED = 3
};
typedef struct {
  /* [kernel][bin][candidate]; bin 0 unused */
  int32_t lanes[GMLS_TUNE_KERNELS][GMLS_TUNE_BINS][GMLS_TUNE_CANDIDATES];          /* per target         */
  int32_t rows[GMLS_TUNE_KERNELS][GMLS_TUNE_BINS][GMLS_TUNE_CANDIDATES];           /* rows per lane      */
  int32_t waves_per_simd[GMLS_TUNE_KERNELS][GMLS_TUNE_BINS][GMLS_TUNE_CANDIDATES]; /* compiled-for
                                                                                       occupancy (0: the
                                                                                       compiler's)      */
  int32_t lds_round[GMLS_TUNE_KERNELS][GMLS_TUNE_BINS][GMLS_TUNE_CANDIDATES];      /* moments per LDS
                                                                                       round (0: none)  */
  int32_t waves_per_cu[GMLS_TUNE_KERNELS][GMLS_TUNE_BINS][GMLS_TUNE_CANDIDATES];   /* persistent grid
                                                                                       (0: not
                                                                                       persistent)      */
  float ms[GMLS_TUNE_KERNELS][GMLS_TUNE_BINS][GMLS_TUNE_CANDIDATES]; /* best time per launch; 0 if not run */
  int32_t chosen[GMLS_TUNE_KERNELS][GMLS_TUNE_BINS];                  /* candidate kept; -1 if not run     */
} gmls_tune_result;

gmls_status gmls_autotune(gmls_ctx ctx, const double *coords, int64_t n_src, const double *targets, int64_t n_tgt,
                          int dim, int order, int basis, unsigned functional_mask, int weight_p, const double *eps,
                          const int64_t *row_ptr, const int32_t *col, int reps, double *weights,
                          uint8_t *target_status, gmls_tune_result *out);

/* The context's autotune table as a JSON file: {"libgmls_autotune": 1,
 * "entries": [...]}, one object per tuned (dim, order, basis, kernel, bin),
 * one per line, with the fields of the chosen shape in this order: "lanes"
 * and "rows_per_lane"; then for kernel "wave" "waves_per_simd" and
 * "lds_round", for kernel "qr" "waves_per_simd" (0: the compiler's choice)
 * and "waves_per_cu" (kernels "moments", "weights",
 * "wave", "qr"; basis 2 is the staggered QR, 3 the shared kernels).  Load merges the
 * entries it names into the table; a file not in this format, or naming a
 * shape that is not compiled, returns GMLS_ERR_ARG and changes nothing.
 * Host only (no device work).  GMLS_ERR_ARG also when the file cannot be
 * opened. */
gmls_status gmls_autotune_save(gmls_ctx ctx, const char *path);
gmls_status gmls_autotune_load(gmls_ctx ctx, const char *path);

#ifdef __cplusplus
}
#endif

#endif /* LIBGMLS_H */
