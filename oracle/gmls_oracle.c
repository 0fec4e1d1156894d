/*
 * gmls_oracle.c -- plain, slow, FP64 CPU oracle for GMLS stencil generation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * What it computes (Ha, Kuberry, Trask, Ryan, "Parallel implementation of a
 * compatible high-order meshless method for the Stokes' equations"):
 *
 *  - neighbour sets: the particles strictly inside the support ball of radius
 *    eps around the target (Section 2.1, the definition of the kernel support),
 *    selected here either as the k nearest (ties broken by index) or as all
 *    points closer than a fixed radius, floored to the k_min nearest;
 *  - the kernel W(r) = (1 - r/eps)^p for r < eps, else 0 (Section 2.1, kernel
 *    equation; the outer power p is a parameter of every call);
 *  - the eps-scaled Taylor monomials p_a(x) = prod_i ((x_i - xT_i)/eps)^a_i/a_i!
 *    (Section 2.1, 1D and 3D basis equations), or a divergence-free vector
 *    basis psi_i = sum_{a,c} T[(a,c),i] p_a e_c (Section 2.2);
 *  - the stencil of a functional lambda: alpha = W P (P^T W P)^{-1} lambda
 *    (Section 2.1, equations for A, B and c; Section 2.5, derivative
 *    approximation: derivatives act on the basis at x_T only).
 *
 * Evaluation: M = diag(sqrt(w)) P is factorised by Householder QR
 * (Golub & Van Loan, Matrix Computations, Alg. 5.2.1), then
 * z = R^{-T} lambda and alpha = sqrt(w) .* (Q1 z).  This equals the formula
 * above because P^T W P = R^T R and sqrt(W) P = Q1 R.
 *
 * Everything is IEEE double; build with -ffp-contract=off so that squared
 * distances (dx*dx + dy*dy) + dz*dz are never fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_NOMEM 3

/* functional bits; output row order is value, gradient, Laplacian, divergence */
#define OR_F_VALUE 1u
#define OR_F_GRAD 2u
#define OR_F_LAP 4u
#define OR_F_DIV 8u

/* ------------------------------------------------------------------------- */
/* monomial enumeration: total degree <= m, graded, then descending in x     */
/* ------------------------------------------------------------------------- */

static int binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return (int)r;
}

int gmls_oracle_num_monomials(int dim, int degree) {
  if (dim < 1 || dim > 3 || degree < 0) return -1;
  return binom(degree + dim, dim);
}

/* exps is [count][dim] */
int gmls_oracle_monomials(int dim, int degree, int32_t *exps) {
  int q = 0;
  for (int deg = 0; deg <= degree; ++deg) {
    if (dim == 1) {
      exps[q++] = deg;
    } else if (dim == 2) {
      for (int a = deg; a >= 0; --a) {
        exps[2 * q] = a;
        exps[2 * q + 1] = deg - a;
        ++q;
      }
    } else {
      for (int a = deg; a >= 0; --a)
        for (int b = deg - a; b >= 0; --b) {
          exps[3 * q] = a;
          exps[3 * q + 1] = b;
          exps[3 * q + 2] = deg - a - b;
          ++q;
        }
    }
  }
  return q;
}

/* ------------------------------------------------------------------------- */
/* neighbour search                                                          */
/* ------------------------------------------------------------------------- */

typedef struct {
  double d2;
  int32_t j;
} cand_t;

static inline int cand_less(cand_t a, cand_t b) {
  return a.d2 < b.d2 || (a.d2 == b.d2 && a.j < b.j);
}

static int cand_cmp(const void *pa, const void *pb) {
  cand_t a = *(const cand_t *)pa, b = *(const cand_t *)pb;
  if (cand_less(a, b)) return -1;
  if (cand_less(b, a)) return 1;
  return 0;
}

static int index_cmp(const void *pa, const void *pb) {
  int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
  return a < b ? -1 : (a > b ? 1 : 0);
}

/* squared distance, source minus target, summed x then y then z */
static inline double dist2(const double *src, const double *tgt, int dim) {
  double dx = src[0] - tgt[0];
  double s = dx * dx;
  if (dim > 1) {
    double dy = src[1] - tgt[1];
    s = s + dy * dy;
  }
  if (dim > 2) {
    double dz = src[2] - tgt[2];
    s = s + dz * dz;
  }
  return s;
}

/* bounded max-heap keeping the k smallest candidates */
typedef struct {
  cand_t *a;
  int n, cap;
} heap_t;

static void heap_push(heap_t *h, cand_t c) {
  if (h->n < h->cap) {
    int i = h->n++;
    h->a[i] = c;
    while (i > 0) {
      int p = (i - 1) / 2;
      if (cand_less(h->a[p], h->a[i])) {
        cand_t t = h->a[p];
        h->a[p] = h->a[i];
        h->a[i] = t;
        i = p;
      } else
        break;
    }
  } else if (cand_less(c, h->a[0])) {
    h->a[0] = c;
    int i = 0;
    for (;;) {
      int l = 2 * i + 1, r = l + 1, m = i;
      if (l < h->n && cand_less(h->a[m], h->a[l])) m = l;
      if (r < h->n && cand_less(h->a[m], h->a[r])) m = r;
      if (m == i) break;
      cand_t t = h->a[m];
      h->a[m] = h->a[i];
      h->a[i] = t;
      i = m;
    }
  }
}

/* uniform bucket grid over the sources, cells numbered x fastest */
typedef struct {
  int dim;
  double lo[3], c;
  int64_t nc[3], ncell;
  int64_t *start; /* ncell + 1 */
  int32_t *pts;   /* source indices, by cell then ascending index */
} ogrid_t;

static void ogrid_free(ogrid_t *g) {
  free(g->start);
  free(g->pts);
  g->start = NULL;
  g->pts = NULL;
}

static inline int64_t cell_coord(const ogrid_t *g, double x, int i) {
  double f = floor((x - g->lo[i]) / g->c);
  if (f < 0) return 0;
  if (f > (double)(g->nc[i] - 1)) return g->nc[i] - 1;
  return (int64_t)f;
}

static int ogrid_build(ogrid_t *g, const double *src, int64_t n, int dim, double c) {
  double hi[3] = {0, 0, 0};
  g->dim = dim;
  for (int i = 0; i < dim; ++i) {
    g->lo[i] = src[i];
    hi[i] = src[i];
  }
  for (int64_t j = 1; j < n; ++j)
    for (int i = 0; i < dim; ++i) {
      double x = src[j * dim + i];
      if (x < g->lo[i]) g->lo[i] = x;
      if (x > hi[i]) hi[i] = x;
    }
  if (!(c > 0)) c = 1.0;
  for (;;) {
    g->ncell = 1;
    for (int i = 0; i < 3; ++i) g->nc[i] = 1;
    for (int i = 0; i < dim; ++i) {
      g->nc[i] = (int64_t)floor((hi[i] - g->lo[i]) / c) + 1;
      g->ncell *= g->nc[i];
    }
    if (g->ncell <= 8 * n + 64) break;
    c *= 1.25;
  }
  g->c = c;
  g->start = (int64_t *)calloc((size_t)g->ncell + 1, sizeof(int64_t));
  g->pts = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int64_t *key = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!g->start || !g->pts || !key) {
    free(key);
    ogrid_free(g);
    return OR_ERR_NOMEM;
  }
  for (int64_t j = 0; j < n; ++j) {
    int64_t id = 0, mul = 1;
    for (int i = 0; i < dim; ++i) {
      id += cell_coord(g, src[j * dim + i], i) * mul;
      mul *= g->nc[i];
    }
    key[j] = id;
    g->start[id + 1]++;
  }
  for (int64_t q = 0; q < g->ncell; ++q) g->start[q + 1] += g->start[q];
  int64_t *fill = (int64_t *)malloc((size_t)g->ncell * sizeof(int64_t));
  if (!fill) {
    free(key);
    ogrid_free(g);
    return OR_ERR_NOMEM;
  }
  memcpy(fill, g->start, (size_t)g->ncell * sizeof(int64_t));
  for (int64_t j = 0; j < n; ++j) g->pts[fill[key[j]]++] = (int32_t)j;
  free(fill);
  free(key);
  return OR_OK;
}

/* visit every source in the block of cells within Chebyshev radius r of the
 * target's cell; returns 1 if the block covers the whole grid.  *delta gets
 * the distance from the target to the nearest face of the block that has
 * cells beyond it (INFINITY if none). */
typedef void (*visit_fn)(void *ctx, int32_t j, double d2);

static int ogrid_visit_block(const ogrid_t *g, const double *src, const double *x, int64_t r,
                             visit_fn fn, void *ctx, double *delta) {
  int dim = g->dim;
  int64_t ct[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  int covers = 1;
  double dl = INFINITY;
  for (int i = 0; i < dim; ++i) {
    ct[i] = cell_coord(g, x[i], i);
    lo[i] = ct[i] - r;
    hi[i] = ct[i] + r;
    if (lo[i] > 0) {
      covers = 0;
      double d = x[i] - (g->lo[i] + (double)lo[i] * g->c);
      if (d < dl) dl = d;
    } else
      lo[i] = 0;
    if (hi[i] < g->nc[i] - 1) {
      covers = 0;
      double d = (g->lo[i] + (double)(hi[i] + 1) * g->c) - x[i];
      if (d < dl) dl = d;
    } else
      hi[i] = g->nc[i] - 1;
  }
  *delta = dl;
  int64_t z0 = dim > 2 ? lo[2] : 0, z1 = dim > 2 ? hi[2] : 0;
  int64_t y0 = dim > 1 ? lo[1] : 0, y1 = dim > 1 ? hi[1] : 0;
  for (int64_t cz = z0; cz <= z1; ++cz)
    for (int64_t cy = y0; cy <= y1; ++cy)
      for (int64_t cx = lo[0]; cx <= hi[0]; ++cx) {
        int64_t id = cx + g->nc[0] * (cy + g->nc[1] * cz);
        for (int64_t q = g->start[id]; q < g->start[id + 1]; ++q) {
          int32_t j = g->pts[q];
          fn(ctx, j, dist2(src + (int64_t)j * dim, x, dim));
        }
      }
  return covers;
}

static void visit_heap(void *ctx, int32_t j, double d2) {
  cand_t c = {d2, j};
  heap_push((heap_t *)ctx, c);
}

/* the k nearest of target x, sorted by (d2, index), into out[0..k) */
static void knn_one_grid(const ogrid_t *g, const double *src, int64_t n_src, const double *x, int k,
                         cand_t *buf, cand_t *out) {
  heap_t h = {buf, 0, k};
  for (int64_t r = 1;; ++r) {
    h.n = 0;
    double delta;
    int covers = ogrid_visit_block(g, src, x, r, visit_heap, &h, &delta);
    if (covers) break;
    if (h.n == k && h.a[0].d2 < delta * delta * (1.0 - 1e-9)) break;
  }
  (void)n_src;
  memcpy(out, h.a, (size_t)h.n * sizeof(cand_t));
  qsort(out, (size_t)h.n, sizeof(cand_t), cand_cmp);
}

static void knn_one_brute(const double *src, int64_t n_src, int dim, const double *x, int k,
                          cand_t *buf, cand_t *out) {
  heap_t h = {buf, 0, k};
  for (int64_t j = 0; j < n_src; ++j) {
    cand_t c = {dist2(src + j * dim, x, dim), (int32_t)j};
    heap_push(&h, c);
  }
  memcpy(out, h.a, (size_t)h.n * sizeof(cand_t));
  qsort(out, (size_t)h.n, sizeof(cand_t), cand_cmp);
}

static double knn_cell_size(const double *src, int64_t n, int dim, int k) {
  double lo[3], hi[3], ext_max = 0;
  for (int i = 0; i < dim; ++i) lo[i] = hi[i] = src[i];
  for (int64_t j = 1; j < n; ++j)
    for (int i = 0; i < dim; ++i) {
      double v = src[j * dim + i];
      if (v < lo[i]) lo[i] = v;
      if (v > hi[i]) hi[i] = v;
    }
  for (int i = 0; i < dim; ++i)
    if (hi[i] - lo[i] > ext_max) ext_max = hi[i] - lo[i];
  if (!(ext_max > 0)) return 1.0;
  double vol = 1.0;
  for (int i = 0; i < dim; ++i) {
    double e = hi[i] - lo[i];
    vol *= e > 1e-3 * ext_max ? e : 1e-3 * ext_max;
  }
  return pow(vol * (double)k / (double)n, 1.0 / dim);
}

static int nthreads_or_default(int nt) {
#ifdef _OPENMP
  return nt > 0 ? nt : omp_get_max_threads();
#else
  (void)nt;
  return 1;
#endif
}

/* k nearest neighbours of every target; col is [n_tgt][k] sorted by (d2, j),
 * eps[t] = eps_mult * (distance to the k-th neighbour).  use_grid = 0 for
 * brute force. */
int gmls_oracle_knn(const double *src, int64_t n_src, const double *tgt, int64_t n_tgt, int dim, int k,
                    double eps_mult, int use_grid, int32_t *col, double *eps, int nthreads) {
  if (dim < 1 || dim > 3 || k < 1 || k > n_src || n_tgt < 0) return OR_ERR_ARG;
  ogrid_t g;
  memset(&g, 0, sizeof g);
  if (use_grid) {
    int rc = ogrid_build(&g, src, n_src, dim, knn_cell_size(src, n_src, dim, k));
    if (rc) return rc;
  }
  int err = 0;
  int nt = nthreads_or_default(nthreads);
#pragma omp parallel num_threads(nt)
  {
    cand_t *buf = (cand_t *)malloc((size_t)k * sizeof(cand_t));
    cand_t *out = (cand_t *)malloc((size_t)k * sizeof(cand_t));
    if (!buf || !out) {
#pragma omp atomic write
      err = OR_ERR_NOMEM;
    } else {
#pragma omp for schedule(dynamic, 64)
      for (int64_t t = 0; t < n_tgt; ++t) {
        const double *x = tgt + t * dim;
        if (use_grid)
          knn_one_grid(&g, src, n_src, x, k, buf, out);
        else
          knn_one_brute(src, n_src, dim, x, k, buf, out);
        for (int q = 0; q < k; ++q) col[t * k + q] = out[q].j;
        eps[t] = eps_mult * sqrt(out[k - 1].d2);
      }
    }
    free(buf);
    free(out);
  }
  if (use_grid) ogrid_free(&g);
  return err;
}

/* fixed-radius search floored to k_min: the neighbours of t are every source
 * with d^2 < r0*r0 (eps = r0); if there are fewer than k_min, they are the
 * k_min nearest by (d2, j) and eps = (d_kmin + d_{kmin+1}) / 2.  A radius row
 * is a set; it is written in ascending source index.  Pass 1 (col == NULL)
 * writes counts[t]; pass 2 fills col[row_ptr[t] ...] and eps[t]. */
typedef struct {
  cand_t *a;
  int64_t n, cap;
  double r2;
  int overflow;
} list_t;

static void visit_list(void *ctx, int32_t j, double d2) {
  list_t *l = (list_t *)ctx;
  if (d2 < l->r2) {
    if (l->n < l->cap)
      l->a[l->n] = (cand_t){d2, j};
    else
      l->overflow = 1;
    l->n++;
  }
}

static int radius_impl(const double *src, int64_t n_src, const double *tgt, int64_t n_tgt, int dim,
                       double r0, int k_min, int use_grid, int64_t *counts, const int64_t *row_ptr,
                       int32_t *col, double *eps, int nthreads) {
  if (dim < 1 || dim > 3 || !(r0 > 0) || k_min < 0 || k_min + 1 > n_src || n_tgt < 0)
    return OR_ERR_ARG;
  ogrid_t g, gk;
  memset(&g, 0, sizeof g);
  memset(&gk, 0, sizeof gk);
  if (use_grid) {
    int rc = ogrid_build(&g, src, n_src, dim, r0);
    if (rc) return rc;
    if (k_min > 0) {
      rc = ogrid_build(&gk, src, n_src, dim, knn_cell_size(src, n_src, dim, k_min + 1));
      if (rc) {
        ogrid_free(&g);
        return rc;
      }
    }
  }
  const double r2 = r0 * r0;
  int err = 0;
  int nt = nthreads_or_default(nthreads);
#pragma omp parallel num_threads(nt)
  {
    int64_t cap = 1024;
    cand_t *lst = (cand_t *)malloc((size_t)cap * sizeof(cand_t));
    cand_t *buf = (cand_t *)malloc((size_t)(k_min + 1) * sizeof(cand_t));
    cand_t *out = (cand_t *)malloc((size_t)(k_min + 1) * sizeof(cand_t));
    if (!lst || !buf || !out) {
#pragma omp atomic write
      err = OR_ERR_NOMEM;
    } else {
#pragma omp for schedule(dynamic, 64)
      for (int64_t t = 0; t < n_tgt; ++t) {
        const double *x = tgt + t * dim;
        list_t l;
        if (!lst) continue;
        for (;;) {
          l = (list_t){lst, 0, cap, r2, 0};
          if (use_grid) {
            double delta;
            int64_t R = (int64_t)ceil(r0 / g.c);
            ogrid_visit_block(&g, src, x, R, visit_list, &l, &delta);
          } else {
            for (int64_t j = 0; j < n_src; ++j) visit_list(&l, (int32_t)j, dist2(src + j * dim, x, dim));
          }
          if (!l.overflow) break;
          cap = 2 * l.n;
          free(lst);
          lst = (cand_t *)malloc((size_t)cap * sizeof(cand_t));
          if (!lst) break;
        }
        if (!lst) {
#pragma omp atomic write
          err = OR_ERR_NOMEM;
          continue;
        }
        if (l.n >= k_min) {
          if (col) {
            for (int64_t q = 0; q < l.n; ++q) col[row_ptr[t] + q] = lst[q].j;
            qsort(col + row_ptr[t], (size_t)l.n, sizeof(int32_t), index_cmp);
            eps[t] = r0;
          } else
            counts[t] = l.n;
        } else {
          if (col) {
            if (use_grid)
              knn_one_grid(&gk, src, n_src, x, k_min + 1, buf, out);
            else
              knn_one_brute(src, n_src, dim, x, k_min + 1, buf, out);
            for (int q = 0; q < k_min; ++q) col[row_ptr[t] + q] = out[q].j;
            qsort(col + row_ptr[t], (size_t)k_min, sizeof(int32_t), index_cmp);
            eps[t] = 0.5 * (sqrt(out[k_min - 1].d2) + sqrt(out[k_min].d2));
          } else
            counts[t] = k_min;
        }
      }
    }
    free(lst);
    free(buf);
    free(out);
  }
  if (use_grid) {
    ogrid_free(&g);
    ogrid_free(&gk);
  }
  return err;
}

int gmls_oracle_radius_count(const double *src, int64_t n_src, const double *tgt, int64_t n_tgt, int dim,
                             double r0, int k_min, int use_grid, int64_t *counts, int nthreads) {
  return radius_impl(src, n_src, tgt, n_tgt, dim, r0, k_min, use_grid, counts, NULL, NULL, NULL, nthreads);
}

int gmls_oracle_radius_fill(const double *src, int64_t n_src, const double *tgt, int64_t n_tgt, int dim,
                            double r0, int k_min, int use_grid, const int64_t *row_ptr, int32_t *col,
                            double *eps, int nthreads) {
  if (!col || !row_ptr || !eps) return OR_ERR_ARG;
  return radius_impl(src, n_src, tgt, n_tgt, dim, r0, k_min, use_grid, NULL, row_ptr, col, eps, nthreads);
}

/* ------------------------------------------------------------------------- */
/* stencils                                                                  */
/* ------------------------------------------------------------------------- */

/* number of output functional rows for a basis (0 scalar, 1 vector) and mask;
 * -1 if a requested functional is not defined on that basis */
int gmls_oracle_num_rows(int dim, int basis, unsigned mask) {
  int f = 0;
  if (basis == 0) {
    if (mask & OR_F_DIV) return -1;
    if (mask & OR_F_VALUE) f += 1;
    if (mask & OR_F_GRAD) f += dim;
    if (mask & OR_F_LAP) f += 1;
  } else {
    if (mask & OR_F_GRAD) return -1;
    if (mask & OR_F_VALUE) f += dim;
    if (mask & OR_F_LAP) f += dim;
    if (mask & OR_F_DIV) f += 1;
  }
  return f;
}

/* D^beta of the scaled monomial p_alpha at the target: in the scaled variable
 * s = (x - xT)/eps every x-derivative brings a factor 1/eps, and the
 * beta-derivative of s^alpha/alpha! at s = 0 is 1 when alpha == beta, else 0
 * (Section 2.5). */
static double deriv_at_target(const int32_t *alpha, const int *beta, int dim, double eps) {
  int order = 0;
  for (int i = 0; i < dim; ++i) {
    if (alpha[i] != beta[i]) return 0.0;
    order += beta[i];
  }
  double v = 1.0;
  for (int q = 0; q < order; ++q) v /= eps;
  return v;
}

/* One term of a functional: coefficient * D^beta applied to component comp
 * (comp is ignored for the scalar basis). */
typedef struct {
  int beta[3];
  int comp;
  double coef;
} term_t;

/* the terms of every output row; returns the row count */
static int build_rows(int dim, int basis, unsigned mask, term_t rows[][3], int nterms[]) {
  int f = 0;
  memset(rows, 0, sizeof(term_t) * 16 * 3);
  if (basis == 0) {
    if (mask & OR_F_VALUE) {
      rows[f][0].coef = 1.0;
      nterms[f] = 1;
      f++;
    }
    if (mask & OR_F_GRAD)
      for (int i = 0; i < dim; ++i) {
        rows[f][0].beta[i] = 1;
        rows[f][0].coef = 1.0;
        nterms[f] = 1;
        f++;
      }
    if (mask & OR_F_LAP) {
      for (int i = 0; i < dim; ++i) {
        rows[f][i].beta[i] = 2;
        rows[f][i].coef = 1.0;
      }
      nterms[f] = dim;
      f++;
    }
  } else {
    if (mask & OR_F_VALUE)
      for (int c = 0; c < dim; ++c) {
        rows[f][0].comp = c;
        rows[f][0].coef = 1.0;
        nterms[f] = 1;
        f++;
      }
    if (mask & OR_F_LAP)
      for (int c = 0; c < dim; ++c) {
        for (int i = 0; i < dim; ++i) {
          rows[f][i].beta[i] = 2;
          rows[f][i].comp = c;
          rows[f][i].coef = 1.0;
        }
        nterms[f] = dim;
        f++;
      }
    if (mask & OR_F_DIV) {
      for (int c = 0; c < dim; ++c) {
        rows[f][c].beta[c] = 1;
        rows[f][c].comp = c;
        rows[f][c].coef = 1.0;
      }
      nterms[f] = dim;
      f++;
    }
  }
  return f;
}

static double monomial_value(const int32_t *alpha, const double *s, int dim) {
  double v = 1.0;
  for (int i = 0; i < dim; ++i) {
    double fact = 1.0;
    for (int e = 1; e <= alpha[i]; ++e) {
      v *= s[i];
      fact *= (double)e;
    }
    v /= fact;
  }
  return v;
}

/* Householder QR in place of the column-major m x n matrix A (m >= n):
 * R on and above the diagonal, reflector tails v (v_k = 1 implicit) below,
 * tau[k] the reflector scalars (Golub & Van Loan, Alg. 5.2.1). */
static void householder_qr(double *A, int m, int n, double *tau) {
  for (int k = 0; k < n; ++k) {
    double *a = A + (int64_t)k * m;
    double norm2 = 0.0;
    for (int i = k; i < m; ++i) norm2 += a[i] * a[i];
    double norm = sqrt(norm2);
    if (norm == 0.0) {
      tau[k] = 0.0;
      continue;
    }
    double alpha = a[k];
    double beta = alpha >= 0 ? -norm : norm;
    double v0 = alpha - beta;
    for (int i = k + 1; i < m; ++i) a[i] /= v0;
    tau[k] = (beta - alpha) / beta;
    a[k] = beta;
    for (int j = k + 1; j < n; ++j) {
      double *b = A + (int64_t)j * m;
      double s = b[k];
      for (int i = k + 1; i < m; ++i) s += a[i] * b[i];
      s *= tau[k];
      b[k] -= s;
      for (int i = k + 1; i < m; ++i) b[i] -= s * a[i];
    }
  }
}

/* u <- Q1 u, where Q1 = H_0 H_1 ... H_{n-1} */
static void apply_q(const double *A, int m, int n, const double *tau, double *u) {
  for (int k = n - 1; k >= 0; --k) {
    if (tau[k] == 0.0) continue;
    const double *a = A + (int64_t)k * m;
    double s = u[k];
    for (int i = k + 1; i < m; ++i) s += a[i] * u[i];
    s *= tau[k];
    u[k] -= s;
    for (int i = k + 1; i < m; ++i) u[i] -= s * a[i];
  }
}

/* Weights layout: target t owns F*C*row_ptr[t] ... ; inside it entry
 * (f*N + j)*C + c for functional row f, neighbour j, input component c.
 * basis 0: scalar Taylor basis of the given order (C = 1).
 * basis 1: vector basis psi_i = sum T[(a*dim + c)*Qd + i] p_a e_c (C = dim),
 *          with a running over the monomials of degree <= order in the order
 *          of gmls_oracle_monomials.
 * status[t]: 0 ok, 1 rank deficient (weights set to NaN).  */
int gmls_oracle_stencils(const double *src, const double *tgt, int64_t n_tgt, int dim, int order, int basis,
                         const double *T, int Qd, unsigned mask, int p, const double *eps,
                         const int64_t *row_ptr, const int32_t *col, double *weights, uint8_t *status,
                         int nthreads) {
  if (dim < 1 || dim > 3 || order < 0 || order > 8 || (basis != 0 && basis != 1) || p < 1) return OR_ERR_ARG;
  if (basis == 1 && (!T || Qd < 1)) return OR_ERR_ARG;
  int F = gmls_oracle_num_rows(dim, basis, mask);
  if (F <= 0) return OR_ERR_ARG;
  const int Qs = gmls_oracle_num_monomials(dim, order);
  const int C = basis == 0 ? 1 : dim;
  const int ncol = basis == 0 ? Qs : Qd;
  int32_t *ex = (int32_t *)malloc((size_t)Qs * dim * sizeof(int32_t));
  if (!ex) return OR_ERR_NOMEM;
  gmls_oracle_monomials(dim, order, ex);
  term_t rows[16][3];
  int nterms[16];
  build_rows(dim, basis, mask, rows, nterms);

  int64_t nmax = 0;
  for (int64_t t = 0; t < n_tgt; ++t) {
    int64_t n = row_ptr[t + 1] - row_ptr[t];
    if (n > nmax) nmax = n;
  }
  const int64_t mmax = nmax * C;
  int err = 0;
  int nt = nthreads_or_default(nthreads);
#pragma omp parallel num_threads(nt)
  {
    double *A = (double *)malloc((size_t)(mmax > 0 ? mmax : 1) * ncol * sizeof(double));
    double *u = (double *)malloc((size_t)(mmax > ncol ? mmax : ncol) * sizeof(double));
    double *sw = (double *)malloc((size_t)(nmax > 0 ? nmax : 1) * sizeof(double));
    double *pv = (double *)malloc((size_t)Qs * sizeof(double));
    double *lam = (double *)malloc((size_t)ncol * sizeof(double));
    double *tau = (double *)malloc((size_t)ncol * sizeof(double));
    if (!A || !u || !sw || !pv || !lam || !tau) {
#pragma omp atomic write
      err = OR_ERR_NOMEM;
    } else {
#pragma omp for schedule(dynamic, 16)
      for (int64_t t = 0; t < n_tgt; ++t) {
        const int64_t base = row_ptr[t];
        const int N = (int)(row_ptr[t + 1] - base);
        const int m = N * C;
        double *wout = weights + (int64_t)F * C * base;
        const double e = eps[t];
        const double *xt = tgt + t * dim;
        if (m < ncol) {
          for (int64_t q = 0; q < (int64_t)F * m; ++q) wout[q] = NAN;
          status[t] = 1;
          continue;
        }
        /* sample matrix M = sqrt(W) P, column-major m x ncol */
        for (int j = 0; j < N; ++j) {
          const double *xj = src + (int64_t)col[base + j] * dim;
          double s[3] = {0, 0, 0}, r2 = 0.0;
          for (int i = 0; i < dim; ++i) {
            s[i] = (xj[i] - xt[i]) / e;
            r2 += s[i] * s[i];
          }
          double r = sqrt(r2), w = 0.0;
          if (r < 1.0) {
            w = 1.0;
            for (int q = 0; q < p; ++q) w *= (1.0 - r);
          }
          sw[j] = sqrt(w);
          for (int a = 0; a < Qs; ++a) pv[a] = monomial_value(ex + a * dim, s, dim);
          if (basis == 0) {
            for (int a = 0; a < Qs; ++a) A[(int64_t)a * m + j] = sw[j] * pv[a];
          } else {
            for (int c = 0; c < dim; ++c)
              for (int i = 0; i < Qd; ++i) {
                double v = 0.0;
                for (int a = 0; a < Qs; ++a) v += T[((int64_t)a * dim + c) * Qd + i] * pv[a];
                A[(int64_t)i * m + (j * dim + c)] = sw[j] * v;
              }
          }
        }
        householder_qr(A, m, ncol, tau);
        double rmax = 0.0, rmin = INFINITY;
        for (int k = 0; k < ncol; ++k) {
          double d = fabs(A[(int64_t)k * m + k]);
          if (d > rmax) rmax = d;
          if (d < rmin) rmin = d;
        }
        if (!(rmin > 1e-12 * rmax)) {
          for (int64_t q = 0; q < (int64_t)F * m; ++q) wout[q] = NAN;
          status[t] = 1;
          continue;
        }
        status[t] = 0;
        for (int f = 0; f < F; ++f) {
          /* lambda_i = functional applied to basis function i at x_T */
          for (int i = 0; i < ncol; ++i) {
            double v = 0.0;
            for (int q = 0; q < nterms[f]; ++q) {
              const term_t *tm = &rows[f][q];
              if (basis == 0) {
                v += tm->coef * deriv_at_target(ex + i * dim, tm->beta, dim, e);
              } else {
                for (int a = 0; a < Qs; ++a) {
                  double tv = T[((int64_t)a * dim + tm->comp) * Qd + i];
                  if (tv != 0.0) v += tm->coef * tv * deriv_at_target(ex + a * dim, tm->beta, dim, e);
                }
              }
            }
            lam[i] = v;
          }
          /* z = R^{-T} lambda (forward substitution) */
          for (int k = 0; k < ncol; ++k) {
            double v = lam[k];
            for (int i = 0; i < k; ++i) v -= A[(int64_t)k * m + i] * u[i];
            u[k] = v / A[(int64_t)k * m + k];
          }
          for (int i = ncol; i < m; ++i) u[i] = 0.0;
          apply_q(A, m, ncol, tau, u);
          for (int j = 0; j < N; ++j)
            for (int c = 0; c < C; ++c) wout[((int64_t)f * N + j) * C + c] = sw[j] * u[j * C + c];
        }
      }
    }
    free(A);
    free(u);
    free(sw);
    free(pv);
    free(lam);
    free(tau);
  }
  free(ex);
  return err;
}
