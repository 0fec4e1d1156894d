// stencil_mixed.hpp -- mixed-precision stencils: FP32 Gram + Cholesky, FP64
// corrected semi-normal-equation refinement and FP64 weights.
//
// The stencil of functional lambda is alpha = W P y with (P^T W P) y = lambda
// (Section 2.1, normal equations A = P^T W P; Section 2.5, functionals on the
// basis).  Work split per target (a group of G lanes; 64/G targets share a
// wavefront, each lane owns the rows j = lane_in_group + G*i):
//
//  1. rows: s_j = (x_j - x_T)/eps and w_j = (1 - |s_j|)^p in FP64, kept in LDS;
//  2. Gram: A_ab = sum_j w_j p_a(s_j) p_b(s_j) = mu_(a+b) / (a! b!) where
//     mu_g = sum_j w_j s_j^g are the weighted moments of degree <= 2m, so the
//     accumulation is one FP32 multiply-add per moment and row (84 moments in
//     3D at m = 3 instead of 210 Gram entries), then a group all-reduce;
//     for the divergence-free basis (Section 2.2) A_d = T^T (A (x) I_d) T
//     with the +-1 table T;
//  3. Jacobi equilibration A~ = D A D, D = diag(A)^-1/2, FP32 Cholesky
//     (Crout order, rows of L spread over the group, L in LDS); a pivot that
//     is not positive sends the target to the FP64 QR fallback;
//  4. explicit FP32 inverse A~^-1 = L^-T L^-1 (columns of L^-1 in parallel),
//     so that every solve below is one parallel matrix-vector product, and
//     the exact 1-norm condition number ||A~||_1 ||A~^-1||_1; above the
//     threshold the target goes to the fallback;
//  5. y0 = D A~^-1 D lambda in FP32;
//  6. refinement (FP64 residual, FP32 correction):
//        r = lambda - P^T W (P y)  evaluated over the rows in FP64,
//        y += D A~^-1 D r
//     until the predicted remaining error rho*|dy| <= tol*|y|, with
//     rho = 2 n cond u_32 the contraction factor of the FP32 inverse, at most
//     max_sweeps times (else fallback);
//  7. weights alpha_j = w_j p(s_j) . y accumulated in FP64.
#pragma once

#include <float.h>
#include <math.h>

#include "basis.hpp"
#include "divfree.hpp"
#include "gmls_internal.hpp"

namespace gmls {

// flat moment index (in Mono<DIM, 2m> order) of a + b for basis monomials a, b
template <int DIM, int ORDER>
struct SumIndex {
  static constexpr int Q = num_mono(DIM, ORDER);
  int idx[Q][Q];
  float inv_fact[Q];  // 1 / a!
  constexpr SumIndex() : idx{}, inv_fact{} {
    Mono<DIM, ORDER> M{};
    Mono<DIM, 2 * ORDER> M2{};
    for (int a = 0; a < Q; ++a) {
      double f = 1.0;
      for (int d = 0; d < 3; ++d)
        for (int k = 2; k <= M.e[a][d]; ++k) f *= k;
      inv_fact[a] = (float)(1.0 / f);
      for (int b = 0; b < Q; ++b)
        idx[a][b] = M2.index(M.e[a][0] + M.e[b][0], M.e[a][1] + M.e[b][1], M.e[a][2] + M.e[b][2]);
    }
  }
};

template <int DIM, int ORDER>
__constant__ SumIndex<DIM, ORDER> kSumIndex = SumIndex<DIM, ORDER>();

// Moments of degree <= 2m as (monomial of the first DIM-1 coordinates) x
// (power of the last coordinate); midx gives the flat index in Mono<DIM, 2m>.
template <int DIM, int ORDER>
struct MomentSplit {
  static constexpr int NP = num_mono(DIM - 1, 2 * ORDER);
  int parent[NP], pdim[NP], deg[NP];
  int midx[NP][2 * ORDER + 1];
  constexpr MomentSplit() : parent{}, pdim{}, deg{}, midx{} {
    Mono<DIM - 1, 2 * ORDER> MP{};
    Mono<DIM, 2 * ORDER> M2{};
    for (int pi = 0; pi < NP; ++pi) {
      parent[pi] = MP.parent[pi];
      pdim[pi] = MP.pdim[pi];
      deg[pi] = MP.e[pi][0] + MP.e[pi][1] + MP.e[pi][2];
      for (int c = 0; c <= 2 * ORDER; ++c) {
        int ex[3] = {0, 0, 0};
        for (int d = 0; d < DIM - 1; ++d) ex[d] = MP.e[pi][d];
        ex[DIM - 1] = c;
        midx[pi][c] = deg[pi] + c <= 2 * ORDER ? M2.index(ex[0], ex[1], ex[2]) : 0;
      }
    }
  }
};

template <int DIM, int ORDER, int BASIS, int G>
struct MixedCfg {
  static constexpr int Q = num_mono(DIM, ORDER);
  static constexpr int NM = num_mono(DIM, 2 * ORDER);
  static constexpr int QA = BASIS == 0 ? Q : DivFreeTab<DIM, ORDER>::QD;  // system size
  static constexpr int C = BASIS == 0 ? 1 : DIM;
  static constexpr int TPW = 64 / G;      // targets per wavefront
  static constexpr int RPL = 8;           // rows per lane
  static constexpr int NMAX = G * RPL;    // rows per target
  static constexpr int LDM = QA + 1;      // leading dimension of the LDS matrix
  static constexpr int RS = (QA + G - 1) / G;  // vector slots per lane
  static constexpr int FMAX = BASIS == 0 ? 5 : 7;     // value + gradient + Laplacian (+ divergence)
  static constexpr int NV = BASIS == 0 ? Q : DIM * Q;  // length of the refinement partials
  static constexpr int FU = BASIS == 0 ? 1 : FMAX;     // T y is only needed for the vector basis
};

template <int DIM, int ORDER, int BASIS, int G>
struct MixedLDS {
  using Cf = MixedCfg<DIM, ORDER, BASIS, G>;
  double rows[Cf::NMAX][DIM + 1];  // s, w of every row (FP64)
  double y[Cf::FMAX][Cf::QA];      // current solution, shared by the group
  double u[Cf::FU][Cf::NV];        // T y (vector basis)
  double pw[Cf::NV];               // reduced P^T W P y of one functional
  float mu[Cf::NM];
  float A[Cf::QA][Cf::LDM];        // equilibrated system; then L (lower) with L^-T (strict upper); then A~^-1
  float bv[Cf::QA];                // right-hand side of the current solve
  float dsc[Cf::QA];               // D
};

// ---------------------------------------------------------------------------
// group helpers
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ float gsum(float v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}
template <int G>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}
template <int G>
__device__ __forceinline__ float gmaxf(float v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, G));
  return v;
}
template <int G>
__device__ __forceinline__ double gmaxd(double v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, G));
  return v;
}

// u_f = T y_f for every functional row (vector basis); lane 0 of the group
template <int DIM, int ORDER, int G, int FY, int QAV, int FUV, int NVV>
__device__ __forceinline__ void divfree_apply_T(const double (&y)[FY][QAV], double (&u)[FUV][NVV], int F,
                                                int lg) {
  const DivFreeTab<DIM, ORDER> &T = kDivFree<DIM, ORDER>;
  for (int f = 0; f < F; ++f)
    for (int v = lg; v < NVV; v += G) u[f][v] = 0.0;
  __syncthreads();
  if (lg == 0)
    for (int f = 0; f < F; ++f)
      for (int i = 0; i < QAV; ++i) {
        u[f][T.ia[i] * DIM + T.ca[i]] += T.va[i] * y[f][i];
        if (T.ib[i] >= 0) u[f][T.ib[i] * DIM + T.cb[i]] += T.vb[i] * y[f][i];
      }
}

// lambda_f[i] of the system (scalar or divergence-free basis)
template <int DIM, int ORDER, int BASIS>
__device__ __forceinline__ double sys_lambda(int kind, int comp, int i, double ie) {
  if (BASIS == 0) {
    double v = 0.0;
    constexpr int Q = num_mono(DIM, ORDER);
#pragma unroll
    for (int a = 0; a < Q; ++a)
      if (a == i) v = scalar_lambda<DIM, ORDER>(kind, a, ie);
    return v;
  }
  return divfree_lambda<DIM, ORDER>(i, kind, comp, ie);
}

// ---------------------------------------------------------------------------
// one group of G lanes = one target
// ---------------------------------------------------------------------------
template <int DIM, int ORDER, int BASIS, int G>
__device__ void mixed_target(const StencilArgs &a, const RowKinds &rk, int t, bool valid, int lg,
                             MixedLDS<DIM, ORDER, BASIS, G> &S, int *fb_list, BinMeta *meta, Stats *stats,
                             const Options &opt) {
  using Cf = MixedCfg<DIM, ORDER, BASIS, G>;
  constexpr int Q = Cf::Q, NM = Cf::NM, QA = Cf::QA, RPL = Cf::RPL, RS = Cf::RS, C = Cf::C;
  const SumIndex<DIM, ORDER> &SI = kSumIndex<DIM, ORDER>;
  const int F = a.F;

  // ---- 1. rows ----
  int64_t base = 0;
  int N = 0;
  double e = 1.0;
  double xt[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xt[d] = 0.0;
  if (valid) {
    base = a.row_ptr[t];
    N = (int)(a.row_ptr[t + 1] - base);
    e = a.eps[t];
#pragma unroll
    for (int d = 0; d < DIM; ++d) xt[d] = a.targets[(int64_t)t * DIM + d];
  }
  const double ie = 1.0 / e;
  float mu[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) mu[m] = 0.f;
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int j = lg + G * r;
    double s[DIM], w = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) s[d] = 0.0;
    if (j < N) {
      const int c = a.col[base + j];
      double rr = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        s[d] = (a.coords[(int64_t)c * a.cstride + d] - xt[d]) * ie;
        rr += s[d] * s[d];
      }
      const double rad = sqrt(rr);
      w = rad < 1.0 ? int_pow(1.0 - rad, a.p) : 0.0;
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) S.rows[j][d] = s[d];
    S.rows[j][DIM] = w;
    // weighted moments w * s^g, |g| <= 2m (FP32): prefix monomials of the
    // first DIM-1 coordinates times powers of the last one
    constexpr MomentSplit<DIM, ORDER> MS{};
    float sf[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) sf[d] = (float)s[d];
    float lastp[2 * ORDER + 1];
    lastp[0] = 1.f;
#pragma unroll
    for (int c = 1; c <= 2 * ORDER; ++c) lastp[c] = lastp[c - 1] * sf[DIM - 1];
    float wp[MS.NP];
    wp[0] = (float)w;
#pragma unroll
    for (int pi = 1; pi < MS.NP; ++pi) wp[pi] = wp[MS.parent[pi]] * sf[MS.pdim[pi]];
#pragma unroll
    for (int pi = 0; pi < MS.NP; ++pi)
#pragma unroll
      for (int c = 0; c <= 2 * ORDER - MS.deg[pi]; ++c) mu[MS.midx[pi][c]] += wp[pi] * lastp[c];
  }
#pragma unroll
  for (int m = 0; m < NM; ++m) mu[m] = gsum<G>(mu[m]);
#pragma unroll
  for (int m = 0; m < NM; ++m)
    if (m % G == lg) S.mu[m] = mu[m];
  __syncthreads();

  // ---- 2./3. system matrix, equilibration ----
  if (BASIS == 0) {
    for (int i = lg; i < QA; i += G) S.dsc[i] = 1.0f / (sqrtf(S.mu[SI.idx[i][i]]) * SI.inv_fact[i]);
  } else {
    const DivFreeTab<DIM, ORDER> &T = kDivFree<DIM, ORDER>;
    for (int i = lg; i < QA; i += G) {
      float v = T.va[i] * T.va[i] * S.mu[SI.idx[T.ia[i]][T.ia[i]]] * SI.inv_fact[T.ia[i]] * SI.inv_fact[T.ia[i]];
      if (T.ib[i] >= 0) {
        v += T.vb[i] * T.vb[i] * S.mu[SI.idx[T.ib[i]][T.ib[i]]] * SI.inv_fact[T.ib[i]] * SI.inv_fact[T.ib[i]];
        if (T.ca[i] == T.cb[i])
          v += 2.f * T.va[i] * T.vb[i] * S.mu[SI.idx[T.ia[i]][T.ib[i]]] * SI.inv_fact[T.ia[i]] *
               SI.inv_fact[T.ib[i]];
      }
      S.dsc[i] = 1.0f / sqrtf(v);
    }
  }
  __syncthreads();
  for (int el = lg; el < QA * QA; el += G) {
    const int i = el / QA, k = el - (el / QA) * QA;
    if (k > i) continue;
    float v;
    if (BASIS == 0) {
      v = S.mu[SI.idx[i][k]] * SI.inv_fact[i] * SI.inv_fact[k];
    } else {
      const DivFreeTab<DIM, ORDER> &T = kDivFree<DIM, ORDER>;
      int ai[2] = {T.ia[i], T.ib[i]}, ci[2] = {T.ca[i], T.cb[i]};
      float vi[2] = {(float)T.va[i], (float)T.vb[i]};
      int ak[2] = {T.ia[k], T.ib[k]}, ck[2] = {T.ca[k], T.cb[k]};
      float vk[2] = {(float)T.va[k], (float)T.vb[k]};
      v = 0.f;
      for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q)
          if (ai[p] >= 0 && ak[q] >= 0 && ci[p] == ck[q])
            v += vi[p] * vk[q] * S.mu[SI.idx[ai[p]][ak[q]]] * SI.inv_fact[ai[p]] * SI.inv_fact[ak[q]];
    }
    S.A[i][k] = v * S.dsc[i] * S.dsc[k];
  }
  __syncthreads();
  // 1-norm of the equilibrated matrix (symmetric: column sums of the lower part)
  float cn = 0.f;
  for (int k = lg; k < QA; k += G) {
    float sum = 0.f;
    for (int i = 0; i < QA; ++i) sum += fabsf(i >= k ? S.A[i][k] : S.A[k][i]);
    cn = fmaxf(cn, sum);
  }
  const float anorm = gmaxf<G>(cn);

  // ---- 3. Cholesky (Crout): column k after columns < k ----
  bool ok = valid;
  for (int k = 0; k < QA; ++k) {
    float dk = S.A[k][k];
    for (int q = 0; q < k; ++q) dk -= S.A[k][q] * S.A[k][q];
    const bool pos = dk > 1e-12f;  // unit-diagonal matrix: tiny pivots mean near-singular
    ok = ok && pos;
    const float lkk = pos ? sqrtf(dk) : 1.0f;
    const float inv = 1.0f / lkk;
    for (int i = k + 1 + lg; i < QA; i += G) {
      float v = S.A[i][k];
      for (int q = 0; q < k; ++q) v -= S.A[i][q] * S.A[k][q];
      S.A[i][k] = v * inv;
    }
    __syncthreads();
    if (lg == 0) S.A[k][k] = lkk;
    __syncthreads();
  }

  // ---- 4. explicit inverse A~^-1 = L^-T L^-1: columns of L^-1 in parallel
  // (lane j solves L x = e_j), kept transposed in the strict upper triangle
  // (the diagonal of L^-1 is 1/L_jj); then the symmetric product, held in
  // registers until every lane is done reading L^-1.  Every later solve is
  // one parallel matrix-vector product. ----
  for (int j = lg; j < QA; j += G) {
    for (int i = j + 1; i < QA; ++i) {
      float v = -S.A[i][j] / S.A[j][j];  // k = j term, with L^-1_jj = 1/L_jj
      for (int k = j + 1; k < i; ++k) v -= S.A[i][k] * S.A[j][k];
      S.A[j][i] = v / S.A[i][i];
    }
  }
  __syncthreads();
  constexpr int NE = (QA * (QA + 1) / 2 + G - 1) / G;  // lower-triangle entries per lane
  float gi[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int el = lg + G * q;
    gi[q] = 0.f;
    if (el < QA * (QA + 1) / 2) {
      int i = 0;
      while ((i + 1) * (i + 2) / 2 <= el) ++i;
      const int k = el - i * (i + 1) / 2;  // k <= i
      // sum_{m >= i} L^-1[m][i] L^-1[m][k]; L^-1[m][c] = A[c][m] (m > c), 1/A[c][c] (m == c)
      float v = (1.0f / S.A[i][i]) * (i == k ? 1.0f / S.A[k][k] : S.A[k][i]);
      for (int m = i + 1; m < QA; ++m) v += S.A[i][m] * S.A[k][m];
      gi[q] = v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int el = lg + G * q;
    if (el < QA * (QA + 1) / 2) {
      int i = 0;
      while ((i + 1) * (i + 2) / 2 <= el) ++i;
      const int k = el - i * (i + 1) / 2;
      S.A[i][k] = gi[q];
      S.A[k][i] = gi[q];
    }
  }
  __syncthreads();
  // exact 1-norm condition number of the equilibrated system
  float inorm = 0.f;
  for (int k = lg; k < QA; k += G) {
    float sum = 0.f;
    for (int i = 0; i < QA; ++i) sum += fabsf(S.A[i][k]);
    inorm = fmaxf(inorm, sum);
  }
  const float cond = anorm * gmaxf<G>(inorm);
  if (!(cond <= opt.cond_threshold)) ok = false;
  if (opt.force_fallback) ok = false;
  // refinement contracts errors by about rho per sweep (FP32 inverse)
  const double rho = fmin(0.5, 2.0 * QA * (double)cond * 5.960464477539063e-08);

  // ---- 5. y0 = D A~^-1 D lambda ----
  for (int f = 0; f < F; ++f) {
    for (int i = lg; i < QA; i += G)
      S.bv[i] = (float)sys_lambda<DIM, ORDER, BASIS>(rk.kind[f], rk.comp[f], i, ie) * S.dsc[i];
    __syncthreads();
    for (int i = lg; i < QA; i += G) {
      float v = 0.f;
      for (int k = 0; k < QA; ++k) v += S.A[i][k] * S.bv[k];
      S.y[f][i] = (double)(v * S.dsc[i]);
    }
    __syncthreads();
  }

  // ---- 6. refinement: FP64 residual over the rows, FP32 correction ----
  int sweeps = 0;
  bool conv = false;
  for (int it = 0; it < opt.max_sweeps; ++it) {
    // wave-uniform loop: stop when every group of the wave has converged
    if (__ballot(ok && !conv) == 0) break;
    const bool active = ok && !conv;
    if constexpr (BASIS == 1) {
      divfree_apply_T<DIM, ORDER, G>(S.y, S.u, F, lg);
      __syncthreads();
    }
    double dmax = 0.0, ymax = 0.0;
    for (int f = 0; f < F; ++f) {
      // P^T W P y, component by component for the vector basis
      for (int c = 0; c < C; ++c) {
        double yr[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          if constexpr (BASIS == 0)
            yr[q] = S.y[f][q];
          else
            yr[q] = S.u[f][q * DIM + c];
        }
        double part[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) part[q] = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int j = lg + G * r;
          if (j < N) {
            double sv[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) sv[d] = S.rows[j][d];
            double p[Q];
            scaled_basis<DIM, ORDER, double>(sv, p);
            double u = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) u += p[q] * yr[q];
            const double tw = S.rows[j][DIM] * u;
#pragma unroll
            for (int q = 0; q < Q; ++q) part[q] += tw * p[q];
          }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) part[q] = gsum<G>(part[q]);
#pragma unroll
        for (int q = 0; q < Q; ++q)
          if (q % G == lg) S.pw[q * C + c] = part[q];
      }
      __syncthreads();
      // residual r = lambda - A y in system coordinates, scaled by D
      for (int i = lg; i < QA; i += G) {
        double ay;
        if constexpr (BASIS == 0) {
          ay = S.pw[i];
        } else {
          const DivFreeTab<DIM, ORDER> &T = kDivFree<DIM, ORDER>;
          ay = T.va[i] * S.pw[T.ia[i] * DIM + T.ca[i]];
          if (T.ib[i] >= 0) ay += T.vb[i] * S.pw[T.ib[i] * DIM + T.cb[i]];
        }
        const double ri = sys_lambda<DIM, ORDER, BASIS>(rk.kind[f], rk.comp[f], i, ie) - ay;
        S.bv[i] = (float)(ri * (double)S.dsc[i]);
      }
      __syncthreads();
      for (int i = lg; i < QA; i += G) {
        float v = 0.f;
        for (int k = 0; k < QA; ++k) v += S.A[i][k] * S.bv[k];
        if (active) {
          const double dy = (double)v * (double)S.dsc[i];
          const double yn = S.y[f][i] + dy;
          S.y[f][i] = yn;
          // a non-finite correction must never look converged
          dmax = (fabs(dy) <= dmax) ? dmax : (isfinite(dy) ? fabs(dy) : INFINITY);
          ymax = fmax(ymax, fabs(yn));
        }
      }
      __syncthreads();
    }
    dmax = gmaxd<G>(dmax);
    ymax = gmaxd<G>(ymax);
    if (active) {
      sweeps = it + 1;
      // predicted error after this correction: rho * |dy|
      if (rho * dmax <= opt.refine_tol * ymax) conv = true;
    }
  }
  const bool not_conv = ok && !conv;
  const bool good = ok && conv;

  // ---- 7. weights (FP64) ----
  if constexpr (BASIS == 1) {
    divfree_apply_T<DIM, ORDER, G>(S.y, S.u, F, lg);
    __syncthreads();
  }
  if (good) {
    double *wout = a.weights + (int64_t)F * C * base;
    for (int f = 0; f < F; ++f)
      for (int c = 0; c < C; ++c) {
        double yr[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          if constexpr (BASIS == 0)
            yr[q] = S.y[f][q];
          else
            yr[q] = S.u[f][q * DIM + c];
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int j = lg + G * r;
          if (j < N) {
            double sv[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) sv[d] = S.rows[j][d];
            double p[Q];
            scaled_basis<DIM, ORDER, double>(sv, p);
            double u = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) u += p[q] * yr[q];
            wout[((int64_t)f * N + j) * C + c] = S.rows[j][DIM] * u;
          }
        }
      }
  }
  if (valid && lg == 0) {
    if (a.cond_out) a.cond_out[t] = (float)cond;
    if (good) {
      a.status[t] = GMLS_TARGET_OK;
      atomicAdd(&stats->sweep_hist[sweeps < 15 ? sweeps : 15], 1ull);
    } else {
      a.status[t] = not_conv ? GMLS_TARGET_NOT_CONVERGED : GMLS_TARGET_FALLBACK;
      const int slot = atomicAdd(&meta->fb_count, 1);
      fb_list[slot] = t;
      atomicAdd(not_conv ? &stats->n_not_converged : &stats->n_fallback, 1ull);
    }
    const double cd = (double)cond;
    if (cd >= 0.0) atomicMax(&stats->cond_max_bits, (unsigned long long)__double_as_longlong(cd));
  }
  __syncthreads();
}

// Persistent kernel: each wavefront takes TPW consecutive targets of its bin.
template <int DIM, int ORDER, int BASIS, int G>
__global__ __launch_bounds__(64) void k_mixed(StencilArgs a, const int *list, const int *count, const int *offset,
                                              int *cursor, int *fb_list, BinMeta *meta, Stats *stats, Options opt) {
  using Cf = MixedCfg<DIM, ORDER, BASIS, G>;
  __shared__ MixedLDS<DIM, ORDER, BASIS, G> S[Cf::TPW];
  const RowKinds rk = row_kinds(DIM, BASIS, a.mask);
  const int n = readfirstlane_i(*count);
  const int off = readfirstlane_i(*offset);
  const int lane = lane_id();
  const int grp = lane / G, lg = lane % G;
  for (;;) {
    int i0 = 0;
    if (lane == 0) i0 = atomicAdd(cursor, Cf::TPW);
    i0 = readfirstlane_i(i0);
    if (i0 >= n) break;
    const int i = i0 + grp;
    const bool valid = i < n;
    const int t = valid ? list[off + i] : 0;
    mixed_target<DIM, ORDER, BASIS, G>(a, rk, t, valid, lg, S[grp], fb_list, meta, stats, opt);
  }
}

}  // namespace gmls
