// stencil_mixed64.hpp -- mixed-precision stencils with an FP64 moment Gram as
// the refinement operator ("gram64" variant).
//
// Same problem as stencil_mixed.hpp: alpha = W P y with (P^T W P) y = lambda
// (Section 2.1 normal equations, Section 2.5 functionals), one group of G
// lanes per target.  Differences:
//  1. the weighted moments mu_g = sum_j w_j s_j^g (|g| <= 2m) are accumulated
//     in FP64 in the single pass over the rows and reduce-scattered over the
//     group into LDS; A64_ab = mu_(a+b)/(a! b!) is then the exact (to FP64
//     rounding) Gram, and the FP32 equilibrated Gram used for the Cholesky
//     factor and the explicit inverse is rounded from it;
//  2. the refinement residual r = lambda - A64 y is a Q x Q product on the
//     moments instead of a pass over the rows (mixed-precision iterative
//     refinement: FP32 inverse, FP64 residual), so the rows are read twice in
//     total: once for the moments and once for the FP64 weights;
//  3. on gfx950 with packed FP32 disabled an FP64 FMA issues at the FP32 FMA
//     rate, so accumulating the moments in FP64 costs registers, not time.
// The converged solution is the FP64 normal-equations solution; its error is
// about cond(A) * 2^-53, below 1e-10 for every target that passes the
// condition threshold (1e6 by default); others take the FP64 QR fallback.
#pragma once

#include "stencil_mixed.hpp"

namespace gmls {

// moments that fit in registers as FP64 accumulators (3D m <= 3, 2D m <= 4)
template <int DIM, int ORDER>
constexpr bool has_gram64() {
  return num_mono(DIM, 2 * ORDER) <= 96;
}

template <int DIM, int ORDER>
struct InvFact64 {
  static constexpr int Q = num_mono(DIM, ORDER);
  double v[Q];
  constexpr InvFact64() : v{} {
    Mono<DIM, ORDER> M{};
    for (int a = 0; a < Q; ++a) {
      double f = 1.0;
      for (int d = 0; d < 3; ++d)
        for (int k = 2; k <= M.e[a][d]; ++k) f *= k;
      v[a] = 1.0 / f;
    }
  }
};

template <int DIM, int ORDER>
__constant__ InvFact64<DIM, ORDER> kInvFact64 = InvFact64<DIM, ORDER>();

template <int DIM, int ORDER, int BASIS, int G>
struct Mixed64Cfg : MixedCfg<DIM, ORDER, BASIS, G> {
  using Base = MixedCfg<DIM, ORDER, BASIS, G>;
  static constexpr int NMP = ((Base::NM + G - 1) / G) * G;  // moments padded to the group size
};

template <int DIM, int ORDER, int BASIS, int G>
struct Mixed64LDS {
  using Cf = Mixed64Cfg<DIM, ORDER, BASIS, G>;
  double mu[Cf::NMP];               // FP64 weighted moments
  double y[Cf::FMAX][Cf::QA];       // current solution
  double u[Cf::FU][Cf::NV];         // T y (vector basis)
  double v[Cf::NV];                 // (A64 (x) I) T y (vector basis)
  float A[Cf::QA][Cf::LDM];         // equilibrated FP32 system -> L, L^-T -> inverse
  float bv[Cf::QA];
  float dsc[Cf::QA];
};

// Reduce-scatter over the G lanes of a group: on return lane lg holds, in
// v[0 .. NMP/G), the group sums of entries [lg*NMP/G, (lg+1)*NMP/G).
template <int G, int NMP, int M, int HALF>
__device__ __forceinline__ void reduce_scatter_step(double (&v)[NMP], int lg) {
  if constexpr (M >= 1) {
    const bool hi = (lg & M) != 0;
#pragma unroll
    for (int i = 0; i < HALF; ++i) {
      const double keep = hi ? v[i + HALF] : v[i];
      const double send = hi ? v[i] : v[i + HALF];
      v[i] = keep + __shfl_xor(send, M, G);
    }
    reduce_scatter_step<G, NMP, M / 2, HALF / 2>(v, lg);
  }
}

template <int G, int NMP>
__device__ __forceinline__ void group_reduce_scatter(double (&v)[NMP], int lg) {
  reduce_scatter_step<G, NMP, G / 2, NMP / 2>(v, lg);
}

template <int DIM>
__device__ __forceinline__ void load_row(const StencilArgs &a, int64_t base, int j, const double *xt, double ie,
                                         double *s, double &w) {
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

// FP64 Gram entry A64[a][b] of the scalar basis from the moments in LDS
template <int DIM, int ORDER>
__device__ __forceinline__ double gram64(const double *mu, int a, int b) {
  const SumIndex<DIM, ORDER> &SI = kSumIndex<DIM, ORDER>;
  const InvFact64<DIM, ORDER> &IF = kInvFact64<DIM, ORDER>;
  return mu[SI.idx[a][b]] * IF.v[a] * IF.v[b];
}

// system matrix entry (scalar basis, or T^T (A64 (x) I) T for the vector basis)
template <int DIM, int ORDER, int BASIS>
__device__ __forceinline__ double sys64(const double *mu, int i, int k) {
  if constexpr (BASIS == 0) {
    return gram64<DIM, ORDER>(mu, i, k);
  } else {
    const DivFreeTab<DIM, ORDER> &T = kDivFree<DIM, ORDER>;
    int ai[2] = {T.ia[i], T.ib[i]}, ci[2] = {T.ca[i], T.cb[i]};
    double vi[2] = {T.va[i], T.vb[i]};
    int ak[2] = {T.ia[k], T.ib[k]}, ck[2] = {T.ca[k], T.cb[k]};
    double vk[2] = {T.va[k], T.vb[k]};
    double v = 0.0;
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 2; ++q)
        if (ai[p] >= 0 && ak[q] >= 0 && ci[p] == ck[q]) v += vi[p] * vk[q] * gram64<DIM, ORDER>(mu, ai[p], ak[q]);
    return v;
  }
}

template <int DIM, int ORDER, int BASIS, int G>
__device__ void mixed64_target(const StencilArgs &a, const RowKinds &rk, int t, bool valid, int lg,
                               Mixed64LDS<DIM, ORDER, BASIS, G> &S, int *fb_list, BinMeta *meta, Stats *stats,
                               const Options &opt) {
  using Cf = Mixed64Cfg<DIM, ORDER, BASIS, G>;
  constexpr int Q = Cf::Q, QA = Cf::QA, RPL = Cf::RPL, C = Cf::C, NM = Cf::NM, NMP = Cf::NMP;
  const int F = a.F;

  // ---- 1. rows -> FP64 weighted moments ----
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
  double mu[NMP];
#pragma unroll
  for (int m = 0; m < NMP; ++m) mu[m] = 0.0;
  constexpr MomentSplit<DIM, ORDER> MS{};
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int j = lg + G * r;
    if (j < N) {
      double s[DIM], w;
      load_row<DIM>(a, base, j, xt, ie, s, w);
      double lastp[2 * ORDER + 1];
      lastp[0] = 1.0;
#pragma unroll
      for (int c = 1; c <= 2 * ORDER; ++c) lastp[c] = lastp[c - 1] * s[DIM - 1];
      double wp[MS.NP];
      wp[0] = w;
#pragma unroll
      for (int pi = 1; pi < MS.NP; ++pi) wp[pi] = wp[MS.parent[pi]] * s[MS.pdim[pi]];
#pragma unroll
      for (int pi = 0; pi < MS.NP; ++pi)
#pragma unroll
        for (int c = 0; c <= 2 * ORDER - MS.deg[pi]; ++c) mu[MS.midx[pi][c]] += wp[pi] * lastp[c];
    }
  }
  group_reduce_scatter<G, NMP>(mu, lg);
#pragma unroll
  for (int i = 0; i < NMP / G; ++i) S.mu[lg * (NMP / G) + i] = mu[i];
  __syncthreads();
  (void)NM;

  // ---- 2. equilibrated FP32 system from the FP64 Gram ----
  for (int i = lg; i < QA; i += G) S.dsc[i] = (float)(1.0 / sqrt(sys64<DIM, ORDER, BASIS>(S.mu, i, i)));
  __syncthreads();
  for (int el = lg; el < QA * QA; el += G) {
    const int i = el / QA, k = el - (el / QA) * QA;
    if (k > i) continue;
    S.A[i][k] = (float)(sys64<DIM, ORDER, BASIS>(S.mu, i, k) * (double)S.dsc[i] * (double)S.dsc[k]);
  }
  __syncthreads();
  float cn = 0.f;
  for (int k = lg; k < QA; k += G) {
    float sum = 0.f;
    for (int i = 0; i < QA; ++i) sum += fabsf(i >= k ? S.A[i][k] : S.A[k][i]);
    cn = fmaxf(cn, sum);
  }
  const float anorm = gmaxf<G>(cn);

  // ---- 3. FP32 Cholesky (Crout) ----
  bool ok = valid;
  for (int k = 0; k < QA; ++k) {
    float dk = S.A[k][k];
    for (int q = 0; q < k; ++q) dk -= S.A[k][q] * S.A[k][q];
    const bool pos = dk > 1e-12f;
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

  // ---- 4. explicit FP32 inverse (see stencil_mixed.hpp) ----
  for (int j = lg; j < QA; j += G) {
    for (int i = j + 1; i < QA; ++i) {
      float v = -S.A[i][j] / S.A[j][j];
      for (int k = j + 1; k < i; ++k) v -= S.A[i][k] * S.A[j][k];
      S.A[j][i] = v / S.A[i][i];
    }
  }
  __syncthreads();
  constexpr int NE = (QA * (QA + 1) / 2 + G - 1) / G;
  float gi[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int el = lg + G * q;
    gi[q] = 0.f;
    if (el < QA * (QA + 1) / 2) {
      int i = 0;
      while ((i + 1) * (i + 2) / 2 <= el) ++i;
      const int k = el - i * (i + 1) / 2;
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
  float inorm = 0.f;
  for (int k = lg; k < QA; k += G) {
    float sum = 0.f;
    for (int i = 0; i < QA; ++i) sum += fabsf(S.A[i][k]);
    inorm = fmaxf(inorm, sum);
  }
  const float cond = anorm * gmaxf<G>(inorm);
  if (!(cond <= opt.cond_threshold)) ok = false;
  if (opt.force_fallback) ok = false;
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

  // ---- 6. refinement: r = lambda - A64 y (FP64), y += D A~^-1 D r ----
  int sweeps = 0;
  bool conv = false;
  for (int it = 0; it < opt.max_sweeps; ++it) {
    if (__ballot(ok && !conv) == 0) break;
    const bool active = ok && !conv;
    if constexpr (BASIS == 1) {
      divfree_apply_T<DIM, ORDER, G>(S.y, S.u, F, lg);
      __syncthreads();
    }
    double dmax = 0.0, ymax = 0.0;
    for (int f = 0; f < F; ++f) {
      if constexpr (BASIS == 1) {
        // v = (A64 (x) I) u
        for (int el = lg; el < Cf::NV; el += G) {
          const int al = el / DIM, c = el - (el / DIM) * DIM;
          double acc = 0.0;
          for (int b = 0; b < Q; ++b) acc += gram64<DIM, ORDER>(S.mu, al, b) * S.u[f][b * DIM + c];
          S.v[el] = acc;
        }
        __syncthreads();
      }
      for (int i = lg; i < QA; i += G) {
        double ay = 0.0;
        if constexpr (BASIS == 0) {
          for (int k = 0; k < QA; ++k) ay += gram64<DIM, ORDER>(S.mu, i, k) * S.y[f][k];
        } else {
          const DivFreeTab<DIM, ORDER> &T = kDivFree<DIM, ORDER>;
          ay = T.va[i] * S.v[T.ia[i] * DIM + T.ca[i]];
          if (T.ib[i] >= 0) ay += T.vb[i] * S.v[T.ib[i] * DIM + T.cb[i]];
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
      if (rho * dmax <= opt.refine_tol * ymax) conv = true;
    }
  }
  const bool not_conv = ok && !conv;
  const bool good = ok && conv;

  // ---- 7. weights: second pass over the rows, FP64 ----
  if constexpr (BASIS == 1) {
    divfree_apply_T<DIM, ORDER, G>(S.y, S.u, F, lg);
    __syncthreads();
  }
  if (good) {
    double *wout = a.weights + (int64_t)F * C * base;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int j = lg + G * r;
      if (j < N) {
        double s[DIM], w;
        load_row<DIM>(a, base, j, xt, ie, s, w);
        double p[Q];
        scaled_basis<DIM, ORDER, double>(s, p);
        for (int f = 0; f < F; ++f)
          for (int c = 0; c < C; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
              if constexpr (BASIS == 0)
                acc += p[q] * S.y[f][q];
              else
                acc += p[q] * S.u[f][q * DIM + c];
            }
            wout[((int64_t)f * N + j) * C + c] = w * acc;
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

template <int DIM, int ORDER, int BASIS, int G>
__global__ __launch_bounds__(64) void k_mixed64(StencilArgs a, const int *list, const int *count,
                                                const int *offset, int *cursor, int *fb_list, BinMeta *meta,
                                                Stats *stats, Options opt) {
  using Cf = Mixed64Cfg<DIM, ORDER, BASIS, G>;
  __shared__ Mixed64LDS<DIM, ORDER, BASIS, G> S[Cf::TPW];
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
    mixed64_target<DIM, ORDER, BASIS, G>(a, rk, t, valid, lg, S[grp], fb_list, meta, stats, opt);
  }
}

}  // namespace gmls
