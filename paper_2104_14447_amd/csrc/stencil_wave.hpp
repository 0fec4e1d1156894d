// stencil_wave.hpp -- mixed-path stencils with one wavefront per target, for
// bases too large for the one-thread solve of the pipeline (scalar bases of
// up to 35 monomials, divergence-free bases whose scalar part has up to 35).
//
// The stencil of a functional lambda is alpha = W P y with (P^T W P) y =
// lambda (Section 2.1, normal equations; Section 2.5, functionals).  For one
// target the wavefront
//  1. gathers its rows j = lane + 64 r once (eps-scaled offsets s_j, kernel
//     weights w_j, kept in registers);
//  2. forms the FP64 moments mu_g = sum_j w_j s_j^g, |g| <= 2m: per-lane
//     partial sums in lexicographic order of g, summed over the wavefront
//     through LDS in rounds of 16 moments (fixed order: reproducible);
//  3. builds the Jacobi-equilibrated moment Gram E_ik = mu_(i+k) / sqrt(
//     mu_2i mu_2k) (the factorials of the scaled basis cancel), lane i
//     holding row i, and inverts it in FP64 by symmetric sweeps (Gauss-Jordan
//     on a symmetric positive definite matrix, no pivoting: every pivot is a
//     Schur-complement diagonal in (0, 1]); the 1-norm condition number is
//     exact here, ||E||_1 ||E^-1||_1, and is held against the threshold;
//  4. scalar basis: y = G^-1 lambda with G^-1 = Dg E^-1 Dg (Dg_i = i! /
//     sqrt(mu_2i)); divergence-free basis (Section 2.2): the fit over the
//     kernel of the divergence map, as in the pipeline (g = G^-1 (l - D^T t),
//     S t = D G^-1 l, S = D G^-1 D^T), with S equilibrated and swept too;
//  5. alpha_j = w_j p(s_j) . y by Horner steps, the coefficients broadcast
//     through LDS, stores coalesced over the rows.
// Targets whose sweep meets a non-positive pivot or whose condition number
// exceeds the threshold are queued for the FP64 QR fallback.
#pragma once

#include <float.h>
#include <limits.h>
#include <math.h>

#include "basis.hpp"
#include "gmls_internal.hpp"
#include "stencil_mixed64.hpp"
#include "stencil_pipe.hpp"

namespace gmls {

// index of the moment s^(x,y,z), |g| <= D2, in lexicographic order (x
// slowest): the order in which the wavefront accumulates them
template <int DIM, int D2>
struct LexMoments {
  static constexpr int N = num_mono(DIM, D2);
  int id[D2 + 1][D2 + 1][D2 + 1];
  int e[N][3];
  constexpr LexMoments() : id{}, e{} {
    int n = 0;
    for (int x = 0; x <= D2; ++x)
      for (int y = 0; y <= (DIM >= 2 ? D2 - x : 0); ++y)
        for (int z = 0; z <= (DIM == 3 ? D2 - x - y : 0); ++z) {
          id[x][y][z] = n;
          e[n][0] = x;
          e[n][1] = y;
          e[n][2] = z;
          ++n;
        }
  }
};

// lexicographic moment index of basis monomials i + k (row-major Q x Q)
template <int DIM, int ORDER>
struct WavePairs {
  static constexpr int Q = num_mono(DIM, ORDER);
  unsigned char p[Q * Q];
  constexpr WavePairs() : p{} {
    Mono<DIM, ORDER> M{};
    LexMoments<DIM, 2 * ORDER> L{};
    for (int i = 0; i < Q; ++i)
      for (int k = 0; k < Q; ++k)
        p[i * Q + k] =
            (unsigned char)L.id[M.e[i][0] + M.e[k][0]][M.e[i][1] + M.e[k][1]][M.e[i][2] + M.e[k][2]];
  }
};
static_assert(num_mono(3, 8) < 256, "moment indices fit a byte");

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Symmetric sweep of every pivot of the Q x Q symmetric matrix whose row
// `lane` is a[] (lanes >= Q hold zeros): on return a[] is row `lane` of
// -A^-1.  Sweeping the pivot set P: A_PP <- -A_PP^-1, A_iP <- A_iP A_PP^-1,
// A_Pj <- A_PP^-1 A_Pj, A_ij <- A_ij - A_iP A_PP^-1 A_Pj (i, j not in P);
// sweeps of disjoint sets commute, so the pivots are taken two at a time
// (2 x 2 blocks, one reciprocal of the determinant each) and a trailing
// single pivot for odd Q.  The matrix stays symmetric, so columns k, k+1
// (one LDS store per lane) are also rows k, k+1; the column buffers
// alternate between steps (col: 4 x 64 doubles, 16-byte aligned), one
// barrier per step.
// Each step updates the next step's pivot columns first, stores them, and
// takes the next pivot block (from the registers of its lanes) and its
// reciprocal before the rest of its update, so that this chain overlaps
// the step's bulk of independent multiply-adds.
// Returns false when a leading pivot of a block is not above tol
// (wave-uniform).
template <int Q>
__device__ __forceinline__ bool sweep_inverse(double (&a)[Q], double *col, double tol) {
  const int lane = lane_id();
  bool ok = true;
  // a step's two pivot columns, interleaved: cc[j] = (A_jk, A_j,k+1), so
  // that one 16-byte LDS read brings both operands of the update of a[j]
  double2 *cb[2] = {(double2 *)col, (double2 *)(col + 128)};
  // pivot block of the current step: p00, p01, p11 and 1/det (2 x 2), or
  // p00 and 1/p00 (the trailing single pivot)
  double p00 = 0.0, p01 = 0.0, p11 = 0.0, det = 1.0, id = 1.0;
  if constexpr (Q >= 2) {
    if (lane < Q) cb[0][lane] = make_double2(a[0], a[1]);
    p00 = readlane_d(a[0], 0);
    p01 = readlane_d(a[0], 1);
    p11 = readlane_d(a[1], 1);
    det = p00 * p11 - p01 * p01;
    id = 1.0 / det;
  } else {
    if (lane < Q) cb[0][lane].x = a[0];
    p00 = readlane_d(a[0], 0);
    id = 1.0 / p00;
  }
#pragma unroll
  for (int k = 0; k + 1 < Q; k += 2) {
    const double2 *cc = cb[(k >> 1) & 1];
    double2 *nc = cb[((k >> 1) + 1) & 1];  // the next step's columns
    __syncthreads();
    ok = ok && p00 > tol && det > tol * p00;
    const double i00 = p11 * id, i01 = -p01 * id, i11 = p00 * id;
    const double ak = a[k], ak1 = a[k + 1];
    const double f0 = ak * i00 + ak1 * i01, f1 = ak * i01 + ak1 * i11;
    // rows k, k+1 themselves become A_PP^-1 A_Pj: their f is the unit
    // vector up to rounding, so the same update with e = A_PP^-1 applies
    const bool l0 = lane == k, l1 = lane == k + 1;
    const double e0 = (l0 ? i00 : l1 ? i01 : 0.0) - f0;
    const double e1 = (l0 ? i01 : l1 ? i11 : 0.0) - f1;
    // pivots of the next step: 2, 1 (the trailing single pivot) or none
    // (the loop is unrolled, so NX and the indices below are constants)
    const int NX = (k + 3 < Q) ? 2 : (k + 2 < Q ? 1 : 0);
    const int q0 = k + 2 < Q ? k + 2 : Q - 1, q1 = k + 3 < Q ? k + 3 : Q - 1;
    if (NX >= 1) {
      const double2 c = cc[q0];
      a[q0] = fma(e0, c.x, fma(e1, c.y, a[q0]));
    }
    if (NX == 2) {
      const double2 c = cc[q1];
      a[q1] = fma(e0, c.x, fma(e1, c.y, a[q1]));
    }
    if (NX == 2) {
      if (lane < Q) nc[lane] = make_double2(a[q0], a[q1]);
      p00 = readlane_d(a[q0], q0);
      p01 = readlane_d(a[q0], q1);
      p11 = readlane_d(a[q1], q1);
      det = p00 * p11 - p01 * p01;
      id = 1.0 / det;
    } else if (NX == 1) {
      if (lane < Q) nc[lane].x = a[q0];
      p00 = readlane_d(a[q0], q0);
      id = 1.0 / p00;
    }
#pragma unroll
    for (int j = 0; j < Q; ++j)
      if (j != k && j != k + 1 && (j < k + 2 || j >= k + 2 + NX)) {
        const double2 c = cc[j];
        a[j] = fma(e0, c.x, fma(e1, c.y, a[j]));
      }
    a[k] = l0 ? -i00 : l1 ? -i01 : f0;
    a[k + 1] = l0 ? -i01 : l1 ? -i11 : f1;
    // finish this step's updates here: left alone, the compiler defers each
    // a[j] update to the step that first reads it, which keeps every
    // earlier pivot column live (quadratic register use)
#pragma unroll
    for (int j = 0; j < Q; ++j) asm volatile("" : "+v"(a[j]));
  }
  if constexpr (Q % 2 == 1) {
    constexpr int k = Q - 1;
    const double2 *cc = cb[(Q / 2) & 1];
    __syncthreads();
    ok = ok && p00 > tol;
    const double d = id;
    const double f = a[k] * d;
    const double ef = (lane == k ? d : 0.0) - f;
#pragma unroll
    for (int j = 0; j < Q - 1; ++j) a[j] = fma(ef, cc[j].x, a[j]);
    a[k] = lane == k ? -d : f;
  }
  __syncthreads();  // the buffers may be rewritten after this
  return ok;
}

// Moments mu_g (lexicographic order) of the rows held by the wavefront into
// mu[]; red is the LDS reduction buffer (64 x (RS + 1) doubles, 16-byte aligned).  One step per
// moment, unrolled by template recursion so that every exponent, register
// index and round boundary is a compile-time constant.  RS moments go
// through LDS per round (8, 16 or 32: the autotuner's choice, a trade of
// registers and LDS for barriers).

// sum one round over the wavefront: every lane stores its partials
// (moment q of lane L at q * 66 + L: a moment's partials are contiguous),
// then lanes q + RS p add lanes RS p .. RS p + RS - 1 of moment q, read 16
// bytes at a time, and butterfly steps combine the 64 / RS parts (fixed
// order).  red: 16-byte aligned, RS * 66 <= 64 * (RS + 1) doubles.
template <int NM, int RS>
__device__ __forceinline__ void wave_round(const double (&acc)[RS], int g0, double *red, double *mu) {
  static_assert(RS == 8 || RS == 16 || RS == 32, "round size");
  constexpr int W = 66;
  static_assert(RS * W <= 64 * (RS + 1), "the tile fits the reduction buffer");
  const int lane = lane_id();
#pragma unroll
  for (int q = 0; q < RS; ++q) red[q * W + lane] = acc[q];
  __syncthreads();
  const int q = lane & (RS - 1), part = lane / RS;
  // pairwise sum of the RS lanes' values (fixed order; a chain of log2 RS
  // dependent adds instead of RS)
  double v[RS];
  const double2 *row = reinterpret_cast<const double2 *>(red + q * W + part * RS);
#pragma unroll
  for (int l = 0; l < RS / 2; ++l) {
    const double2 t = row[l];
    v[2 * l] = t.x;
    v[2 * l + 1] = t.y;
  }
#pragma unroll
  for (int h = RS / 2; h >= 1; h >>= 1)
#pragma unroll
    for (int l = 0; l < h; ++l) v[l] = v[l] + v[l + h];
  double t = v[0];
#pragma unroll
  for (int o = RS; o < 64; o <<= 1) t += __shfl_xor(t, o);
  if (lane < RS && g0 + lane < NM) mu[g0 + lane] = t;
  __syncthreads();
}

template <int DIM, int ORDER, int RPL, int RS, int G>
struct WaveMoment {
  static constexpr int D2 = 2 * ORDER;
  static constexpr int NM = num_mono(DIM, D2);
  // wab = w s_x^a [s_y^b] of the current prefix, pl = powers of the last coordinate
  static __device__ __forceinline__ void run(const double (&s)[RPL][DIM], const double (&pl)[RPL][D2 + 1],
                                             double (&wa)[RPL], double (&wab)[RPL], double (&acc)[RS],
                                             double *red, double *mu) {
    constexpr LexMoments<DIM, D2> LM{};
    constexpr int ey = LM.e[G][1];
    constexpr int el = DIM == 3 ? LM.e[G][2] : LM.e[G][1];
    // a new (x[, y]) prefix starts where the last exponent is 0
    if constexpr (G > 0 && el == 0) {
      if constexpr (DIM == 3 && ey == 0) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          wa[r] *= s[r][0];
          wab[r] = wa[r];
        }
      } else if constexpr (DIM == 3) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) wab[r] *= s[r][1];
      } else {
#pragma unroll
        for (int r = 0; r < RPL; ++r) wab[r] *= s[r][0];
      }
    }
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) v = fma(wab[r], pl[r][el], v);
    acc[G % RS] = v;
    if constexpr (G % RS == RS - 1 || G == NM - 1) wave_round<NM, RS>(acc, G - G % RS, red, mu);
    if constexpr (G + 1 < NM) WaveMoment<DIM, ORDER, RPL, RS, G + 1>::run(s, pl, wa, wab, acc, red, mu);
  }
};

template <int DIM, int ORDER, int RPL, int RS>
__device__ __forceinline__ void wave_moments(const double (&s)[RPL][DIM], const double (&w)[RPL], double *red,
                                             double *mu) {
  constexpr int D2 = 2 * ORDER;
  double pl[RPL][D2 + 1], wa[RPL], wab[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    pl[r][0] = 1.0;
#pragma unroll
    for (int c = 1; c <= D2; ++c) pl[r][c] = pl[r][c - 1] * s[r][DIM - 1];
    wa[r] = w[r];
    wab[r] = w[r];
  }
  double acc[RS];
  WaveMoment<DIM, ORDER, RPL, RS, 0>::run(s, pl, wa, wab, acc, red, mu);
}

// sum_q e[q] Dg_q lambda_q over the nonzero entries lambda_q of a functional
// on the scaled basis (Section 2.5), Dg_q = q! dsc_q: the value reads monomial
// 0; a gradient component the linear monomial s_d (1/eps); the Laplacian the
// three pure squares s_d^2 (1/eps^2 each, their 1/2! cancelled by q!).  The
// monomial indices are compile-time, so e[] stays in registers.
template <int DIM, int ORDER, int QS, int I>
__device__ __forceinline__ double lam_term(const double (&e)[QS], const double *dsc) {
  constexpr InvFact64<DIM, ORDER> IF{};
  return e[I] * (dsc[I] * (1.0 / IF.v[I]));
}

template <int DIM, int ORDER, int QS>
__device__ __forceinline__ double lambda_dot(int kind, const double (&e)[QS], const double *dsc, double ie) {
  constexpr MonoIndex<DIM, ORDER> MI{};
  if (kind == FK_VALUE) return lam_term<DIM, ORDER, QS, 0>(e, dsc);
  if constexpr (ORDER >= 1) {
    if (kind == FK_GRAD0) return ie * lam_term<DIM, ORDER, QS, MI.idx[1][0][0]>(e, dsc);
    if (kind == FK_GRAD1) return ie * lam_term<DIM, ORDER, QS, MI.idx[0][1][0]>(e, dsc);
    if constexpr (DIM == 3)
      if (kind == FK_GRAD2) return ie * lam_term<DIM, ORDER, QS, MI.idx[0][0][1]>(e, dsc);
  }
  if constexpr (ORDER >= 2) {
    if (kind == FK_LAP) {
      double t = lam_term<DIM, ORDER, QS, MI.idx[2][0][0]>(e, dsc) + lam_term<DIM, ORDER, QS, MI.idx[0][2][0]>(e, dsc);
      if constexpr (DIM == 3) t += lam_term<DIM, ORDER, QS, MI.idx[0][0][2]>(e, dsc);
      return ie * ie * t;
    }
  }
  return 0.0;
}

// Per-block counters, added to the call's statistics once per block.
struct WaveCounts {
  unsigned long long good = 0, fell = 0;
  double cond = 0.0;
};

// Queue of one stencil set: its arguments, fallback list and counter.
struct WaveSet {
  StencilArgs a;
  int *fb_list;
  int *fb_count;
};

// The rows are written in two steps: first the polynomial coefficients of
// every functional of every set, into LDS, while the rows of E^-1 (and of
// S^-1) are in registers; then the weights of every row from those
// coefficients, with the inverses dead (their registers free for the
// coefficients of the Horner steps).

// Scalar basis, coefficients: y_i / i! = dsc_i (E^-1 Dg lambda)_i of
// functional f into cf[f * 64 + i], from e = row `lane` of -E^-1.
template <int DIM, int ORDER>
__device__ __forceinline__ void wave_scalar_coefs(const StencilArgs &as, const RowKinds &rk,
                                                  const double (&e)[num_mono(DIM, ORDER)], double dsc,
                                                  const double *dscv, double ie, double *cf) {
  constexpr int QS = num_mono(DIM, ORDER);
  const int lane = lane_id();
  for (int f = 0; f < as.F; ++f) cf[f * 64 + lane] = -dsc * lambda_dot<DIM, ORDER, QS>(rk.kind[f], e, dscv, ie);
}

// Scalar basis, weights of every row of `as` (cfb: the coefficients above,
// visible to the whole wavefront).
template <int DIM, int ORDER, int RPL>
__device__ __forceinline__ void wave_scalar_weights(const StencilArgs &as, int64_t base, int N,
                                                    const double (&s)[RPL][DIM], const double (&w)[RPL],
                                                    const double *cfb) {
  constexpr int QS = num_mono(DIM, ORDER);
  const int lane = lane_id();
  const int F = as.F;
  double *wout = as.weights + (int64_t)F * base;
  for (int f = 0; f < F; ++f) {
    double cf[QS];
#pragma unroll
    for (int k = 0; k < QS; ++k) cf[k] = cfb[f * 64 + k];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int j = lane + 64 * r;
      const double val = w[r] * horner<DIM, ORDER>(cf, s[r]);
      if (j < N) wout[(int64_t)f * N + j] = val;
    }
  }
}

// Divergence-free basis, offsets in `big` of the coefficient step's buffers:
// [c][QM] ds_b r_b, [c][k][QM] t_b Dg_(b+e_k), then per row group g (at most
// two groups precede the divergence row) [g][c][k][QS] g / q!.
template <int DIM, int ORDER>
struct DivBuf {
  static constexpr int QS = num_mono(DIM, ORDER);
  static constexpr int QM = ORDER >= 1 ? num_mono(DIM, ORDER - 1) : 1;
  static constexpr int RB = 0, TDG = DIM * QM, CF = TDG + DIM * DIM * QM;
  static constexpr int GROUP = DIM * DIM * QS;
  static constexpr int SIZE = CF + 2 * GROUP;
};

// Divergence-free basis, coefficients: S = D G^-1 D^T from E^-1, its sweep,
// and the coefficients of every row group of `av` into big (DivBuf).
// Returns false when S breaks down (the target then goes to the FP64
// kernel); `big`, vb and colb are free on entry.
template <int DIM, int ORDER>
__device__ __forceinline__ bool wave_divfree_coefs(const StencilArgs &av, const RowKinds &rk,
                                                   const double (&e)[num_mono(DIM, ORDER)], double dg, double ifac,
                                                   const int (&ubl)[3], const double *dscv, double ie, double *big,
                                                   double (*vb)[64], double *colb) {
  constexpr int QS = num_mono(DIM, ORDER);
  constexpr int QM = ORDER >= 1 ? num_mono(DIM, ORDER - 1) : 1;
  constexpr DivUp<DIM, ORDER> DU{};
  using DB = DivBuf<DIM, ORDER>;
  const int lane = lane_id();
  const int F = av.F;
  // S = D G^-1 D^T: S_(b,b2) = sum_k G^-1_(up[b][k], up[b2][k]); lane b holds row b
  if (lane < QS)
#pragma unroll
    for (int k = 0; k < QS; ++k) big[lane * QS + k] = e[k];
  vb[2][lane] = dg;
  __syncthreads();
  double sr[QM];
  double sdiag = 1.0;
#pragma unroll
  for (int b2 = 0; b2 < QM; ++b2) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) v -= vb[2][ubl[k]] * big[ubl[k] * QS + DU.up[b2][k]] * vb[2][DU.up[b2][k]];
    sr[b2] = lane < QM ? v : 0.0;
    if (lane == b2) sdiag = v;
  }
  // equilibrate S (ds_b = 1/sqrt(S_bb)) and sweep it: sr = -(ds S ds)^-1
  const double ds = lane < QM ? 1.0 / sqrt(sdiag) : 0.0;
  vb[3][lane] = ds;
  __syncthreads();
#pragma unroll
  for (int b2 = 0; b2 < QM; ++b2) sr[b2] *= ds * vb[3][b2];
  if (!sweep_inverse<QM>(sr, colb, 1e-14)) return false;  // ends with a barrier: big is free
  // rows come in groups of DIM (one kind, components 0..DIM-1), then the
  // divergence row; per group, for component c of the functional:
  //   v = G^-1 l (the same for every c), r_b = v_(b + e_c),
  //   t = S^-1 r = ds (ds S ds)^-1 ds r,
  //   g_(c,k) = delta_(k,c) v - G^-1 D_k^T t, D_k^T t = sum_b t_b e_(b+e_k),
  // whose columns of E^-1 are this lane's registers
  double *rb = big + DB::RB;
  double *tdg = big + DB::TDG;
  for (int f0 = 0, g = 0; f0 < F; f0 += DIM, ++g) {
    const int kind = rk.kind[f0];
    if (kind == FK_DIV) break;  // identically zero on a divergence-free fit: the last row
    double *cfb = big + DB::CF + g * DB::GROUP;
    const double v = -dg * lambda_dot<DIM, ORDER, QS>(kind, e, dscv, ie);
    vb[1][lane] = v;
    __syncthreads();
    if (lane < QM)
#pragma unroll
      for (int c = 0; c < DIM; ++c) rb[c * QM + lane] = vb[1][ubl[c]] * ds;
    __syncthreads();
    if (lane < QM) {
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        double tt = 0.0;
#pragma unroll
        for (int b2 = 0; b2 < QM; ++b2) tt = fma(sr[b2], rb[c * QM + b2], tt);
        tt = -ds * tt;
#pragma unroll
        for (int k = 0; k < DIM; ++k) tdg[(c * DIM + k) * QM + lane] = tt * vb[2][ubl[k]];
      }
    }
    __syncthreads();
    if (lane < QS) {
#pragma unroll
      for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          double u = 0.0;
#pragma unroll
          for (int b = 0; b < QM; ++b) u = fma(e[DU.up[b][k]], tdg[(c * DIM + k) * QM + b], u);
          const double gv = (k == c ? v : 0.0) + dg * u;
          cfb[(c * DIM + k) * QS + lane] = gv * ifac;
        }
    }
  }
  return true;
}

// Divergence-free basis, weights of every row of `av` from the coefficients
// in big (visible to the whole wavefront).
template <int DIM, int ORDER, int RPL>
__device__ __forceinline__ void wave_divfree_weights(const StencilArgs &av, const RowKinds &rk, int64_t base,
                                                     int N, const double (&s)[RPL][DIM], const double (&w)[RPL],
                                                     const double *big) {
  constexpr int QS = num_mono(DIM, ORDER);
  using DB = DivBuf<DIM, ORDER>;
  const int lane = lane_id();
  const int F = av.F;
  double *wout = av.weights + (int64_t)F * DIM * base;
  for (int f0 = 0, g = 0; f0 < F; f0 += DIM, ++g) {
    if (rk.kind[f0] == FK_DIV) {
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int j = lane + 64 * r;
#pragma unroll
        for (int k = 0; k < DIM; ++k)
          if (j < N) wout[((int64_t)f0 * N + j) * DIM + k] = 0.0;
      }
      break;  // the last row
    }
    const double *cfb = big + DB::CF + g * DB::GROUP;
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        double cf[QS];
#pragma unroll
        for (int q = 0; q < QS; ++q) cf[q] = cfb[(c * DIM + k) * QS + q];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int j = lane + 64 * r;
          const double val = w[r] * horner<DIM, ORDER>(cf, s[r]);
          if (j < N) wout[((int64_t)(f0 + c) * N + j) * DIM + k] = val;
        }
      }
  }
}

// BASIS 0 scalar set (ss), 1 divergence-free set (sv), 3 both on the same
// neighbour lists: the moments and the swept Gram are formed once per target
// for both sets (Section 2.2: the divergence-free fit is the scalar fit under
// D c = 0, so both take the same G).
// CAND: the compiled variant (kWaveCand).
template <int DIM, int ORDER, int BASIS, int RPL, int CAND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWaveCand[CAND].wpe))) void k_wave(
    WaveSet ss, WaveSet sv, const int *list, BinMeta *meta, int bin, Stats *stats, Options opt) {
  constexpr bool SCAL = BASIS == 0 || BASIS == 3, DIVF = BASIS == 1 || BASIS == 3;
  constexpr int QS = num_mono(DIM, ORDER);
  constexpr int NM = num_mono(DIM, 2 * ORDER);
  constexpr int QM = ORDER >= 1 ? num_mono(DIM, ORDER - 1) : 1;
  constexpr int RS = kWaveCand[CAND].rs;
  constexpr int RED = 64 * (RS + 1);
  constexpr int BIG = (DIVF && QS * QS > RED) ? QS * QS : RED;
  static_assert(QS <= 64, "one basis function per lane");
  static_assert(!DIVF || DivBuf<DIM, ORDER>::SIZE <= BIG, "divergence-free buffers fit");
  static_assert(5 * 64 <= BIG, "scalar coefficients fit");
  __shared__ __align__(16) double big[BIG];  // moment reduction, then (divergence-free) -E^-1
  __shared__ double mu[NM];        // moments, lexicographic order
  __shared__ double vb[4][64];     // broadcast vectors
  __shared__ __align__(16) double colb[4 * 64];  // pivot columns of the sweeps
  __shared__ unsigned char pidx[QS * QS];
  // the scalar set's coefficients [f][64]: their own buffer when the
  // divergence-free set's coefficients take `big` (shared calls)
  __shared__ double cfs_own[BASIS == 3 ? 5 * 64 : 1];
  double *cfs = BASIS == 3 ? cfs_own : big;
  constexpr WavePairs<DIM, ORDER> WP{};
  constexpr InvFact64<DIM, ORDER> IF{};
  const StencilArgs &a = SCAL ? ss.a : sv.a;  // the common inputs
  const int lane = lane_id();
  for (int q = lane; q < QS * QS; q += 64) pidx[q] = WP.p[q];
  const double ifac = IF.v[lane < QS ? lane : 0];  // 1 / i!
  int ubl[3] = {0, 0, 0};                             // divergence-free: index of b + e_k, b = lane
  if constexpr (DIVF) {
    constexpr DivUp<DIM, ORDER> DU{};
    if (lane < QM)
#pragma unroll
      for (int k = 0; k < DIM; ++k) ubl[k] = DU.up[lane][k];
  }
  __syncthreads();
  const RowKinds rks = row_kinds(DIM, 0, ss.a.mask), rkv = row_kinds(DIM, 1, sv.a.mask);
  WaveCounts cnt, cntv;
  const SlotRange R = slot_range(meta, bin, -1, INT_MAX);
  for (int i = R.first + xcd_block(); i < R.last; i += gridDim.x) {
    const int t = list[i];
    const int64_t base = a.row_ptr[t];
    const int N = (int)(a.row_ptr[t + 1] - base);
    const double ie = 1.0 / a.eps[t];
    double xt[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) xt[d] = a.targets[(int64_t)t * DIM + d];
    double s[RPL][DIM], w[RPL];
    {
      double xs[RPL][DIM];
      gather_rows<DIM, RPL, 64>(a, base, N, lane, xs);
#pragma unroll
      for (int r = 0; r < RPL; ++r) w[r] = row_sw<DIM>(xs[r], xt, ie, a.p, lane + 64 * r < N, s[r]);
    }
    wave_moments<DIM, ORDER, RPL, RS>(s, w, big, mu);

    // equilibrated Gram, row `lane` (lanes >= QS hold zeros; li keeps their
    // table reads in bounds)
    const int li = lane < QS ? lane : 0;
    const double dsc = lane < QS ? 1.0 / sqrt(mu[pidx[li * QS + li]]) : 0.0;
    vb[0][lane] = dsc;
    __syncthreads();
    double e[QS];
#pragma unroll
    for (int k = 0; k < QS; ++k) {
      // every lane loads (li is in range), so the QS reads go out together
      const double v = mu[pidx[li * QS + k]] * dsc * vb[0][k];
      e[k] = lane < QS ? v : 0.0;
    }
    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < QS; ++k) rs += fabs(e[k]);
    const double anorm = wave_max(rs);
    bool ok = sweep_inverse<QS>(e, colb, 1e-14);  // e = row `lane` of -E^-1
    rs = 0.0;
#pragma unroll
    for (int k = 0; k < QS; ++k) rs += fabs(e[k]);
    const double cond = anorm * wave_max(rs);
    if (lane == 0 && a.cond_out) a.cond_out[t] = (float)cond;
    if (!(cond <= opt.cond_threshold)) ok = false;
    if (opt.force_fallback) ok = false;
    const double dg = dsc / ifac;  // Dg_lane: G^-1 = Dg E^-1 Dg

    // the coefficients of both sets while the inverse rows are in
    // registers, then the weights of every row with those registers free
    if constexpr (SCAL)
      if (ok) wave_scalar_coefs<DIM, ORDER>(ss.a, rks, e, dsc, vb[0], ie, cfs);
    bool okv = ok;
    if constexpr (DIVF)
      if (ok) okv = wave_divfree_coefs<DIM, ORDER>(sv.a, rkv, e, dg, ifac, ubl, vb[0], ie, big, vb, colb);
    __syncthreads();
    if constexpr (SCAL) {
      if (ok) wave_scalar_weights<DIM, ORDER, RPL>(ss.a, base, N, s, w, cfs);
      if (lane == 0) {
        ss.a.status[t] = ok ? GMLS_TARGET_OK : GMLS_TARGET_FALLBACK;
        if (!ok) ss.fb_list[atomicAdd(ss.fb_count, 1)] = t;
      }
    }
    if constexpr (DIVF) {
      if (okv) wave_divfree_weights<DIM, ORDER, RPL>(sv.a, rkv, base, N, s, w, big);
      if (lane == 0) {
        sv.a.status[t] = okv ? GMLS_TARGET_OK : GMLS_TARGET_FALLBACK;
        if (!okv) sv.fb_list[atomicAdd(sv.fb_count, 1)] = t;
      }
    }
    __syncthreads();
    const bool good = SCAL ? ok : okv;  // statistics of the first set
    cnt.good += good ? 1 : 0;
    cnt.fell += good ? 0 : 1;
    if (cond >= 0.0) cnt.cond = fmax(cnt.cond, cond);  // NaN estimates are skipped
    if constexpr (BASIS == 3) {  // the divergence-free set of a shared call: its own counters
      cntv.good += okv ? 1 : 0;
      cntv.fell += okv ? 0 : 1;
    }
  }
  if (lane == 0) {
    if (cnt.good) atomicAdd(&stats->sweep_hist[0], cnt.good);
    if (cnt.fell) atomicAdd(&stats->n_fallback, cnt.fell);
    if (cnt.cond > 0.0) atomicMax(&stats->cond_max_bits, (unsigned long long)__double_as_longlong(cnt.cond));
    if constexpr (BASIS == 3) {  // stats[1]: the second set (shared calls pass two records)
      if (cntv.good) atomicAdd(&stats[1].sweep_hist[0], cntv.good);
      if (cntv.fell) atomicAdd(&stats[1].n_fallback, cntv.fell);
      if (cnt.cond > 0.0)
        atomicMax(&stats[1].cond_max_bits, (unsigned long long)__double_as_longlong(cnt.cond));
    }
  }
}

// One launch per non-empty row-count bin (bin b: rows <= 64 b, b rows per
// lane).  With a host copy of the bin table (hm) empty bins are skipped and
// grids sized to the bin; without one every bin is launched, sized for n_max
// targets, its bounds read on the device.
template <int DIM, int ORDER, int BASIS>
hipError_t launch_wave(const WaveSet &ss, const WaveSet &sv, const int *list, const BinMeta *hm, BinMeta *meta,
                       Stats *stats, const Options &opt, int n_max, int cus, PipeTimer *timer, hipStream_t s) {
  for (int b = 1; b < kNumBins; ++b) {
    int cnt = n_max;
    if (hm) {
      cnt = hm->count[b];
      if (cnt == 0) continue;
    }
    if (b == kLongBin) {  // rows over 256: the FP64 QR kernels take them in chunks
      hipError_t e = hipSuccess;
      if constexpr (BASIS == 0 || BASIS == 3)
        e = launch_defer_bin(ss.a.status, list, meta, b, ss.fb_list, ss.fb_count, stats, s);
      if constexpr (BASIS == 1 || BASIS == 3)
        if (e == hipSuccess)
          e = launch_defer_bin(sv.a.status, list, meta, b, sv.fb_list, sv.fb_count, BASIS == 3 ? stats + 1 : stats,
                               s);
      if (e != hipSuccess) return e;
      continue;
    }
    int nb = cnt < cus * 16 ? cnt : cus * 16;
    nb = xcd_grid(nb);
    const int c = opt.wave_shape[b] >= 0 && opt.wave_shape[b] < kWaveCands ? opt.wave_shape[b] : 0;
    if (timer) {
      const hipError_t e = hipEventRecord(timer->ev[2][b][0], s);
      if (e != hipSuccess) return e;
    }
    switch (b * 4 + c) {
#define GMLS_WAVE_CASE(B_, C_)                                                                                  \
  case B_ * 4 + C_:                                                                                             \
    k_wave<DIM, ORDER, BASIS, B_, C_><<<nb, 64, 0, s>>>(ss, sv, list, meta, b, stats, opt);                     \
    break;
      GMLS_WAVE_CASE(1, 0) GMLS_WAVE_CASE(1, 1) GMLS_WAVE_CASE(1, 2)
      GMLS_WAVE_CASE(2, 0) GMLS_WAVE_CASE(2, 1) GMLS_WAVE_CASE(2, 2)
      GMLS_WAVE_CASE(3, 0) GMLS_WAVE_CASE(3, 1) GMLS_WAVE_CASE(3, 2)
      GMLS_WAVE_CASE(4, 0) GMLS_WAVE_CASE(4, 1) GMLS_WAVE_CASE(4, 2)
#undef GMLS_WAVE_CASE
      default: return hipErrorInvalidValue;
    }
    if (timer) {
      const hipError_t e = hipEventRecord(timer->ev[2][b][1], s);
      if (e != hipSuccess) return e;
      timer->used[2][b] = 1;
    }
  }
  return hipGetLastError();
}

}  // namespace gmls
