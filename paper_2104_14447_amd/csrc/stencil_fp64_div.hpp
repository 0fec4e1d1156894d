#pragma once
// stencil_fp64_div.hpp -- FP64 stencils of the divergence-free basis
// (Section 2.2), one wavefront per target.
//
// The divergence-free span is the kernel of the divergence map D on the
// vector polynomials of degree <= m (coefficients c_(a,k) of p_a e_k; with
// the eps-scaled Taylor monomials d/ds_k p_a = p_(a - e_k), so (D c)_b =
// sum_k c_(b + e_k, k) for every monomial b of degree < m).  The weighted
// least squares over that span is the vector fit with Gram I (x) G, G = P^T W P
// (Section 2.1), under D c = 0, and for a functional l (scalar part lambda on
// component comp)
//     g_k = G^-1 (delta_(k,comp) lambda - D_k^T t),   S t = D G^-1 l,
//     S = D (I (x) G^-1) D^T = sum_k D_k G^-1 D_k^T,
// D_k the part of D acting on component k.  Everything is taken through the
// Householder factor R of the scalar sample matrix sqrt(W) P (G = R^T R,
// G^-1 = R^-1 R^-T):
//   * R^-1 by back substitution, one column per lane;
//   * S = B^T B with B = [R^-T D_0^T; ...; R^-T D_(d-1)^T] (d*Q x Q_m; column
//     b of block k is column b + e_k of R^-T), factored by a second
//     Householder QR, S = R_B^T R_B, so that neither G nor S is formed;
//   * alpha_(j,k) = w_j p(s_j) . g_k.
// The divergence functional of a divergence-free fit is identically zero.
// Targets whose R is rank deficient are queued for stencil_fp64_kmat.hpp.
#include <float.h>
#include <math.h>

#include "stencil_fp64.hpp"

namespace gmls {

// index of the monomial b + e_k (b of degree < ORDER), in the graded order of
// Mono<DIM, ORDER> whose first num_mono(DIM, ORDER - 1) entries are the
// monomials of degree < ORDER
template <int DIM, int ORDER>
struct DivUpIndex {
  static constexpr int QM = num_mono(DIM, ORDER - 1);
  int up[QM > 0 ? QM : 1][3];
  constexpr DivUpIndex() : up{} {
    Mono<DIM, ORDER> M{};
    MonoIndex<DIM, ORDER> MI{};
    for (int b = 0; b < QM; ++b)
      for (int k = 0; k < 3; ++k)
        up[b][k] = k < DIM ? MI.idx[M.e[b][0] + (k == 0)][M.e[b][1] + (k == 1)][M.e[b][2] + (k == 2)] : 0;
  }
};

template <int DIM, int ORDER>
constexpr int qr_divfree_lds_doubles() {
  constexpr int Q = num_mono(DIM, ORDER);
  constexpr int QM = num_mono(DIM, ORDER - 1);
  // R, R^-1; R_B row- and column-major; three broadcast vectors; u per row.
  // The second factor's column sums use the space after R^-1 before R_B is
  // written.
  constexpr int SOLVE = 2 * Q * Q + 2 * QM * QM + 3 * 64 + 8 * DIM * Q;
  constexpr int SUMS = 2 * Q * Q + kSumBufDoubles;
  return SOLVE > SUMS ? SOLVE : SUMS;
}

// The divergence-free weights from the scalar factor (qr_factor: lane k < Q
// holds row k of R in Rrow[k..Q-1], rdiag = R_kk).  R_IN_LDS: R is already
// in lds[0 .. Q*Q) row-major (qr_scalar_solve leaves it there whenever it
// passes the same rank test), and Rrow is not read.
template <int DIM, int ORDER, int RPL, bool R_IN_LDS = false>
__device__ __forceinline__ void qr_divfree_solve(const StencilArgs &a, const RowKinds &rk, int t,
                                                 Rows<DIM, RPL> &r, const double (&Rrow)[num_mono(DIM, ORDER)],
                                                 double rdiag, double *lds) {
  constexpr int Q = num_mono(DIM, ORDER);
  constexpr int QM = num_mono(DIM, ORDER - 1);
  constexpr int KB = DIM * Q;            // rows of B
  constexpr int KBL = (KB + 63) / 64;    // rows of B per lane
  constexpr DivUpIndex<DIM, ORDER> DU{};
  constexpr MonoIndex<DIM, ORDER> MI{};
  const int lane = lane_id();
  if (!R_IN_LDS && lane < Q) {
#pragma unroll
    for (int l = 0; l < Q; ++l) lds[lane * Q + l] = l >= lane ? Rrow[l] : 0.0;
  }
  const int F = a.F;
  double *Rs = lds;                 // R, row-major
  double *Ri = Rs + Q * Q;          // R^-1, row-major (upper triangular)
  double *RBm = Ri + Q * Q;         // R_B, row-major
  double *RBt = RBm + QM * QM;      // R_B, column-major
  double *V0 = RBt + QM * QM;       // broadcast vectors
  double *V1 = V0 + 64, *V2 = V1 + 64;
  double *U = V2 + 64;              // [f][q * DIM + k]: g_k of row f
  const double rmax = uniform_d(wave_max(lane < Q ? fabs(rdiag) : 0.0));
  const double rmin = uniform_d(wave_min(lane < Q ? fabs(rdiag) : DBL_MAX));
  bool deficient = !(rmin > kRankTol * rmax);
  if (readfirstlane_i(deficient ? 1 : 0) && a.aux_list) {
    // the scalar basis is not unisolvent on these neighbours, which does not
    // make the divergence-free fit singular: queue the target for the kernel
    // that factors the divergence-free sample matrix itself
    if (lane == 0) a.aux_list[atomicAdd(a.aux_count, 1)] = t;
    __syncthreads();
    return;
  }
  __syncthreads();
  // R^-1, column `lane`: R x = e_lane by back substitution (rows above the
  // diagonal only); every lane walks the same rows, so the reads of R are
  // broadcasts
  if (!readfirstlane_i(deficient ? 1 : 0)) {
    double x[Q];
#pragma unroll
    for (int i = Q - 1; i >= 0; --i) {
      double acc = i == lane ? 1.0 : 0.0;
#pragma unroll
      for (int l = i + 1; l < Q; ++l) acc -= Rs[i * Q + l] * x[l];
      x[i] = i <= lane ? acc * (1.0 / Rs[i * Q + i]) : 0.0;  // the reciprocal is off the chain
    }
    if (lane < Q)
#pragma unroll
      for (int i = 0; i < Q; ++i) Ri[i * Q + lane] = x[i];
    __syncthreads();
    // B, rows rho = k Q + a on lane rho % 64: B[rho][b] = R^-T[a][b + e_k] = R^-1[b + e_k][a]
    double MB[KBL][QM];
#pragma unroll
    for (int s = 0; s < KBL; ++s) {
      const int rho = lane + 64 * s;
      const int k = rho / Q, ar = rho - k * Q;
#pragma unroll
      for (int b = 0; b < QM; ++b) {
        const int u = k == 0 ? DU.up[b][0] : k == 1 ? DU.up[b][1] : DU.up[b][2];
        MB[s][b] = rho < KB ? Ri[u * Q + ar] : 0.0;
      }
    }
    double rdb;
    // the column sums through LDS past R^-1 once there are enough columns
    // to batch (a wave sum each is cheaper for a handful)
    wave_householder<QM, KBL, (QM >= 8)>(MB, rdb, lane, RBm);
    const double bmax = uniform_d(wave_max(lane < QM ? fabs(rdb) : 0.0));
    const double bmin = uniform_d(wave_min(lane < QM ? fabs(rdb) : DBL_MAX));
    deficient = !(bmin > kRankTol * bmax);
    if (lane < QM) {
#pragma unroll
      for (int l = 0; l < QM; ++l) {
        const double v = l >= lane ? MB[0][l] : 0.0;
        RBm[lane * QM + l] = v;
        RBt[l * QM + lane] = v;
      }
    }
    __syncthreads();
    if (!readfirstlane_i(deficient ? 1 : 0)) {
      const double ie = 1.0 / uniform_d(a.eps[t]);
      const int li = lane < Q ? lane : 0;  // keeps the lane's row reads in bounds
      for (int f = 0; f < F; ++f) {
        const int kind = rk.kind[f], comp = rk.comp[f];
        if (kind == FK_DIV) {
          if (lane < Q)
#pragma unroll
            for (int k = 0; k < DIM; ++k) U[f * KB + lane * DIM + k] = 0.0;
          continue;
        }
        // w1 = R^-T lambda over the nonzeros of lambda (value: monomial 0;
        // Laplacian: the pure squares, 1/eps^2 each)
        double w1 = 0.0;
        if (kind == FK_VALUE) {
          w1 = Ri[0 * Q + li];
        } else if constexpr (ORDER >= 2) {
          w1 = Ri[MI.idx[2][0][0] * Q + li] + Ri[MI.idx[0][2][0] * Q + li];
          if constexpr (DIM == 3) w1 += Ri[MI.idx[0][0][2] * Q + li];
          w1 *= ie * ie;
        }
        V0[lane] = lane < Q ? w1 : 0.0;
        __syncthreads();
        // v = R^-1 w1 = G^-1 lambda
        double v = 0.0;
#pragma unroll
        for (int l = 0; l < Q; ++l) v += Ri[li * Q + l] * V0[l];
        if (lane >= Q) v = 0.0;
        V1[lane] = v;
        __syncthreads();
        // r_b = v_(b + e_comp); t = S^-1 r = R_B^-1 R_B^-T r
        double rb = 0.0;
        if (lane < QM) {
          int u = 0;
#pragma unroll
          for (int b = 0; b < QM; ++b)
            if (lane == b) u = comp == 0 ? DU.up[b][0] : comp == 1 ? DU.up[b][1] : DU.up[b][2];
          rb = V1[u];
        }
        const double tb = tri_solve_rtr<QM>(RBm, RBt, rb, rdb, lane);
        V2[lane] = lane < QM ? tb : 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          // y = G^-1 D_k^T t = R^-1 (R^-T D_k^T t); (R^-T D_k^T t)_i = sum_b R^-1[b + e_k][i] t_b
          double w2 = 0.0;
#pragma unroll
          for (int b = 0; b < QM; ++b) w2 += Ri[DU.up[b][k] * Q + li] * V2[b];
          V0[lane] = lane < Q ? w2 : 0.0;
          __syncthreads();
          double y = 0.0;
#pragma unroll
          for (int l = 0; l < Q; ++l) y += Ri[li * Q + l] * V0[l];
          if (lane < Q) U[f * KB + lane * DIM + k] = (k == comp ? v : 0.0) - y;
          __syncthreads();
        }
      }
      __syncthreads();
    }
  }
  if (readfirstlane_i(deficient ? 1 : 0)) {
    for (int j = lane; j < r.N; j += 64)
      for (int f = 0; f < F; ++f)
        for (int c = 0; c < DIM; ++c) a.weights[(int64_t)F * DIM * r.base + ((int64_t)f * r.N + j) * DIM + c] = NAN;
    if (lane == 0) a.status[t] = GMLS_TARGET_RANK_DEFICIENT;
    __syncthreads();
    return;
  }
  for (int c0 = 0; c0 < r.N; c0 += 64 * RPL) {  // one pass unless the row is longer than 64 RPL
    if (r.first != c0) load_rows<DIM, RPL>(a, t, r, lane, c0);
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int j = c0 + lane + 64 * i;
      if (j < r.N) {
        double p[Q];
        scaled_basis<DIM, ORDER, double>(r.s[i], p);
        for (int f = 0; f < F; ++f)
          for (int c = 0; c < DIM; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) acc += p[q] * U[f * KB + q * DIM + c];
            a.weights[(int64_t)F * DIM * r.base + ((int64_t)f * r.N + j) * DIM + c] = r.w[i] * acc;
          }
      }
    }
  }
  if (lane == 0 && a.ok_status >= 0) a.status[t] = (uint8_t)a.ok_status;
  __syncthreads();
}

template <int DIM, int ORDER, int RPL>
__device__ __forceinline__ void qr_divfree_target(const StencilArgs &a, const RowKinds &rk, int t, double *lds) {
  constexpr int Q = num_mono(DIM, ORDER);
  Rows<DIM, RPL> r;
  double M[RPL][Q];
  double rdiag;
  qr_factor<DIM, ORDER, RPL>(a, t, r, M, rdiag, lane_id(), lds);  // lds is free until the solves
  qr_divfree_solve<DIM, ORDER, RPL>(a, rk, t, r, M[0], rdiag, lds);
}

}  // namespace gmls
