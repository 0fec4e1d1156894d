#pragma once
// stencil_fp64_kmat.hpp -- FP64 divergence-free stencils for targets whose
// scalar basis of the same order is not unisolvent on their neighbours (for
// instance N < Q scalar monomials while d*N still covers the Q_d
// divergence-free functions): the constrained form through the scalar
// factor R is not available there, so the divergence-free sample matrix is
// factored itself.  With psi = (p (x) I_d) T (Section 2.2; T the +-1
// coefficients of divfree.hpp) the vector sample matrix is
// (sqrt(W) P (x) I_d) T = (Q1 (x) I)(R (x) I) T, so its R factor is that of
// K = (R (x) I_d) T (d*Q x Q_d), factored by Householder QR in LDS:
//   y = R_K^{-1} R_K^{-T} lambda,  u = T y,  alpha_{j,c} = w_j p(s_j) . u_c.
// Targets reach this kernel through a queue filled by qr_divfree_target.
#include <float.h>
#include <math.h>

#include "divfree.hpp"
#include "stencil_fp64.hpp"

namespace gmls {

template <int DIM, int ORDER>
constexpr int qr_kmat_lds_doubles() {
  constexpr int Q = num_mono(DIM, ORDER);
  constexpr int QD = DivFreeTab<DIM, ORDER>::QD;
  constexpr int KR = DIM * Q;
  constexpr int SOLVE = Q * Q + QD * KR + 8 * QD + 8 * KR + QD;
  return SOLVE > kSumBufDoubles ? SOLVE : kSumBufDoubles;  // the factor's column sums come first
}

template <int DIM, int ORDER, int RPL>
__device__ void qr_divfree_kmat_target(const StencilArgs &a, const RowKinds &rk, int t, double *lds) {
  constexpr Mono<DIM, ORDER> MO{};
  constexpr int Q = MO.N;
  const DivFreeTab<DIM, ORDER> &DF = kDivFree<DIM, ORDER>;
  constexpr int QD = DivFreeTab<DIM, ORDER>::QD;
  constexpr int KR = DIM * Q;  // rows of K
  const int lane = lane_id();
  Rows<DIM, RPL> r;
  double M[RPL][Q];
  double rdiag;
  qr_factor<DIM, ORDER, RPL>(a, t, r, M, rdiag, lane, lds);  // any row count (chunked when long)
  const int F = a.F;
  // scalar R in LDS (row-major), then K = (R (x) I) T column-major [QD][KR]
  double *Rs = lds;              // Q*Q
  double *K = lds + Q * Q;       // QD*KR
  double *Y = K + QD * KR;       // F*QD (y), then F*KR (u = T y)
  double *U = Y + 8 * QD;
  if (lane < Q) {
#pragma unroll
    for (int l = 0; l < Q; ++l) Rs[lane * Q + l] = l >= lane ? M[0][l] : 0.0;
  }
  __syncthreads();
  // K[(alpha, c), i] = sum_beta R[alpha][beta] T[(beta, c), i]; T has at most
  // two nonzeros per column: (ia, ca, va) and (ib, cb, vb)
  for (int e = lane; e < QD * KR; e += 64) {
    const int i = e / KR, row = e - i * KR;
    const int al = row / DIM, c = row - al * DIM;
    double v = 0.0;
    const int ia = DF.ia[i], ib = DF.ib[i];
    if (DF.ca[i] == c) v += DF.va[i] * Rs[al * Q + ia];
    if (ib >= 0 && DF.cb[i] == c) v += DF.vb[i] * Rs[al * Q + ib];
    K[e] = v;
  }
  __syncthreads();
  // Householder QR of K (KR x QD, column-major) in LDS, rows across lanes:
  // lane l owns rows l + 64 q of every column, so a column update touches
  // only the lane's own entries; the dot products of the reflector with the
  // later columns are taken CH at a time and summed over the wavefront by
  // DPP (independent chains, no LDS traffic)
  constexpr int KRL = (KR + 63) / 64;
  constexpr int CH = 8;
  double *Kd = U + 8 * KR;  // QD diagonal entries of R_K
  for (int k = 0; k < QD; ++k) {
    double xs[KRL];
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < KRL; ++q) {
      const int row = lane + 64 * q;
      xs[q] = (row >= k && row < KR) ? K[k * KR + row] : 0.0;
      part += xs[q] * xs[q];
    }
    const double sigma = uniform_d(wave_sum_uniform(part));  // a scalar branch below
    const double xk = uniform_d(K[k * KR + k]);
    double beta = 0.0;
    if (sigma > 0.0) {
      const double norm = sqrt(sigma);
      beta = xk >= 0.0 ? -norm : norm;
      const double inv_vtv = 1.0 / (2.0 * beta * (beta - xk));
      double v[KRL];
#pragma unroll
      for (int q = 0; q < KRL; ++q) {
        const int row = lane + 64 * q;
        v[q] = row == k ? xk - beta : xs[q];
      }
      for (int l0 = k + 1; l0 < QD; l0 += CH) {
        double kv[CH][KRL], dp[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          dp[u] = 0.0;
#pragma unroll
          for (int q = 0; q < KRL; ++q) {
            const int row = lane + 64 * q;
            kv[u][q] = (l0 + u < QD && row >= k && row < KR) ? K[(l0 + u) * KR + row] : 0.0;
            dp[u] += v[q] * kv[u][q];
          }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) dp[u] = wave_sum_uniform(dp[u]);
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const double coef = 2.0 * dp[u] * inv_vtv;
#pragma unroll
          for (int q = 0; q < KRL; ++q) {
            const int row = lane + 64 * q;
            if (l0 + u < QD && row >= k && row < KR) K[(l0 + u) * KR + row] = kv[u][q] - coef * v[q];
          }
        }
      }
    }
    __syncthreads();
    if (lane == 0) {
      K[k * KR + k] = beta;
      Kd[k] = beta;
    }
    __syncthreads();
  }
  // rank test on both factors
  double dmax = 0.0, dmin = DBL_MAX;
  for (int k = lane; k < QD; k += 64) {
    dmax = fmax(dmax, fabs(Kd[k]));
    dmin = fmin(dmin, fabs(Kd[k]));
  }
  dmax = uniform_d(wave_max(dmax));
  dmin = uniform_d(wave_min(dmin));
  if (readfirstlane_i(!(dmin > kRankTol * dmax) ? 1 : 0)) {
    for (int j = lane; j < r.N; j += 64)
      for (int f = 0; f < F; ++f)
        for (int c = 0; c < DIM; ++c) a.weights[(int64_t)F * DIM * r.base + ((int64_t)f * r.N + j) * DIM + c] = NAN;
    if (lane == 0) a.status[t] = GMLS_TARGET_RANK_DEFICIENT;
    __syncthreads();
    return;
  }
  const double ie = 1.0 / uniform_d(a.eps[t]);
  // y = R_K^{-1} R_K^{-T} lambda for every row at once; R_K[k][l] = K[l*KR + k].
  // lambda_i = functional on psi_i: value c -> T[(0,c),i]; Laplacian c ->
  // eps^-2 sum_d T[(2e_d,c),i]; divergence -> 0 (a divergence-free fit)
  for (int f = 0; f < F; ++f) {
    const int kind = rk.kind[f], comp = rk.comp[f];
    for (int i = lane; i < QD; i += 64)
      Y[f * QD + i] = kind == FK_DIV ? 0.0 : divfree_lambda<DIM, ORDER>(i, kind, comp, ie);
  }
  // forward R_K^T z = lambda, then back R_K y = z: one pivot per step for all
  // rows, one barrier per step (the pivot's entry was last written by the
  // lane that owns it in the step before)
  for (int k = 0; k < QD; ++k) {
    __syncthreads();
    const double id = 1.0 / uniform_d(Kd[k]);
    double zk[8];
#pragma unroll
    for (int f = 0; f < 8; ++f) zk[f] = f < F ? uniform_d(Y[f * QD + k]) * id : 0.0;
    if (lane == 0)
#pragma unroll
      for (int f = 0; f < 8; ++f)
        if (f < F) Y[f * QD + k] = zk[f];
    for (int l = k + 1 + lane; l < QD; l += 64) {
      const double rkl = K[l * KR + k];
#pragma unroll
      for (int f = 0; f < 8; ++f)
        if (f < F) Y[f * QD + l] -= rkl * zk[f];
    }
  }
  for (int k = QD - 1; k >= 0; --k) {
    __syncthreads();
    const double id = 1.0 / uniform_d(Kd[k]);
    double yk[8];
#pragma unroll
    for (int f = 0; f < 8; ++f) yk[f] = f < F ? uniform_d(Y[f * QD + k]) * id : 0.0;
    if (lane == 0)
#pragma unroll
      for (int f = 0; f < 8; ++f)
        if (f < F) Y[f * QD + k] = yk[f];
    for (int l = lane; l < k; l += 64) {
      const double rlk = K[k * KR + l];
#pragma unroll
      for (int f = 0; f < 8; ++f)
        if (f < F) Y[f * QD + l] -= rlk * yk[f];
    }
  }
  __syncthreads();
  // u = T y (KR entries per row): the first entries (ia, ca) of the columns
  // are distinct, so they are stored in parallel; the second entries
  // (ib, 0) of columns with the same ca are distinct too, so they are added
  // one component ca at a time (a fixed order: reproducible)
  for (int e = lane; e < F * KR; e += 64) U[e] = 0.0;
  __syncthreads();
  for (int i = lane; i < QD; i += 64)
    for (int f = 0; f < F; ++f) U[f * KR + DF.ia[i] * DIM + DF.ca[i]] = DF.va[i] * Y[f * QD + i];
  __syncthreads();
  for (int c = 1; c < DIM; ++c) {
    for (int i = lane; i < QD; i += 64)
      if (DF.ca[i] == c && DF.ib[i] >= 0)
        for (int f = 0; f < F; ++f) U[f * KR + DF.ib[i] * DIM + DF.cb[i]] += DF.vb[i] * Y[f * QD + i];
    __syncthreads();
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
            for (int q = 0; q < Q; ++q) acc += p[q] * U[f * KR + q * DIM + c];
            a.weights[(int64_t)F * DIM * r.base + ((int64_t)f * r.N + j) * DIM + c] = r.w[i] * acc;
          }
      }
    }
  }
  if (lane == 0 && a.ok_status >= 0) a.status[t] = (uint8_t)a.ok_status;
  __syncthreads();
}


// Persistent kernel over the queue aux_list[0 .. *count) (any row count).
template <int DIM, int ORDER, int RPL>
__global__ __launch_bounds__(64) void k_qr_kmat(StencilArgs a, const int *list, const int *count, int *cursor) {
  __shared__ __align__(16) double lds[qr_kmat_lds_doubles<DIM, ORDER>()];
  const RowKinds rk = row_kinds(DIM, 1, a.mask);
  const int n = readfirstlane_i(*count);
  for (;;) {
    int i = 0;
    if (lane_id() == 0) i = atomicAdd(cursor, 1);
    i = __builtin_amdgcn_readfirstlane(i);
    if (i >= n) break;
    const int t = readfirstlane_i(list[i]);
    qr_divfree_kmat_target<DIM, ORDER, RPL>(a, rk, t, lds);
  }
}

}  // namespace gmls
