#pragma once
// stencil_fp64.hpp -- FP64 stencils by Householder QR, one wavefront per target
// (scalar basis; the divergence-free basis is in stencil_fp64_div.hpp and the
// kernel that serves both in qr_kernel.hpp).
//
// For target T with N neighbours the weighted sample matrix M = sqrt(W) P
// (N x Q, Section 2.1: P, W and the scaled basis) lives in registers, row j
// on lane j % 64, slot j / 64.  Householder QR (Golub & Van Loan, Alg. 5.2.1)
// reduces M to R with one batched wave all-reduce per column.  Since
// P^T W P = R^T R, the weights of a functional lambda (Section 2.5) are
//   y = R^{-1} R^{-T} lambda,   alpha_j = w_j p(s_j) . y
// which is alpha = W P (P^T W P)^{-1} lambda (Section 2.1, normal equations)
// evaluated through R: the semi-normal-equations form of the minimum
// W^{-1}-norm solution of P^T alpha = lambda, stable for that problem when R
// comes from a backward-stable QR (Paige 1979; Bjorck 1987).
#include <float.h>
#include <math.h>

#include "basis.hpp"
#include "gmls_internal.hpp"

namespace gmls {

constexpr double kRankTol = 1e-12;  // QR rank test: min|R_kk| <= tol * max|R_kk|

// Rows of one target held by a wavefront: rows first + lane + 64 i of the
// target's neighbour row (a chunk of 64 RPL rows; rows with more neighbours
// are taken chunk by chunk).
template <int DIM, int RPL>
struct Rows {
  double s[RPL][DIM];
  double w[RPL];
  int N;
  int first;  // the chunk held (-1: none)
  int64_t base;
};

// scaled offset and kernel weight of row j of target t (zero for j >= N)
template <int DIM>
__device__ __forceinline__ void row_s_w(const StencilArgs &a, int64_t base, int j, int N, const double *xt,
                                        double ie, double *s, double &w) {
  double rr = 0.0;
  if (j < N) {
    const int c = a.col[base + j];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      s[d] = (a.coords[(int64_t)c * a.cstride + d] - xt[d]) * ie;
      rr += s[d] * s[d];
    }
    const double rad = sqrt(rr);
    w = rad < 1.0 ? int_pow(1.0 - rad, a.p) : 0.0;
  } else {
#pragma unroll
    for (int d = 0; d < DIM; ++d) s[d] = 0.0;
    w = 0.0;
  }
}

template <int DIM, int RPL>
__device__ __forceinline__ void load_rows(const StencilArgs &a, int t, Rows<DIM, RPL> &r, int lane,
                                          int first = 0) {
  r.base = uniform_i64(a.row_ptr[t]);
  r.N = readfirstlane_i((int)(a.row_ptr[t + 1] - r.base));
  r.first = first;
  const double e = uniform_d(a.eps[t]);
  const double ie = 1.0 / e;
  double xt[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xt[d] = uniform_d(a.targets[(int64_t)t * DIM + d]);
#pragma unroll
  for (int i = 0; i < RPL; ++i) row_s_w<DIM>(a, r.base, first + lane + 64 * i, r.N, xt, ie, r.s[i], r.w[i]);
}

// LDS the batched column sums of wave_householder take: a 16 x 66 tile of
// partial values (value q of lane L at q * 66 + L; 66 keeps each lane's
// reads 16-byte aligned) and 16 results.  The array must be 16-byte aligned.
constexpr int kSumStride = 66;
constexpr int kSumBufDoubles = 16 * kSumStride + 16;

// v[0..ch) (ch <= 16) summed over the wavefront and multiplied by scale,
// bitwise the same in every lane, through LDS: every lane stores its partial
// values, lane j + 16 g adds value j over the 16 lanes 16 g .. 16 g + 15
// (contiguous, read 2 at a time; pairwise, a fixed order), the four groups
// are combined by lane swaps (both lanes of a pair add the same operands),
// lane j scales value j, and every lane takes the results: BCAST_LDS, from
// LDS, 2 at a time (broadcast reads, into vector registers), else by lane
// reads (into scalar registers, for kernels short of vector registers).
// Up to 8 values take half the reads (below).  About 25 vector and 33 LDS
// instructions for 16 values (BCAST_LDS), where a full wave sum per value
// (DPP within the rows, then across them) costs about 18 vector
// instructions each.  buf: kSumBufDoubles of LDS owned by this wavefront;
// all 64 lanes active.
template <bool BCAST_LDS>
__device__ __forceinline__ void wave_sum16_lds(double (&v)[16], int ch, double *buf, int lane, double scale) {
  const int j = lane & 15, g = lane >> 4;
  const double2 *part = reinterpret_cast<const double2 *>(buf + j * kSumStride + 16 * g);
  double *res = buf + 16 * kSumStride;
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (q < ch) buf[q * kSumStride + lane] = v[q];
  wave_lds_sync();
  // lanes j >= ch add stale values; their results are never read
  double sum;
  if (ch <= 8) {
    // at most 8 values: lane j + 8 s (j < 8) adds value j over the 8 lanes
    // 8 s .. 8 s + 7 (half the reads), and the lane 8 apart in its row
    // (the same value, the other half of the row's sources) is added by a
    // rotation of the row by 8, which pairs the two lanes both ways
    const double2 *part8 = reinterpret_cast<const double2 *>(buf + (lane & 7) * kSumStride + 8 * (lane >> 3));
    double p[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double2 t = part8[i];
      p[2 * i] = t.x;
      p[2 * i + 1] = t.y;
    }
#pragma unroll
    for (int h = 4; h >= 1; h >>= 1)
#pragma unroll
      for (int i = 0; i < h; ++i) p[i] = p[i] + p[i + h];
    const double r = p[0] + dpp_d<0x128>(p[0]);  // row_ror:8
    sum = swap_pair_sum<32>(swap_pair_sum<16>(r)) * scale;
  } else {
    double p[16];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double2 t = part[i];
      p[2 * i] = t.x;
      p[2 * i + 1] = t.y;
    }
#pragma unroll
    for (int h = 8; h >= 1; h >>= 1)
#pragma unroll
      for (int i = 0; i < h; ++i) p[i] = p[i] + p[i + h];
    sum = swap_pair_sum<32>(swap_pair_sum<16>(p[0])) * scale;
  }
  if constexpr (BCAST_LDS) {
    if (lane < 16) res[lane] = sum;  // ch <= 8: lanes 0..7 hold values 0..7
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 16; q += 2) {
      if (q < ch) {
        const double2 t = reinterpret_cast<const double2 *>(res)[q / 2];
        v[q] = t.x;
        v[q + 1] = t.y;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (q < ch) v[q] = readlane_d(sum, q);  // ch <= 8: lane q holds value q as well
  }
  wave_lds_sync();  // the next call (or the caller) may rewrite buf
}

// One Householder step of wave_householder: column K of M is reduced and the
// reflector applied to columns K+1..Q-1, then the next step (a template
// recursion, so that every column index is a constant and M stays in
// registers).  With v = x - beta e_K (x: column K on rows >= K, beta = -+|x|)
// column l takes a_l -= (2 v.a_l / v.v) v; v.a_l equals x.a_l - beta R_Kl.
template <int K, int Q, int RPL, bool VIA_LDS>
__device__ __forceinline__ void householder_step(double (&M)[RPL][Q], double &rdiag, int lane, double *buf) {
  const double x0 = lane >= K ? M[0][K] : 0.0;
  if constexpr (VIA_LDS) {
    // |x|^2 first (one wave sum), then the products v.a_l of all later
    // columns with v itself, reduced together and scaled by 2 / v.v in LDS
    double ss = x0 * x0;
#pragma unroll
    for (int i = 1; i < RPL; ++i) ss = fma(M[i][K], M[i][K], ss);
    const double sigma = uniform_d(wave_sum_uniform(ss));  // the same in every lane; a scalar branch
    const double xk = readlane_d(M[0][K], K);
    if (sigma > 0.0) {
      // |x| and 2 / v.v = 1 / (|x|^2 + |x_K| |x|) from the hardware
      // reciprocal square root and reciprocal, each refined by Newton steps
      // (quadratic convergence: two steps take an estimate good to 1e-4 to
      // a few ulp), in place of the correctly rounded sqrt and division
      // sequences on the step's dependent chain
      const double y0 = __builtin_amdgcn_rsq(sigma);
      const double y1 = fma(y0, fma(-(0.5 * sigma) * y0, y0, 0.5), y0);
      const double n0 = sigma * y1;
      const double norm = fma(fma(-n0, n0, sigma), 0.5 * y1, n0);
      const double beta = xk >= 0.0 ? -norm : norm;
      const double d = fma(fabs(xk), norm, sigma);
      const double r0 = __builtin_amdgcn_rcp(d);
      const double r1 = fma(r0, fma(-d, r0, 1.0), r0);
      const double two_inv_vtv = fma(r1, fma(-d, r1, 1.0), r1);
      const double v0 = lane > K ? M[0][K] : (lane == K ? xk - beta : 0.0);
      // 16 columns at a time: their products, sums and updates (a chunk's
      // values are all that is held beyond M)
#pragma unroll
      for (int c0 = K + 1; c0 < Q; c0 += 16) {
        const int ch = Q - c0 < 16 ? Q - c0 : 16;
        double coef[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          if (q < ch) {
            double t = v0 * M[0][c0 + q];
#pragma unroll
            for (int i = 1; i < RPL; ++i) t = fma(M[i][K], M[i][c0 + q], t);
            coef[q] = t;
          }
        }
        wave_sum16_lds<(RPL * Q <= 80)>(coef, ch, buf, lane, two_inv_vtv);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          if (q < ch) {
            M[0][c0 + q] -= coef[q] * v0;
#pragma unroll
            for (int i = 1; i < RPL; ++i) M[i][c0 + q] -= coef[q] * M[i][K];
          }
        }
      }
      if (lane == K) M[0][K] = beta;
    } else if (lane == K) {
      M[0][K] = 0.0;
    }
  } else {
    // every x.a_l by its own wave sum (no LDS)
    double dots[Q];
#pragma unroll
    for (int l = K; l < Q; ++l) {
      double v = x0 * (lane >= K ? M[0][l] : 0.0);
#pragma unroll
      for (int i = 1; i < RPL; ++i) v += M[i][K] * M[i][l];
      dots[l] = wave_sum_uniform(v);
    }
    const double sigma = uniform_d(dots[K]);  // the same in every lane; a scalar branch
    const double xk = readlane_d(M[0][K], K);
    if (sigma > 0.0) {
      const double norm = sqrt(sigma);
      const double beta = xk >= 0.0 ? -norm : norm;
      const double inv_vtv = 1.0 / (2.0 * beta * (beta - xk));
      const double v0 = lane > K ? M[0][K] : (lane == K ? xk - beta : 0.0);
#pragma unroll
      for (int l = K + 1; l < Q; ++l) {
        const double rkl = readlane_d(M[0][l], K);
        const double coef = 2.0 * (dots[l] - beta * rkl) * inv_vtv;
        M[0][l] -= coef * v0;
#pragma unroll
        for (int i = 1; i < RPL; ++i) M[i][l] -= coef * M[i][K];
      }
      if (lane == K) M[0][K] = beta;
    } else if (lane == K) {
      M[0][K] = 0.0;
    }
  }
  if (lane == K) rdiag = M[0][K];
  // finish this column's updates here: left alone, the compiler defers the
  // updates of later columns to where they are next read, keeping every
  // reflector live (registers grow with the column count)
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int l = K + 1; l < Q; ++l) asm volatile("" : "+v"(M[i][l]));
  if constexpr (K + 1 < Q) householder_step<K + 1, Q, RPL, VIA_LDS>(M, rdiag, lane, buf);
}

// Householder QR of the register-resident M (rows across lanes).  On return
// lane k (k < Q) holds row k of R in M[0][k..Q-1] and rdiag = R_kk.  The
// reflector's products with the later columns of each step are summed over
// the wavefront together, through `buf` (kSumBufDoubles of LDS;
// wave_sum16_lds), or one by one by DPP and lane swaps when VIA_LDS is false
// (no LDS; buf unused); all 64 lanes take part.
template <int Q, int RPL, bool VIA_LDS = true>
__device__ __forceinline__ void wave_householder(double (&M)[RPL][Q], double &rdiag, int lane, double *buf) {
  rdiag = 0.0;
  householder_step<0, Q, RPL, VIA_LDS>(M, rdiag, lane, buf);
}

// Solve R^T z = b then R y = z for a Q x Q upper-triangular R stored
// row-major (Rm) and column-major (Rt) in LDS; lane a < Q holds b_a on entry
// and y_a on return.  rdiag is R_aa on lane a.
template <int Q>
__device__ __forceinline__ double tri_solve_rtr(const double *Rm, const double *Rt, double b, double rdiag,
                                                int lane) {
  // 1/R_aa once per lane, so that each of the 2Q dependent steps multiplies
  // instead of dividing
  const double rinv = lane < Q ? 1.0 / rdiag : 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const double zk = readlane_d(b, k) * readlane_d(rinv, k);
    if (lane == k) b = zk;
    if (lane > k && lane < Q) b -= Rm[k * Q + lane] * zk;
  }
#pragma unroll
  for (int k = Q - 1; k >= 0; --k) {
    const double yk = readlane_d(b, k) * readlane_d(rinv, k);
    if (lane == k) b = yk;
    if (lane < k) b -= Rt[k * Q + lane] * yk;
  }
  return b;
}

// tri_solve_rtr for NR right-hand sides at once (b[r] on lane a: entry a of
// right-hand side r): the same operations for each, interleaved, so that the
// 2Q dependent steps are walked once and each step's row of R is read once.
template <int Q, int NR>
__device__ __forceinline__ void tri_solve_rtr_multi(const double *Rm, const double *Rt, double (&b)[NR],
                                                    double rdiag, int lane) {
  const double rinv = lane < Q ? 1.0 / rdiag : 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const double ik = readlane_d(rinv, k);
    const double rm = Rm[k * Q + (lane < Q ? lane : 0)];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double zk = readlane_d(b[r], k) * ik;
      if (lane == k) b[r] = zk;
      if (lane > k && lane < Q) b[r] -= rm * zk;
    }
  }
#pragma unroll
  for (int k = Q - 1; k >= 0; --k) {
    const double ik = readlane_d(rinv, k);
    const double rt = Rt[k * Q + (lane < Q ? lane : 0)];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double yk = readlane_d(b[r], k) * ik;
      if (lane == k) b[r] = yk;
      if (lane < k) b[r] -= rt * yk;
    }
  }
}

// The target's rows, its weighted sample matrix and the Householder factor:
// on return lane k < Q holds row k of R in M[0][k..Q-1] and rdiag = R_kk.
// A row of more than 64 RPL neighbours is factored chunk by chunk (tall-skinny
// QR): R of the rows so far stays on lanes 0..Q-1 of slot 0, with its
// strictly lower part cleared, and the next 64 RPL - Q rows fill the other
// positions; the Householder QR of that stack is R of all the rows so far
// (the same R up to the signs of its rows, which y = R^-1 R^-T lambda does not
// see).  r then holds no chunk (first = -1): the solves reload the rows.
template <int DIM, int ORDER, int RPL, int SKIP = 0>
__device__ __forceinline__ void qr_factor(const StencilArgs &a, int t, Rows<DIM, RPL> &r,
                                          double (&M)[RPL][num_mono(DIM, ORDER) - SKIP], double &rdiag,
                                          int lane, double *buf) {
  constexpr int QF = num_mono(DIM, ORDER);
  constexpr int Q = QF - SKIP;
  load_rows<DIM, RPL>(a, t, r, lane);
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    double p[QF];
    scaled_basis<DIM, ORDER, double>(r.s[i], p);
    const double sw = sqrt(r.w[i]);
#pragma unroll
    for (int q = 0; q < Q; ++q) M[i][q] = sw * p[q + SKIP];
  }
  wave_householder<Q, RPL>(M, rdiag, lane, buf);
  if (r.N > 64 * RPL) {
    static_assert(Q < 64, "R and the next rows share the wavefront");
    constexpr int CAP = 64 * RPL - Q;  // rows added per step
    const double ie = 1.0 / uniform_d(a.eps[t]);
    double xt[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) xt[d] = uniform_d(a.targets[(int64_t)t * DIM + d]);
    for (int c = 64 * RPL; c < r.N; c += CAP) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        if (i == 0 && lane < Q) {  // row `lane` of R: clear the reflector left below its diagonal
#pragma unroll
          for (int l = 0; l < Q; ++l) M[0][l] = l < lane ? 0.0 : M[0][l];
          continue;
        }
        const int q = i == 0 ? lane - Q : (64 - Q) + 64 * (i - 1) + lane;
        double s[DIM], w;
        row_s_w<DIM>(a, r.base, c + q, r.N, xt, ie, s, w);
        double p[QF];
        scaled_basis<DIM, ORDER, double>(s, p);
        const double sw = sqrt(w);
#pragma unroll
        for (int l = 0; l < Q; ++l) M[i][l] = sw * p[l + SKIP];
      }
      wave_householder<Q, RPL>(M, rdiag, lane, buf);
    }
    r.first = -1;
  }
}

// SKIP = 1 drops the constant monomial: the staggered scheme (Section 2.4).
// Its sample of the vector basis phi_(a,k) = e_k p_a along the segment
// x_T -> x_j is xi = eps s_k p_a(s) / (|a| + 1); the span of those columns is
// that of the scalar monomials of degree 1..m+1 evaluated at s (by Euler's
// relation every homogeneous h of degree n+1 is grad(h) . s / (n+1)), and
// the gradient and divergence of the fit at x_T are the first and second
// derivatives of the scalar fit there.  The data are p_j - p(x_T), so the
// target's own value carries the weight -sum_j alpha_j (into hweights).
//
// The weights from the factor (lane k < Q holds row k of R in Rrow[k..Q-1],
// rdiag = R_kk): rank test, R to LDS, the functionals' solves and the rows.
template <int DIM, int ORDER, int RPL, int SKIP = 0>
__device__ __forceinline__ void qr_scalar_solve(const StencilArgs &a, const RowKinds &rk, int t,
                                                Rows<DIM, RPL> &r, const double (&Rrow)[num_mono(DIM, ORDER) - SKIP],
                                                double rdiag, double *lds) {
  constexpr Mono<DIM, ORDER> MO{};
  constexpr int QF = MO.N;       // monomials of degree <= ORDER
  constexpr int Q = QF - SKIP;   // columns of the sample matrix
  const int lane = lane_id();
  const double amax = uniform_d(wave_max(lane < Q ? fabs(rdiag) : 0.0));
  const double amin = uniform_d(wave_min(lane < Q ? fabs(rdiag) : DBL_MAX));
  double *Rm = lds, *Rt = lds + Q * Q, *Y = lds + 2 * Q * Q;
  const int F = a.F;
  const int rank_def = readfirstlane_i(!(amin > kRankTol * amax) ? 1 : 0);
  if (rank_def) {
    for (int j = lane; j < r.N; j += 64)
      for (int f = 0; f < F; ++f) a.weights[(int64_t)F * r.base + (int64_t)f * r.N + j] = NAN;
    if (a.hweights && lane < F) a.hweights[(int64_t)t * F + lane] = NAN;
    if (lane == 0) a.status[t] = GMLS_TARGET_RANK_DEFICIENT;
    __syncthreads();
    return;
  }
  if (lane < Q) {
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      const double v = l >= lane ? Rrow[l] : 0.0;
      Rm[lane * Q + l] = v;
      Rt[l * Q + lane] = v;
    }
  }
  __syncthreads();
  const double ie = 1.0 / uniform_d(a.eps[t]);
  // Neumann constraint (Section 2.3): minimise the weighted residual subject
  // to F^T c = h, F = n . grad p(x_T) (only the linear monomials, index
  // 1 + d, carry 1/eps).  With y = A^-1 lambda and z = A^-1 F the solution of
  // the bordered system gives lambda^T c = (W P (y - g z))^T u + g h with
  // g = F^T y / F^T z; lane q holds component q of every vector.
  double Fq = 0.0, zc = 0.0, sF = 0.0;
  bool con = false;
  if (SKIP == 0 && a.normals) {
    for (int d = 0; d < DIM; ++d) {
      const double nd = uniform_d(a.normals[(int64_t)t * DIM + d]);
      if (lane == 1 + d) Fq = nd * ie;
      con = con || nd != 0.0;
    }
    if (con) {
      zc = tri_solve_rtr<Q>(Rm, Rt, Fq, rdiag, lane);
      sF = uniform_d(wave_sum(lane < Q ? Fq * zc : 0.0));
    }
  }
  int f = 0;
  if (!con) {
    // two to four functionals at once: one walk of the dependent steps
    for (; f + 1 < F; f += 4) {
      double bb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        bb[u] = 0.0;
        if (f + u < F) {
#pragma unroll
          for (int q = 0; q < Q; ++q)
            if (lane == q) bb[u] = scalar_lambda<DIM, ORDER>(rk.kind[f + u], q + SKIP, ie);
        }
      }
      tri_solve_rtr_multi<Q, 4>(Rm, Rt, bb, rdiag, lane);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (f + u < F) {
          if (SKIP == 0 && a.hweights && lane == 0) a.hweights[(int64_t)t * F + f + u] = 0.0;
          if (lane < Q) Y[(f + u) * Q + lane] = bb[u];
        }
      }
    }
  }
  for (; f < F; ++f) {
    double b = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (lane == q) b = scalar_lambda<DIM, ORDER>(rk.kind[f], q + SKIP, ie);
    double y = tri_solve_rtr<Q>(Rm, Rt, b, rdiag, lane);
    if (con) {
      const double g = uniform_d(wave_sum(lane < Q ? Fq * y : 0.0)) / sF;
      y -= g * zc;
      if (lane == 0) a.hweights[(int64_t)t * F + f] = g;
    } else if (SKIP == 0 && a.hweights && lane == 0) {
      a.hweights[(int64_t)t * F + f] = 0.0;
    }
    if (lane < Q) Y[f * Q + lane] = y;
  }
  __syncthreads();
  double rsum[4] = {0.0, 0.0, 0.0, 0.0};  // staggered: F <= 4 (gradient, Laplacian)
  for (int c = 0; c < r.N; c += 64 * RPL) {  // one pass unless the row is longer than 64 RPL
    if (r.first != c) load_rows<DIM, RPL>(a, t, r, lane, c);
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int j = c + lane + 64 * i;
      if (j < r.N) {
        double p[QF];
        scaled_basis<DIM, ORDER, double>(r.s[i], p);
        for (int f = 0; f < F; ++f) {
          double acc = 0.0;
#pragma unroll
          for (int q = 0; q < Q; ++q) acc += p[q + SKIP] * Y[f * Q + q];
          const double wv = r.w[i] * acc;
          a.weights[(int64_t)F * r.base + (int64_t)f * r.N + j] = wv;
          if constexpr (SKIP != 0) {
#pragma unroll
            for (int g = 0; g < 4; ++g)
              if (g == f) rsum[g] += wv;
          }
        }
      }
    }
  }
  if constexpr (SKIP != 0) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const double tot = wave_sum(rsum[f]);
      if (f < F && lane == 0) a.hweights[(int64_t)t * F + f] = -tot;
    }
  }
  if (lane == 0 && a.ok_status >= 0) a.status[t] = (uint8_t)a.ok_status;
  __syncthreads();
}

template <int DIM, int ORDER, int RPL, int SKIP = 0>
__device__ __forceinline__ void qr_scalar_target(const StencilArgs &a, const RowKinds &rk, int t, double *lds) {
  constexpr int Q = num_mono(DIM, ORDER) - SKIP;
  Rows<DIM, RPL> r;
  double M[RPL][Q];
  double rdiag;
  qr_factor<DIM, ORDER, RPL, SKIP>(a, t, r, M, rdiag, lane_id(), lds);  // lds is free until the solves
  qr_scalar_solve<DIM, ORDER, RPL, SKIP>(a, rk, t, r, M[0], rdiag, lds);
}

}  // namespace gmls
