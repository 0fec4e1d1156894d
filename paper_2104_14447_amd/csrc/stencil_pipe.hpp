// stencil_pipe.hpp -- mixed-precision stencils as a three-kernel pipeline for
// small scalar bases (Q <= 20: 3D order <= 3, 2D order <= 4).
//
// The stencil of a functional lambda is alpha = W P y with (P^T W P) y = lambda
// (Section 2.1, normal equations; Section 2.5, functionals on the basis).
//
//  A. moments (a group of G lanes per target, rows spread over the group):
//     mu_g = sum_j w_j s_j^g for |g| <= 2m in FP64, reduce-scattered over the
//     group and stored to HBM, moment-major [g][slot];
//  B. solve (one thread per target, the whole system in registers):
//     A64_ab = mu_(a+b)/(a! b!) is the Gram; its Jacobi-equilibrated FP32
//     copy is factored by a fully unrolled packed Cholesky, its 1-norm
//     condition number is estimated (Hager's estimator, three solves), then
//     y = D A~^-1 D lambda is refined with FP64 residuals r = lambda - A64 y
//     (FP32 correction, FP64 accumulation) until the predicted error
//     rho*|dy| <= tol*|y|; y is stored to HBM, [f][a][slot];
//  C. weights (a group of G lanes per target): alpha_j = w_j p(s_j) . y in
//     FP64, the rows gathered again.
// Targets that break down, exceed the condition threshold or do not converge
// are queued for the FP64 QR fallback.  Every lane of kernel B runs the same
// instruction stream (no row-count divergence), and no lane is idle.
#pragma once

#include <float.h>
#include <limits.h>
#include <math.h>

#include "basis.hpp"
#include "gmls_internal.hpp"
#include "stencil_mixed64.hpp"

namespace gmls {

// Per-target record of one pipeline chunk, in list-slot order, so that the
// three kernels read what they need about a target with one coalesced load
// instead of a chain of scattered ones (list -> row_ptr, eps, coordinates).
struct PipeRec {
  int64_t base;  // row_ptr[t]
  int n;         // row count
  int t;         // target index
  double ie;     // 1 / eps_t
  double x[3];   // target coordinates
  int ok;        // written by the solve: 1 = weights to be formed here
  int pad;
  double pad2;
};
static_assert(sizeof(PipeRec) == kPipeRecBytes, "record size");

// List slots a launch covers: bin `bin` (0: bins 1..4 together) clipped to
// the window [win_lo, win_hi); win_lo < 0 opens the window at the first slot
// of bin 1.  c0 is the window's first slot (records and buffers are indexed
// from it).  The bounds come from the device bin table, so a launch needs no
// host copy of it.
struct SlotRange {
  int first, last, c0;
};

__device__ __forceinline__ SlotRange slot_range(const BinMeta *meta, int bin, int win_lo, int win_hi) {
  const int c0 = win_lo >= 0 ? win_lo : meta->offset[1];
  int lo, hi;
  if (bin > 0) {
    lo = meta->offset[bin];
    hi = lo + meta->count[bin];
  } else {
    lo = meta->offset[1];
    hi = meta->offset[kNumBins - 1] + meta->count[kNumBins - 1];
  }
  lo = lo > c0 ? lo : c0;
  hi = hi < win_hi ? hi : win_hi;
  return {readfirstlane_i(lo), readfirstlane_i(hi), readfirstlane_i(c0)};
}

template <int DIM>
__global__ __launch_bounds__(256) void k_pipe_prep(StencilArgs a, const int *list, const BinMeta *meta, int win_lo,
                                                   int win_hi, PipeRec *rec) {
  const SlotRange R = slot_range(meta, 0, win_lo, win_hi);
  const int first = R.first, last = R.last;
  for (int i = first + blockIdx.x * blockDim.x + threadIdx.x; i < last; i += gridDim.x * blockDim.x) {
    const int t = list[i];
    PipeRec r;
    r.base = a.row_ptr[t];
    r.n = (int)(a.row_ptr[t + 1] - r.base);
    r.t = t;
    r.ie = 1.0 / a.eps[t];
    for (int d = 0; d < 3; ++d) r.x[d] = d < DIM ? a.targets[(int64_t)t * DIM + d] : 0.0;
    r.ok = 0;
    r.pad = 0;
    rec[i - R.c0] = r;
  }
}

// ---------------------------------------------------------------------------
// A. moments
// ---------------------------------------------------------------------------
// Rows j = lg + G*r (r < RPL) of a target, gathered without branches: rows
// past N re-read row N-1 and get weight 0, so all column indices, then all
// coordinates, are requested together (two memory round trips per target
// instead of two per row).
template <int DIM, int RPL, int G>
__device__ __forceinline__ void gather_rows(const StencilArgs &a, int64_t base, int N, int lg,
                                            double (&xs)[RPL][DIM]) {
  int c[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int j = lg + G * r;
    c[r] = a.col[base + (j < N ? j : N - 1)];
  }
#pragma unroll
  for (int r = 0; r < RPL; ++r)
#pragma unroll
    for (int d = 0; d < DIM; ++d) xs[r][d] = a.coords[(int64_t)c[r] * a.cstride + d];
}

// scaled offset s = (x_j - x_T)/eps and kernel weight (1 - |s|)^p (0 outside
// the support, and 0 when `live` is false)
template <int DIM>
__device__ __forceinline__ double row_sw(const double *xj, const double *xt, double ie, int p, bool live,
                                         double *s) {
  double rr = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    s[d] = (xj[d] - xt[d]) * ie;
    rr += s[d] * s[d];
  }
  // |s| from the hardware reciprocal square root and one Newton step for the
  // square root (relative error about the square of the estimate's, far
  // below the mixed path's tolerance), in place of the correctly rounded
  // sqrt sequence; the support test uses |s|^2 itself
  const double y = __builtin_amdgcn_rsq(rr);
  const double r0 = rr * y;
  const double rad = rr > 0.0 ? fma(fma(-r0, r0, rr), 0.5 * y, r0) : 0.0;
  return (live && rr < 1.0) ? int_pow(1.0 - rad, p) : 0.0;
}

// Trip count of the chunk loop over a row: one pass of G * RPL rows, or for
// the long bin (LOOP) enough passes for the longest row of the wavefront's
// targets (the same for every lane: the loop holds no divergent barrier).
template <bool LOOP, int CH>
__device__ __forceinline__ int chunk_end(int N) {
  if constexpr (!LOOP) {
    return 1;
  } else {
    int m = N;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = max(m, __shfl_xor(m, o));
    return readfirstlane_i(m);
  }
}

// `t` is a target of the bin even for an invalid group (whose sums are not
// stored), so that every gathered row exists.  LOOP: rows in chunks of
// G * RPL (the long bin), the partial sums carried over the chunks.
template <int DIM, int ORDER, int G, int RPL, bool LOOP = false>
__device__ void pipe_moments_target(const StencilArgs &a, const PipeRec &rc, bool valid, int slot, int lg,
                                    double *mom) {
  constexpr int NM = num_mono(DIM, 2 * ORDER);
  constexpr int RS = 32;  // moments per LDS reduction round
  constexpr int RW = 66;  // row of the reduction tile: one moment, 64 lanes (+2: rows start in other banks)
  __shared__ __align__(16) double red[RS * RW];
  const int64_t base = rc.base;
  const int N = rc.n;
  const double ie = rc.ie;
  double xt[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xt[d] = rc.x[d];
  double mu[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) mu[m] = 0.0;
  constexpr MomentSplit<DIM, ORDER> MS{};
  const int cend = chunk_end<LOOP, G * RPL>(N);
  for (int c0 = 0; c0 < cend; c0 += G * RPL) {
    const int nrem = N - c0;  // rows of this chunk and after (may be <= 0 in a long loop)
    double xs[RPL][DIM];
    gather_rows<DIM, RPL, G>(a, base + (nrem > 0 ? c0 : 0), nrem > 0 ? nrem : N, lg, xs);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      double s[DIM];
      const double w = row_sw<DIM>(xs[r], xt, ie, a.p, lg + G * r < nrem, s);
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
  // the sums are complete here: without this the compiler sinks each
  // moment's FMA chain into the reduction round that stores it and keeps
  // every row's products live until then
#pragma unroll
  for (int m = 0; m < NM; ++m) asm volatile("" : "+v"(mu[m]));
  // sum the G lanes' partial moments through LDS, RS moments per round:
  // every lane writes its partials (moment q of lane L at q * RW + L), then
  // lane lg of the group adds moment lg + G*k (< RS) over the group's lanes,
  // in lane order, reading them two at a time (the group's lanes are
  // contiguous in a moment's row), and stores it
  const int lane = lane_id(), grp0 = lane - lg;
#pragma unroll
  for (int r0 = 0; r0 < NM; r0 += RS) {
#pragma unroll
    for (int q = 0; q < RS; ++q) red[q * RW + lane] = r0 + q < NM ? mu[r0 + q] : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < (RS + G - 1) / G; ++k) {
      const int q = lg + G * k;
      if (q < RS) {
        const double2 *row = reinterpret_cast<const double2 *>(red + q * RW + grp0);
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < G / 2; ++l) {
          const double2 t = row[l];
          acc += t.x;
          acc += t.y;
        }
        if (valid && r0 + q < NM) mom[(int64_t)slot * NM + r0 + q] = acc;
      }
    }
    __syncthreads();
  }
}

// Targets list[first .. last) of one row-count bin; moment g of the target
// in list slot i goes to mom[(i - c0) * NM + g] (target-major, so that a
// group writes its target's moments contiguously).
template <int DIM, int ORDER, int G, int RPL, bool LOOP = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_pipe_moments(
    StencilArgs a, const PipeRec *rec, const BinMeta *meta, int bin, int win_lo, int win_hi, double *mom) {
  const SlotRange R = slot_range(meta, bin, win_lo, win_hi);
  const int first = R.first, last = R.last, c0 = R.c0;
  constexpr int TPW = 64 / G;
  const int lane = lane_id();
  const int grp = lane / G, lg = lane % G;
  for (int i0 = first + xcd_block() * TPW; i0 < last; i0 += gridDim.x * TPW) {
    const int i = i0 + grp;
    const bool valid = i < last;
    const PipeRec rc = rec[(valid ? i : first) - c0];
    pipe_moments_target<DIM, ORDER, G, RPL, LOOP>(a, rc, valid, i - c0, lg, mom);
  }
}

// ---------------------------------------------------------------------------
// B. solve, one thread per target
// ---------------------------------------------------------------------------
template <int Q>
struct Packed {
  static constexpr int n = Q * (Q + 1) / 2;
  static constexpr int at(int i, int k) { return i * (i + 1) / 2 + k; }  // k <= i
};

// x <- (L L^T)^-1 x for a packed lower-triangular L whose diagonal slots hold
// 1/L_jj (registers, fully unrolled)
template <int Q>
__device__ __forceinline__ void packed_solve(const float (&L)[Q * (Q + 1) / 2], float (&x)[Q]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    float v = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= L[Packed<Q>::at(i, k)] * x[k];
    x[i] = v * L[Packed<Q>::at(i, i)];
  }
#pragma unroll
  for (int i = Q - 1; i >= 0; --i) {
    float v = x[i];
#pragma unroll
    for (int k = i + 1; k < Q; ++k) v -= L[Packed<Q>::at(k, i)] * x[k];
    x[i] = v * L[Packed<Q>::at(i, i)];
  }
}

// All (a, b) pairs of the Q x Q moment Gram ordered by the moment index of
// a + b, so that the residual streams each moment once.
template <int DIM, int ORDER>
struct MomentPairs {
  static constexpr int Q = num_mono(DIM, ORDER);
  static constexpr int NM = num_mono(DIM, 2 * ORDER);
  static constexpr int P = Q * Q;
  int m[P], a[P], b[P];
  constexpr MomentPairs() : m{}, a{}, b{} {
    SumIndex<DIM, ORDER> S{};
    int p = 0;
    for (int g = 0; g < NM; ++g)
      for (int i = 0; i < Q; ++i)
        for (int k = 0; k < Q; ++k)
          if (S.idx[i][k] == g) {
            m[p] = g;
            a[p] = i;
            b[p] = k;
            ++p;
          }
  }
};

// SKIP = 1 (staggered stencils): the constant monomial is not a column, so
// the Gram is the trailing (Q-1) x (Q-1) block of the moment Gram and the
// functionals act on monomials 1..Q-1.
template <int DIM, int ORDER, int SKIP = 0>
__global__ __launch_bounds__(64) void k_pipe_solve(StencilArgs a, PipeRec *rec, int win_lo, int win_hi,
                                                   const double *mom, double *yout, int *fb_list, BinMeta *meta,
                                                   Stats *stats, Options opt) {
  constexpr int Q = num_mono(DIM, ORDER) - SKIP;
  constexpr int NP = Q * (Q + 1) / 2;
  constexpr InvFact64<DIM, ORDER> IF{};
  constexpr SumIndex<DIM, ORDER> SI{};
  constexpr MomentPairs<DIM, ORDER> MP{};
  constexpr int NM = MomentPairs<DIM, ORDER>::NM;
  // thread-private LDS columns (lane l uses [.][l] only)
  __shared__ double mls[NM][64];  // FP64 moments of this thread's target
  __shared__ double ybuf[Q][64];  // this thread's solution
  const int lane = lane_id();
  const RowKinds rk = row_kinds(DIM, 0, a.mask);
  const int F = a.F;
  const SlotRange R = slot_range(meta, 0, win_lo, win_hi);
  const int first = R.first, last = R.last, c0 = R.c0;
  for (int slot = first + xcd_block() * 64 + lane; slot - lane < last; slot += gridDim.x * 64) {
    const bool valid = slot < last;
    const int sl = valid ? slot : first;
    const int t = rec[sl - c0].t;
    const double ie = rec[sl - c0].ie;
    const int64_t loc = sl - c0;
    // stage this thread's moments into its LDS column; the wave's 84 loads
    // walk one contiguous block of 64*NM doubles, so lines are reused from L1
    if (valid) {
#pragma unroll
      for (int m = 0; m < NM; ++m) mls[m][lane] = mom[loc * NM + m];
    }
#define GMLS_MU(g, off) mls[(g)][lane + (off)]
    // equilibration D_a = 1/sqrt(A64_aa) = a!/sqrt(mu_2a); equilibrated FP32
    // Gram D A64 D, packed lower
    float dsc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
      dsc[i] = (float)(1.0 / IF.v[i + SKIP]) * rsqrtf((float)GMLS_MU(SI.idx[i + SKIP][i + SKIP], 0));
    float L[NP];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double di = (double)dsc[i] * IF.v[i + SKIP];
#pragma unroll
      for (int k = 0; k <= i; ++k)
        L[Packed<Q>::at(i, k)] =
            (float)(GMLS_MU(SI.idx[i + SKIP][k + SKIP], 0) * di * ((double)dsc[k] * IF.v[k + SKIP]));
    }
    float anorm = 0.f;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      float sum = 0.f;
#pragma unroll
      for (int i = 0; i < Q; ++i) sum += fabsf(i >= k ? L[Packed<Q>::at(i, k)] : L[Packed<Q>::at(k, i)]);
      anorm = fmaxf(anorm, sum);
    }
    // Cholesky in place; the diagonal keeps 1/L_jj
    bool ok = valid;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      float dj = L[Packed<Q>::at(j, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) dj -= L[Packed<Q>::at(j, k)] * L[Packed<Q>::at(j, k)];
      const bool pos = dj > 1e-12f;
      ok = ok && pos;
      const float inv = pos ? rsqrtf(dj) : 1.0f;
      L[Packed<Q>::at(j, j)] = inv;
#pragma unroll
      for (int i = j + 1; i < Q; ++i) {
        float v = L[Packed<Q>::at(i, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= L[Packed<Q>::at(i, k)] * L[Packed<Q>::at(j, k)];
        L[Packed<Q>::at(i, j)] = v * inv;
      }
    }
    // Hager's 1-norm estimate of A~^-1 (A~ symmetric)
    float x[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) x[i] = 1.0f / Q;
    packed_solve<Q>(L, x);
    float est = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) est += fabsf(x[i]);
#pragma unroll
    for (int i = 0; i < Q; ++i) x[i] = x[i] >= 0.f ? 1.f : -1.f;
    packed_solve<Q>(L, x);
    int jmax = 0;
    float zmax = -1.f;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (fabsf(x[i]) > zmax) {
        zmax = fabsf(x[i]);
        jmax = i;
      }
#pragma unroll
    for (int i = 0; i < Q; ++i) x[i] = i == jmax ? 1.f : 0.f;
    packed_solve<Q>(L, x);
    float est2 = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) est2 += fabsf(x[i]);
    const float cond = anorm * fmaxf(est, est2);
    if (valid && a.cond_out) a.cond_out[t] = cond;
    if (!(cond <= opt.cond_threshold)) ok = false;
    if (opt.force_fallback) ok = false;
    const double rho = fmin(0.5, 2.0 * Q * (double)cond * 5.960464477539063e-08);

    int sweeps_max = 0;
    bool conv_all = true;
    for (int f = 0; f < F; ++f) {
      const int kind = rk.kind[f];
      // y0 = D A~^-1 D lambda
#pragma unroll
      for (int i = 0; i < Q; ++i) x[i] = (float)scalar_lambda<DIM, ORDER>(kind, i + SKIP, ie) * dsc[i];
      packed_solve<Q>(L, x);
#pragma unroll
      for (int i = 0; i < Q; ++i) ybuf[i][lane] = (double)(x[i] * dsc[i]);
      bool conv = false;
      int sweeps = 0;
      for (int it = 0; it < opt.max_sweeps && ok && !conv; ++it) {
        // r_a = lambda_a - (1/a!) sum_b mu_(a+b) y_b / b!  (FP64), moment-major;
        // the empty asm keeps the moment loads inside the sweep (hoisting
        // all of them would hold NM doubles live across the loop)
        int zoff = 0;
        asm volatile("" : "+v"(zoff));
        double yf[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) yf[k] = ybuf[k][lane] * IF.v[k + SKIP];
        double acc[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) acc[i] = 0.0;
#pragma unroll
        for (int pp = 0; pp < MP.P; ++pp) {
          if (MP.a[pp] < SKIP || MP.b[pp] < SKIP) continue;
          const double mv = GMLS_MU(MP.m[pp], zoff);
          acc[MP.a[pp] - SKIP] += mv * yf[MP.b[pp] - SKIP];
        }
#pragma unroll
        for (int i = 0; i < Q; ++i)
          x[i] = (float)((scalar_lambda<DIM, ORDER>(kind, i + SKIP, ie) - IF.v[i + SKIP] * acc[i]) * (double)dsc[i]);
        packed_solve<Q>(L, x);
        double dmax = 0.0, ymax = 0.0;
        bool finite = true;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const double dy = (double)x[i] * (double)dsc[i];
          const double yn = ybuf[i][lane] + dy;
          ybuf[i][lane] = yn;
          finite = finite && isfinite(dy);
          dmax = fmax(dmax, fabs(dy));
          ymax = fmax(ymax, fabs(yn));
        }
        sweeps = it + 1;
        if (!finite) break;
        if (rho * dmax <= opt.refine_tol * ymax) conv = true;
      }
      conv_all = conv_all && conv;
      sweeps_max = sweeps > sweeps_max ? sweeps : sweeps_max;
      if (valid) {
#pragma unroll
        for (int i = 0; i < Q; ++i) yout[(loc * F + f) * Q + i] = ybuf[i][lane];
      }
    }
    const bool good = valid && ok && conv_all;
    const bool not_conv = valid && ok && !conv_all;
    const bool fell = valid && !ok;
    if (valid) {
      a.status[t] = good ? GMLS_TARGET_OK : not_conv ? GMLS_TARGET_NOT_CONVERGED : GMLS_TARGET_FALLBACK;
      rec[sl - c0].ok = good ? 1 : 0;
    }
    if (not_conv || fell) fb_list[atomicAdd(&meta->fb_count, 1)] = t;
    // statistics, aggregated over the wavefront (one atomic per counter)
    const int sw = sweeps_max < 15 ? sweeps_max : 15;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const unsigned long long m = __ballot(good && sw == k);
      if (lane == 0 && m) atomicAdd(&stats->sweep_hist[k], (unsigned long long)__popcll(m));
    }
    const unsigned long long mnc = __ballot(not_conv), mfb = __ballot(fell);
    if (lane == 0 && mnc) atomicAdd(&stats->n_not_converged, (unsigned long long)__popcll(mnc));
    if (lane == 0 && mfb) atomicAdd(&stats->n_fallback, (unsigned long long)__popcll(mfb));
    double cd = valid && (double)cond >= 0.0 ? (double)cond : 0.0;  // NaN estimates are skipped
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) cd = fmax(cd, __shfl_xor(cd, o));
    if (lane == 0 && cd > 0.0) atomicMax(&stats->cond_max_bits, (unsigned long long)__double_as_longlong(cd));
  }
#undef GMLS_MU
}

// ---------------------------------------------------------------------------
// C. weights
// ---------------------------------------------------------------------------
// F functional rows (compile time, so that the group's solutions stay in
// registers: F*Q doubles per lane).
// SKIP = 1 (staggered): columns are monomials 1..Q-1, and the group also
// writes each row's target weight -sum_j alpha_j.
template <int DIM, int ORDER, int G, int RPL, int F, int SKIP = 0, bool LOOP = false>
__global__ __launch_bounds__(64) void k_pipe_weights(StencilArgs a, const PipeRec *rec, const BinMeta *meta, int bin,
                                                     int win_lo, int win_hi, const double *yin) {
  const SlotRange R = slot_range(meta, bin, win_lo, win_hi);
  const int first = R.first, last = R.last, c0 = R.c0;
  constexpr int QF = num_mono(DIM, ORDER);
  constexpr int Q = QF - SKIP;
  constexpr int TPW = 64 / G;
  const int lane = lane_id();
  const int grp = lane / G, lg = lane % G;
  for (int i0 = first + xcd_block() * TPW; i0 < last; i0 += gridDim.x * TPW) {
    const int i = i0 + grp;
    const bool valid = i < last;
    const int64_t loc = (valid ? i : first) - c0;
    const PipeRec rc = rec[loc];
    const bool good = valid && rc.ok;
    double y[F][Q];
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
      for (int q = 0; q < Q; ++q) y[f][q] = yin[(loc * F + f) * Q + q];
    const int64_t base = rc.base;
    const int N = rc.n;
    const double ie = rc.ie;
    double xt[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) xt[d] = rc.x[d];
    // p(s) . y = sum_a (y_a / a!) s^a: the factorials go into the
    // coefficients once per target, the rows take a Horner evaluation
    constexpr InvFact64<DIM, ORDER> IFW{};
    double cf[F][QF];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      if constexpr (SKIP != 0) cf[f][0] = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) cf[f][q + SKIP] = y[f][q] * IFW.v[q + SKIP];
    }
    double *wout = a.weights + (int64_t)F * base;
    double rsum[F];
#pragma unroll
    for (int f = 0; f < F; ++f) rsum[f] = 0.0;
    const int cend = chunk_end<LOOP, G * RPL>(N);
    for (int q0 = 0; q0 < cend; q0 += G * RPL) {  // one pass unless LOOP (the long bin)
      const int nrem = N - q0;
      double xs[RPL][DIM];
      gather_rows<DIM, RPL, G>(a, base + (nrem > 0 ? q0 : 0), nrem > 0 ? nrem : N, lg, xs);
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        double s[DIM];
        const double w = row_sw<DIM>(xs[r], xt, ie, a.p, true, s);
        const int j = lg + G * r;
#pragma unroll
        for (int f = 0; f < F; ++f) {
          const double acc = horner<DIM, ORDER>(cf[f], s);
          if (good && j < nrem) wout[(int64_t)f * N + q0 + j] = w * acc;
          if constexpr (SKIP != 0) rsum[f] += j < nrem ? w * acc : 0.0;
        }
      }
    }
    if constexpr (SKIP != 0) {
      // the group's row sums, its G lanes in a fixed butterfly order
#pragma unroll
      for (int f = 0; f < F; ++f) {
#pragma unroll
        for (int off = 1; off < G; off <<= 1) rsum[f] += __shfl_xor(rsum[f], off, 64);
        if (good && lg == 0) a.hweights[(int64_t)rc.t * F + f] = -rsum[f];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Divergence-free basis (Section 2.2) on the pipeline, for scalar bases of
// at most 10 monomials.  The divergence-free span is the kernel of the
// divergence map D on the full vector polynomial space (coefficients c_(a,k)
// of p_a e_k): with the eps-scaled Taylor monomials, d/ds_k p_a = p_(a-e_k),
// so (D c)_b = sum_k c_(b+e_k, k) for every monomial b of degree < m.  The
// weighted least squares over that span is the vector fit with Gram
// I (x) G_s (G_s the scalar moment Gram, Section 2.1) under D c = 0; for a
// functional l its value is g^T (P^T W u) with
//     g = G^-1 (l - D^T t),   S t = D G^-1 l,   S = D G^-1 D^T
// (G = I (x) G_s), which takes only solves with the scalar Gram and a small
// Schur complement.  Solve kernel: one thread per target, G_s equilibrated
// and factored by Cholesky in FP64 (the moment Gram has at most 10 columns
// here), Hager's estimate of its condition number against the threshold;
// g for every (functional, component) goes to HBM, and the weights kernel
// forms alpha_(j,c) = w_j p(s_j) . g_c.  The divergence functional of a
// divergence-free fit is identically zero: its g is 0.
// ---------------------------------------------------------------------------
template <int DIM, int ORDER>
struct DivUp {
  static constexpr int QS = num_mono(DIM, ORDER);
  static constexpr int QM = ORDER >= 1 ? num_mono(DIM, ORDER - 1) : 1;
  int up[QM][3];  // index of the monomial b + e_k
  constexpr DivUp() : up{} {
    Mono<DIM, ORDER> M{};
    for (int b = 0; b < QM; ++b)
      for (int k = 0; k < 3; ++k) {
        up[b][k] = -1;
        if (k >= DIM) continue;
        int e[3] = {M.e[b][0], M.e[b][1], M.e[b][2]};
        e[k] += 1;
        for (int a = 0; a < QS; ++a)
          if (M.e[a][0] == e[0] && M.e[a][1] == e[1] && M.e[a][2] == e[2]) up[b][k] = a;
      }
  }
};

// x <- (L L^T)^-1 x for a packed lower-triangular FP64 L with 1/L_jj on the
// diagonal
template <int Q>
__device__ __forceinline__ void packed_solve64(const double *L, double *x) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    double v = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= L[Packed<Q>::at(i, k)] * x[k];
    x[i] = v * L[Packed<Q>::at(i, i)];
  }
#pragma unroll
  for (int i = Q - 1; i >= 0; --i) {
    double v = x[i];
#pragma unroll
    for (int k = i + 1; k < Q; ++k) v -= L[Packed<Q>::at(k, i)] * x[k];
    x[i] = v * L[Packed<Q>::at(i, i)];
  }
}

// in-place packed Cholesky (diagonal keeps 1/L_jj); false on a pivot <= tol
template <int Q>
__device__ __forceinline__ bool packed_cholesky64(double *L, double tol) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    double dj = L[Packed<Q>::at(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= L[Packed<Q>::at(j, k)] * L[Packed<Q>::at(j, k)];
    const bool pos = dj > tol;
    ok = ok && pos;
    const double inv = pos ? 1.0 / sqrt(dj) : 1.0;
    L[Packed<Q>::at(j, j)] = inv;
#pragma unroll
    for (int i = j + 1; i < Q; ++i) {
      double v = L[Packed<Q>::at(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[Packed<Q>::at(i, k)] * L[Packed<Q>::at(j, k)];
      L[Packed<Q>::at(i, j)] = v * inv;
    }
  }
  return ok;
}

template <int DIM, int ORDER>
__global__ __launch_bounds__(64) void k_pipe_solve_div(StencilArgs a, PipeRec *rec, int win_lo, int win_hi,
                                                       const double *mom, double *gout, int *fb_list, BinMeta *meta,
                                                       Stats *stats, Options opt) {
  constexpr int QS = num_mono(DIM, ORDER);
  constexpr int QM = DivUp<DIM, ORDER>::QM;
  constexpr int NP = QS * (QS + 1) / 2;
  constexpr InvFact64<DIM, ORDER> IF{};
  constexpr SumIndex<DIM, ORDER> SI{};
  constexpr DivUp<DIM, ORDER> DU{};
  constexpr int NM = num_mono(DIM, 2 * ORDER);
  __shared__ double mls[NM][64];  // thread-private columns: lane l uses [.][l]
  const int lane = lane_id();
  const RowKinds rk = row_kinds(DIM, 1, a.mask);
  const int F = a.F;
  const SlotRange R = slot_range(meta, 0, win_lo, win_hi);
  const int first = R.first, last = R.last, c0 = R.c0;
  for (int slot = first + xcd_block() * 64 + lane; slot - lane < last; slot += gridDim.x * 64) {
    const bool valid = slot < last;
    const int sl = valid ? slot : first;
    const int t = rec[sl - c0].t;
    const double ie = rec[sl - c0].ie;
    const int64_t loc = sl - c0;
    if (valid) {
#pragma unroll
      for (int m = 0; m < NM; ++m) mls[m][lane] = mom[loc * NM + m];
    }
    // G_s_ab = mu_(a+b)/(a! b!); its equilibration sc G_s sc (sc_a =
    // 1/sqrt(G_s_aa)) is the moment matrix scaled by dsc_a = 1/sqrt(mu_2a)
    double dsc[QS], sc[QS];
#pragma unroll
    for (int i = 0; i < QS; ++i) {
      dsc[i] = 1.0 / sqrt(mls[SI.idx[i][i]][lane]);
      sc[i] = dsc[i] / IF.v[i];
    }
    double L[NP];
#pragma unroll
    for (int i = 0; i < QS; ++i)
#pragma unroll
      for (int k = 0; k <= i; ++k) L[Packed<QS>::at(i, k)] = mls[SI.idx[i][k]][lane] * dsc[i] * dsc[k];
    double anorm = 0.0;
#pragma unroll
    for (int k = 0; k < QS; ++k) {
      double sum = 0.0;
#pragma unroll
      for (int i = 0; i < QS; ++i) sum += fabs(i >= k ? L[Packed<QS>::at(i, k)] : L[Packed<QS>::at(k, i)]);
      anorm = fmax(anorm, sum);
    }
    bool ok = valid && packed_cholesky64<QS>(L, 1e-12);
    // Hager's 1-norm estimate of the inverse
    double x[QS];
#pragma unroll
    for (int i = 0; i < QS; ++i) x[i] = 1.0 / QS;
    packed_solve64<QS>(L, x);
    double est = 0.0;
#pragma unroll
    for (int i = 0; i < QS; ++i) est += fabs(x[i]);
#pragma unroll
    for (int i = 0; i < QS; ++i) x[i] = x[i] >= 0.0 ? 1.0 : -1.0;
    packed_solve64<QS>(L, x);
    int jmax = 0;
    double zmax = -1.0;
#pragma unroll
    for (int i = 0; i < QS; ++i)
      if (fabs(x[i]) > zmax) {
        zmax = fabs(x[i]);
        jmax = i;
      }
#pragma unroll
    for (int i = 0; i < QS; ++i) x[i] = i == jmax ? 1.0 : 0.0;
    packed_solve64<QS>(L, x);
    double est2 = 0.0;
#pragma unroll
    for (int i = 0; i < QS; ++i) est2 += fabs(x[i]);
    const double cond = anorm * fmax(est, est2);
    if (valid && a.cond_out) a.cond_out[t] = (float)cond;
    if (!(cond <= opt.cond_threshold)) ok = false;
    if (opt.force_fallback) ok = false;
    // solves with the Gram: G_s^-1 v = sc . (L L^T)^-1 (sc . v)
    // S = D G^-1 D^T, column b2: component k contributes G_s^-1 e_(b2+e_k)
    // at rows b+e_k
    double S[QM * (QM + 1) / 2];
#pragma unroll
    for (int q = 0; q < QM * (QM + 1) / 2; ++q) S[q] = 0.0;
#pragma unroll
    for (int b2 = 0; b2 < QM; ++b2)
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
#pragma unroll
        for (int i = 0; i < QS; ++i) x[i] = i == DU.up[b2][k] ? sc[i] : 0.0;
        packed_solve64<QS>(L, x);
#pragma unroll
        for (int b = b2; b < QM; ++b) S[Packed<QM>::at(b, b2)] += x[DU.up[b][k]] * sc[DU.up[b][k]];
      }
    ok = ok && packed_cholesky64<QM>(S, 1e-300);
    for (int f = 0; f < F; ++f) {
      const int kind = rk.kind[f], comp = rk.comp[f];
      double g[DIM][QS];
      if (kind == FK_DIV) {
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
          for (int i = 0; i < QS; ++i) g[k][i] = 0.0;
      } else {
        // v = G_s^-1 l (component comp), r_b = v_(b + e_comp), t = S^-1 r
        double lam[QS];
#pragma unroll
        for (int i = 0; i < QS; ++i) lam[i] = scalar_lambda<DIM, ORDER>(kind, i, ie);
#pragma unroll
        for (int i = 0; i < QS; ++i) x[i] = lam[i] * sc[i];
        packed_solve64<QS>(L, x);
        double tv[QM];
#pragma unroll
        for (int b = 0; b < QM; ++b) {
          tv[b] = 0.0;
#pragma unroll
          for (int k = 0; k < DIM; ++k)
            if (k == comp) tv[b] = x[DU.up[b][k]] * sc[DU.up[b][k]];
        }
        packed_solve64<QM>(S, tv);
        // g_k = G_s^-1 (delta_(k,comp) l - sum_b t_b e_(b+e_k))
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
#pragma unroll
          for (int i = 0; i < QS; ++i) {
            double v = k == comp ? lam[i] : 0.0;
#pragma unroll
            for (int b = 0; b < QM; ++b)
              if (DU.up[b][k] == i) v -= tv[b];
            g[k][i] = v * sc[i];
          }
          packed_solve64<QS>(L, g[k]);
#pragma unroll
          for (int i = 0; i < QS; ++i) g[k][i] *= sc[i];
        }
      }
      if (valid) {
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
          for (int i = 0; i < QS; ++i) gout[((loc * F + f) * DIM + k) * QS + i] = g[k][i];
      }
    }
    const bool good = valid && ok;
    const bool fell = valid && !ok;
    if (valid) {
      a.status[t] = good ? GMLS_TARGET_OK : GMLS_TARGET_FALLBACK;
      rec[sl - c0].ok = good ? 1 : 0;
    }
    if (fell) fb_list[atomicAdd(&meta->fb_count, 1)] = t;
    const unsigned long long mg = __ballot(good), mfb = __ballot(fell);
    if (lane == 0 && mg) atomicAdd(&stats->sweep_hist[0], (unsigned long long)__popcll(mg));
    if (lane == 0 && mfb) atomicAdd(&stats->n_fallback, (unsigned long long)__popcll(mfb));
    double cd = valid && cond >= 0.0 ? cond : 0.0;  // NaN estimates are skipped
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) cd = fmax(cd, __shfl_xor(cd, o));
    if (lane == 0 && cd > 0.0) atomicMax(&stats->cond_max_bits, (unsigned long long)__double_as_longlong(cd));
  }
}

// alpha_(j, f, c) = w_j p(s_j) . g_(f,c), one functional row f (its DIM
// components' coefficients in registers, Horner evaluation) per pass over
// the rows.  The G lanes of a group hold G consecutive rows, whose DIM
// components form one contiguous run of G*DIM doubles: the values are staged
// in LDS and stored as DIM fully coalesced runs instead of DIM stores with a
// DIM-double stride (which split every cache line between instructions).
template <int DIM, int ORDER, int G, int RPL, bool LOOP = false>
__global__ __launch_bounds__(64) void k_pipe_weights_div(StencilArgs a, const PipeRec *rec, const BinMeta *meta,
                                                         int bin, int win_lo, int win_hi, const double *gin) {
  const SlotRange R = slot_range(meta, bin, win_lo, win_hi);
  const int first = R.first, last = R.last, c0 = R.c0;
  constexpr int QS = num_mono(DIM, ORDER);
  constexpr int TPW = 64 / G;
  constexpr int CW = DIM * QS;                 // coefficients of one target and row
  constexpr int NL = (TPW * CW + 63) / 64;     // of the wavefront's targets, per lane
  constexpr InvFact64<DIM, ORDER> IFW{};
  __shared__ double stage[64 * DIM];  // group g: [g * G * DIM, (g + 1) * G * DIM)
  __shared__ double cfs[2][TPW * CW];  // row f's coefficients of the wavefront's targets, by f % 2
  const int lane = lane_id();
  const int grp = lane / G, lg = lane % G;
  const int F = a.F, FC = F * DIM;
  double *gst = stage + grp * G * DIM;
  for (int i0 = first + xcd_block() * TPW; i0 < last; i0 += gridDim.x * TPW) {
    // the coefficients of row f of the wavefront's TPW targets, fetched by
    // all lanes together one row ahead (row 0 with the neighbour gathers)
    double pre[NL];
    auto fetch = [&](int f) {
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int e = lane + 64 * u, tt = e / CW;
        pre[u] = e < TPW * CW && i0 + tt < last ? gin[((int64_t)(i0 + tt - c0) * FC * QS) + f * CW + (e - tt * CW)] : 0.0;
      }
    };
    fetch(0);
    const int i = i0 + grp;
    const bool valid = i < last;
    const int64_t loc = (valid ? i : first) - c0;
    const PipeRec rc = rec[loc];
    const bool good = valid && rc.ok;
    const int64_t base = rc.base;
    const int N = rc.n;
    double xt[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) xt[d] = rc.x[d];
    double *wout = a.weights + (int64_t)FC * base;
    // one pass unless LOOP (the long bin): then every chunk of G * RPL rows
    // is gathered again for each functional row
    const int cend = chunk_end<LOOP, G * RPL>(N);
    double xs[RPL][DIM];
    gather_rows<DIM, RPL, G>(a, base, N, lg, xs);
    double s[RPL][DIM], w[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) w[r] = row_sw<DIM>(xs[r], xt, rc.ie, a.p, true, s[r]);
    for (int f = 0; f < F; ++f) {
      double *cb = cfs[f & 1];
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int e = lane + 64 * u;
        if (e < TPW * CW) cb[e] = pre[u];
      }
      __syncthreads();
      if (f + 1 < F) fetch(f + 1);
      double cf[DIM][QS];
#pragma unroll
      for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int q = 0; q < QS; ++q) cf[c][q] = cb[grp * CW + c * QS + q] * IFW.v[q];
      for (int q0 = 0; q0 < cend; q0 += G * RPL) {
        const int nrem = N - q0;
        if (LOOP && (q0 > 0 || f > 0)) {  // the rows of this chunk (chunk 0 of row 0 is loaded above)
          gather_rows<DIM, RPL, G>(a, base + (nrem > 0 ? q0 : 0), nrem > 0 ? nrem : N, lg, xs);
#pragma unroll
          for (int r = 0; r < RPL; ++r) w[r] = row_sw<DIM>(xs[r], xt, rc.ie, a.p, true, s[r]);
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
#pragma unroll
          for (int c = 0; c < DIM; ++c) gst[lg * DIM + c] = w[r] * horner<DIM, ORDER>(cf[c], s[r]);
          __syncthreads();
          // the group's rows q0 + G r .. q0 + G r + G - 1: doubles (f N + q0 + G r) DIM + m, m < G DIM
          double *run = wout + ((int64_t)f * N + q0 + G * r) * DIM;
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
            const int m = k * G + lg;
            if (good && G * r + m / DIM < nrem) run[m] = gst[m];
          }
          __syncthreads();
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host: the pipeline over the bins of one call, in chunks of list slots
// ---------------------------------------------------------------------------
template <int DIM, int ORDER>
constexpr bool has_pipe() {
  return num_mono(DIM, ORDER) <= 20;
}

// the divergence-free pipeline factors the scalar Gram in FP64 registers
template <int DIM, int ORDER>
constexpr bool has_pipe_div() {
  return ORDER >= 1 && num_mono(DIM, ORDER) <= 10;
}

template <int DIM, int ORDER, int G, int RPL, int SKIP, int BASIS = 0, bool LOOP = false>
static void pipe_bin_launch(bool weights, const StencilArgs &a, const PipeRec *rec, const BinMeta *meta, int bin,
                            int win_lo, int win_hi, int n_max, double *buf, int cus, hipStream_t s) {
  constexpr int TPW = 64 / G;
  int nb = (n_max + TPW - 1) / TPW;
  if (nb > cus * 32) nb = cus * 32;
  nb = xcd_grid(nb);
  if (!weights) {
    k_pipe_moments<DIM, ORDER, G, RPL, LOOP><<<nb, 64, 0, s>>>(a, rec, meta, bin, win_lo, win_hi, buf);
    return;
  }
  if constexpr (BASIS == 1) {
    k_pipe_weights_div<DIM, ORDER, G, RPL, LOOP><<<nb, 64, 0, s>>>(a, rec, meta, bin, win_lo, win_hi, buf);
    return;
  }
  switch (a.F) {  // scalar basis: value + up to DIM gradient rows + Laplacian
    case 1: k_pipe_weights<DIM, ORDER, G, RPL, 1, SKIP, LOOP><<<nb, 64, 0, s>>>(a, rec, meta, bin, win_lo, win_hi, buf); break;
    case 2: k_pipe_weights<DIM, ORDER, G, RPL, 2, SKIP, LOOP><<<nb, 64, 0, s>>>(a, rec, meta, bin, win_lo, win_hi, buf); break;
    case 3: k_pipe_weights<DIM, ORDER, G, RPL, 3, SKIP, LOOP><<<nb, 64, 0, s>>>(a, rec, meta, bin, win_lo, win_hi, buf); break;
    case 4: k_pipe_weights<DIM, ORDER, G, RPL, 4, SKIP, LOOP><<<nb, 64, 0, s>>>(a, rec, meta, bin, win_lo, win_hi, buf); break;
    default:
      if constexpr (DIM == 3 && SKIP == 0)
        k_pipe_weights<DIM, ORDER, G, RPL, 5, SKIP, LOOP><<<nb, 64, 0, s>>>(a, rec, meta, bin, win_lo, win_hi, buf);
      break;
  }
}

// the bin's launch in row shape `cand` (kPipeShapes)
template <int DIM, int ORDER, int SKIP, int BASIS, int BIN>
static void pipe_bin_shape(int cand, bool weights, const StencilArgs &a, const PipeRec *rec, const BinMeta *meta,
                           int win_lo, int win_hi, int n_max, double *buf, int cus, hipStream_t s) {
  constexpr PipeShape S0 = kPipeShapes[BIN][0], S1 = kPipeShapes[BIN][1], S2 = kPipeShapes[BIN][2];
  constexpr bool L = BIN == kLongBin;
  if (cand == 1)
    pipe_bin_launch<DIM, ORDER, S1.g, S1.rpl, SKIP, BASIS, L>(weights, a, rec, meta, BIN, win_lo, win_hi, n_max,
                                                              buf, cus, s);
  else if (cand == 2)
    pipe_bin_launch<DIM, ORDER, S2.g, S2.rpl, SKIP, BASIS, L>(weights, a, rec, meta, BIN, win_lo, win_hi, n_max,
                                                              buf, cus, s);
  else
    pipe_bin_launch<DIM, ORDER, S0.g, S0.rpl, SKIP, BASIS, L>(weights, a, rec, meta, BIN, win_lo, win_hi, n_max,
                                                              buf, cus, s);
}

// The pipeline over list slots [count[0], n) (bins 1..4, contiguous, in bin
// order).  With a host copy of the bin table (hm) it runs in chunks of
// `chunk` slots and skips empty bins; without one (hm == nullptr: nothing
// may wait for the device) it covers every slot in one window, all bounds
// read from the device table, grids sized for n_max slots.
// Lanes x rows per lane of the moment and weight kernels: the candidate
// opt.pipe_shape[kernel][bin] of kPipeShapes (default, candidate 0: bin 1
// (<= 64 rows) 8 x 8, bin 2 (<= 128) 16 x 8, bin 3 (<= 192) 32 x 6, bin 4
// (<= 256) 32 x 8).  With a timer, events bracket every per-bin launch.
template <int DIM, int ORDER, int SKIP = 0, int BASIS = 0>
hipError_t launch_pipe(const StencilArgs &a, const int *list, const BinMeta *hm, BinMeta *meta, int *fb,
                       Stats *stats, const Options &opt, double *mom, double *y, PipeRec *rec, int64_t chunk,
                       int n_max, int cus, PipeTimer *timer, hipStream_t s) {
  int begin = 0, end = 1;
  if (hm) {
    begin = hm->offset[1];
    end = hm->offset[kNumBins - 1] + hm->count[kNumBins - 1];
  } else {
    chunk = 1;
  }
  for (int64_t c0 = begin; c0 < end; c0 += chunk) {
    const int win_lo = hm ? (int)c0 : -1;
    const int win_hi = hm ? (int)(c0 + chunk < end ? c0 + chunk : end) : INT_MAX;
    const int n_win = hm ? win_hi - win_lo : n_max;
    if (!opt.reuse_moments) {
      int nbp = (n_win + 255) / 256;
      if (nbp > cus * 8) nbp = cus * 8;
      if (nbp < 1) nbp = 1;
      k_pipe_prep<DIM><<<nbp, 256, 0, s>>>(a, list, meta, win_lo, win_hi, rec);
    }
    // a second stencil set on the same neighbour lists (one window) takes
    // the records and moments of the first
    for (int pass = opt.reuse_moments ? 1 : 0; pass < 2; ++pass) {
      if (pass == 1) {
        int nb = (n_win + 63) / 64;
        if (nb > cus * 16) nb = cus * 16;
        nb = xcd_grid(nb);
        if constexpr (BASIS == 1)
          k_pipe_solve_div<DIM, ORDER><<<nb, 64, 0, s>>>(a, rec, win_lo, win_hi, mom, y, fb, meta, stats, opt);
        else
          k_pipe_solve<DIM, ORDER, SKIP><<<nb, 64, 0, s>>>(a, rec, win_lo, win_hi, mom, y, fb, meta, stats, opt);
      }
      const bool wts = pass == 1;
      for (int b = 1; b < kNumBins; ++b) {
        int nbin = n_max;
        if (hm) {
          const int lo = hm->offset[b] > win_lo ? hm->offset[b] : win_lo;
          const int hi = hm->offset[b] + hm->count[b] < win_hi ? hm->offset[b] + hm->count[b] : win_hi;
          if (lo >= hi) continue;
          nbin = hi - lo;
        }
        double *buf = wts ? y : mom;
        const int cand = opt.pipe_shape[pass][b];
        if (timer) {
          hipError_t e = hipEventRecord(timer->ev[pass][b][0], s);
          if (e != hipSuccess) return e;
        }
        if (b == 1)
          pipe_bin_shape<DIM, ORDER, SKIP, BASIS, 1>(cand, wts, a, rec, meta, win_lo, win_hi, nbin, buf, cus, s);
        else if (b == 2)
          pipe_bin_shape<DIM, ORDER, SKIP, BASIS, 2>(cand, wts, a, rec, meta, win_lo, win_hi, nbin, buf, cus, s);
        else if (b == 3)
          pipe_bin_shape<DIM, ORDER, SKIP, BASIS, 3>(cand, wts, a, rec, meta, win_lo, win_hi, nbin, buf, cus, s);
        else if (b == 4)
          pipe_bin_shape<DIM, ORDER, SKIP, BASIS, 4>(cand, wts, a, rec, meta, win_lo, win_hi, nbin, buf, cus, s);
        else
          pipe_bin_shape<DIM, ORDER, SKIP, BASIS, kLongBin>(cand, wts, a, rec, meta, win_lo, win_hi, nbin, buf, cus,
                                                            s);
        if (timer) {
          hipError_t e = hipEventRecord(timer->ev[pass][b][1], s);
          if (e != hipSuccess) return e;
          timer->used[pass][b] = 1;
        }
      }
    }
  }
  return hipGetLastError();
}

}  // namespace gmls
