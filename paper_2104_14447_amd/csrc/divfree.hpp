// divfree.hpp -- a divergence-free vector basis of degree <= m (Section 2.2).
//
// In the scaled monomials p_b (s = (x - x_T)/eps, p_b = s^b/b!) one has
// d/ds_c p_b = p_(b - e_c), so for every monomial p_b and every component
// c >= 1 the field
//     psi = p_b e_c - p_(b - e_c + e_x) e_x      (second term only if b_c >= 1)
// has zero divergence, and so has p_g e_x for every g with g_x = 0.  Taken
// over all monomials of degree <= m these fields are linearly independent
// (component c >= 1 of each field of the first kind is a distinct monomial)
// and their number equals dim*C(m+dim,dim) - C(m-1+dim,dim), the dimension of
// the divergence-free polynomials, so they span that space.  Each column of
// the coefficient matrix T (rows (b, c)) therefore has at most two entries,
// both +-1.
#pragma once

#include "basis.hpp"

namespace gmls {

template <int DIM, int ORDER>
struct DivFreeTab {
  static constexpr int Q = num_mono(DIM, ORDER);
  static constexpr int QD = DIM * num_mono(DIM, ORDER) - num_mono(DIM, ORDER - 1);
  int ia[QD], ca[QD], ib[QD], cb[QD];
  double va[QD], vb[QD];
  // indices of the pure squares 2e_d and of e_d (for functionals)
  constexpr DivFreeTab() : ia{}, ca{}, ib{}, cb{}, va{}, vb{} {
    Mono<DIM, ORDER> M{};
    int n = 0;
    for (int deg = 0; deg <= ORDER; ++deg)
      for (int b = 0; b < M.N; ++b) {
        if (M.e[b][0] + M.e[b][1] + M.e[b][2] != deg) continue;
        for (int c = 1; c < DIM; ++c) {
          ia[n] = b;
          ca[n] = c;
          va[n] = 1.0;
          ib[n] = -1;
          cb[n] = 0;
          vb[n] = 0.0;
          if (M.e[b][c] >= 1) {
            int w[3] = {M.e[b][0], M.e[b][1], M.e[b][2]};
            w[c] -= 1;
            w[0] += 1;
            ib[n] = M.index(w[0], w[1], w[2]);
            cb[n] = 0;
            vb[n] = -1.0;
          }
          ++n;
        }
        if (M.e[b][0] == 0) {
          ia[n] = b;
          ca[n] = 0;
          va[n] = 1.0;
          ib[n] = -1;
          cb[n] = 0;
          vb[n] = 0.0;
          ++n;
        }
      }
  }
};

template <int DIM, int ORDER>
__constant__ DivFreeTab<DIM, ORDER> kDivFree = DivFreeTab<DIM, ORDER>();

// functional of `kind` (output component comp) applied at x_T to the scaled
// monomial field p_b e_c: value -> [b == 0][c == comp]; Laplacian ->
// eps^-2 [b is a pure square][c == comp]; divergence -> eps^-1 [b == e_c]
template <int DIM, int ORDER>
__device__ __forceinline__ double vec_mono_functional(int b, int c, int kind, int comp, double ie) {
  constexpr Mono<DIM, ORDER> M{};
  (void)M;
  if (kind == FK_VALUE) return (b == 0 && c == comp) ? 1.0 : 0.0;
  if (kind == FK_LAP) {
    if (c != comp) return 0.0;
    // pure squares in graded order: the degree-2 monomials with one exponent 2
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < M.N; ++q) {
      const bool pure2 = (M.e[q][0] + M.e[q][1] + M.e[q][2] == 2) &&
                         (M.e[q][0] == 2 || M.e[q][1] == 2 || M.e[q][2] == 2);
      if (pure2 && b == q) v = ie * ie;
    }
    return v;
  }
  if (kind == FK_DIV) return (b >= 1 && b <= DIM && b - 1 == c) ? ie : 0.0;
  return 0.0;
}

// lambda_i: the functional applied to basis field i
template <int DIM, int ORDER>
__device__ __forceinline__ double divfree_lambda(int i, int kind, int comp, double ie) {
  const DivFreeTab<DIM, ORDER> &T = kDivFree<DIM, ORDER>;
  double v = T.va[i] * vec_mono_functional<DIM, ORDER>(T.ia[i], T.ca[i], kind, comp, ie);
  if (T.ib[i] >= 0) v += T.vb[i] * vec_mono_functional<DIM, ORDER>(T.ib[i], T.cb[i], kind, comp, ie);
  return v;
}

}  // namespace gmls
