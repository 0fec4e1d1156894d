// basis.hpp -- device evaluation of the eps-scaled Taylor basis
// p_a(s) = prod_i s_i^a_i / a_i!  with s = (x - x_T)/eps (Section 2.1, basis
// equations), and the functionals of Section 2.5 applied to it at x_T.
#pragma once

#include "common.hpp"

namespace gmls {

// p[a] for every monomial of total degree <= DEG (scaled basis)
template <int DIM, int DEG, typename T>
__device__ __forceinline__ void scaled_basis(const T *s, T *p) {
  constexpr Mono<DIM, DEG> M{};
  T sd[DIM][DEG + 1];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    sd[d][0] = (T)1;
#pragma unroll
    for (int k = 1; k <= DEG; ++k) sd[d][k] = s[d] * (T)(1.0 / k);
  }
  p[0] = (T)1;
#pragma unroll
  for (int a = 1; a < M.N; ++a) p[a] = p[M.parent[a]] * sd[M.pdim[a]][M.pexp[a]];
}

// Index of the monomial x^i y^j z^k in the graded order of Mono<DIM, DEG>.
template <int DIM, int DEG>
struct MonoIndex {
  int idx[DEG + 1][DEG + 1][DEG + 1];
  constexpr MonoIndex() : idx{} {
    Mono<DIM, DEG> M{};
    for (int i = 0; i <= DEG; ++i)
      for (int j = 0; j <= DEG; ++j)
        for (int k = 0; k <= DEG; ++k) idx[i][j][k] = -1;
    for (int a = 0; a < M.N; ++a) idx[M.e[a][0]][M.e[a][1]][M.e[a][2]] = a;
  }
};

// sum_a c[a] s^a (plain monomials, total degree <= DEG) by nested Horner
// steps in z, then y, then x: one multiply-add per coefficient after the
// first of each innermost sum.
template <int DIM, int DEG>
__device__ __forceinline__ double horner(const double *c, const double *s) {
  constexpr MonoIndex<DIM, DEG> H{};
  double ax = 0.0;
#pragma unroll
  for (int i = DEG; i >= 0; --i) {
    double ay = 0.0;
    if constexpr (DIM == 1) {
      ay = c[H.idx[i][0][0]];
    } else {
#pragma unroll
      for (int j = DEG - i; j >= 0; --j) {
        double az;
        if constexpr (DIM == 3) {
          az = c[H.idx[i][j][DEG - i - j]];
#pragma unroll
          for (int k = DEG - i - j - 1; k >= 0; --k) az = az * s[2] + c[H.idx[i][j][k]];
        } else {
          az = c[H.idx[i][j][0]];
        }
        ay = j == DEG - i ? az : ay * s[1] + az;
      }
    }
    ax = i == DEG ? ay : ax * s[0] + ay;
  }
  return ax;
}

// plain monomials s^g (no factorials), total degree <= DEG
template <int DIM, int DEG, typename T>
__device__ __forceinline__ void plain_monomials(const T *s, T *p) {
  constexpr Mono<DIM, DEG> M{};
  p[0] = (T)1;
#pragma unroll
  for (int a = 1; a < M.N; ++a) p[a] = p[M.parent[a]] * s[M.pdim[a]];
}

// Functional kinds of the output rows.
enum FKind { FK_VALUE = 0, FK_GRAD0 = 1, FK_GRAD1 = 2, FK_GRAD2 = 3, FK_LAP = 4, FK_DIV = 5 };

struct RowKinds {
  int n;
  int kind[8];  // scalar basis: FKind; vector basis: kind with the output component in comp
  int comp[8];
};

// Row list of a mask in the output order value, gradient, Laplacian, divergence.
__host__ __device__ inline RowKinds row_kinds(int dim, int basis, unsigned mask) {
  RowKinds r{};
  r.n = 0;
  if (basis == 0) {
    if (mask & 1u) { r.kind[r.n] = FK_VALUE; r.comp[r.n++] = 0; }
    if (mask & 2u)
      for (int d = 0; d < dim; ++d) { r.kind[r.n] = FK_GRAD0 + d; r.comp[r.n++] = 0; }
    if (mask & 4u) { r.kind[r.n] = FK_LAP; r.comp[r.n++] = 0; }
  } else {
    if (mask & 1u)
      for (int c = 0; c < dim; ++c) { r.kind[r.n] = FK_VALUE; r.comp[r.n++] = c; }
    if (mask & 4u)
      for (int c = 0; c < dim; ++c) { r.kind[r.n] = FK_LAP; r.comp[r.n++] = c; }
    if (mask & 8u) { r.kind[r.n] = FK_DIV; r.comp[r.n++] = 0; }
  }
  return r;
}

// lambda[a] = (functional of kind) applied to the scaled monomial a at x_T:
// D^beta p_a(x_T) = eps^-|beta| when a == beta, else 0.
template <int DIM, int DEG>
__device__ __forceinline__ double scalar_lambda(int kind, int a, double ie) {
  constexpr Mono<DIM, DEG> M{};
  double v = 0.0;
  if (kind == FK_VALUE) {
    v = (a == 0) ? 1.0 : 0.0;
  } else if (kind >= FK_GRAD0 && kind <= FK_GRAD2) {
    const int d = kind - FK_GRAD0;
#pragma unroll
    for (int q = 1; q < M.N && q <= DIM; ++q)
      if (a == q && M.e[q][d] == 1) v = ie;
  } else if (kind == FK_LAP) {
#pragma unroll
    for (int q = 0; q < M.N; ++q) {
      const int deg = M.e[q][0] + M.e[q][1] + M.e[q][2];
      const bool pure2 = deg == 2 && (M.e[q][0] == 2 || M.e[q][1] == 2 || M.e[q][2] == 2);
      if (pure2 && a == q) v = ie * ie;
    }
  }
  return v;
}

}  // namespace gmls
