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
