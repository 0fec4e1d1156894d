"""Staggered GMLS stencils (Section 2.4), plain numpy -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module (through the ``oracle`` package); the
product library never calls it and shares no code with it.

Definition, in the section's order and notation.  The gradient field
q = grad p near a target x_T is fitted by a vector polynomial
q_h(x) = Phi(x) c, with Phi the vector polynomials of order <= m: here
phi_(a,k)(x) = e_k p_a((x - x_T)/eps), p_a(s) = prod s_i^a_i / a_i! (the
eps-scaled Taylor monomials of Section 2.1 in every component).  The data are
edge integrals: for neighbour j,

    xi_i(x_j) = integral of phi_i . dx along the segment x_T -> x_j,
    rho_j     = p_j - p(x_T),

and c minimises sum_j W(d_j) (xi(x_j) c - rho_j)^2, i.e. A_s c = B_s rho with
A_s = Xi^T W Xi, B_s = Xi^T W.  The segment integrals are taken by
Gauss-Legendre quadrature on [0, 1] (exact: the integrand is a polynomial of
degree m in the segment parameter).  The functionals act on the fit at x_T:
grad p(x_T) ~ Phi(x_T) c and Laplacian p(x_T) ~ (div Phi)(x_T) c.

Reading: the vector polynomials that circulate around x_T (phi(x) . (x - x_T)
= 0, e.g. the rotation (-(y - y_T), x - x_T)) have zero integral along every
segment from x_T, so A_s is singular.  A_s^-1 is read as the pseudo-inverse,
which gives the minimum-norm c = (W^1/2 Xi)^+ W^1/2 rho (SVD, singular values
below 1e-11 of the largest dropped); the null space changes neither
Phi(x_T) c nor (div Phi)(x_T) c, so the stencils are unique.

The stencil of a functional lambda is returned as weights alpha_j of the
neighbour values p_j and a target weight beta = -sum_j alpha_j of p(x_T)
(rho = D p with D p_j = p_j - p(x_T)).
"""
from __future__ import annotations

import math

import numpy as np

from .constrained import exponents

F_GRAD, F_LAPLACIAN = 2, 4
RCOND = 1e-11


def vector_basis(dim: int, m: int):
    """(monomial exponent, component) of every phi_i: monomial-major."""
    return [(tuple(int(v) for v in e[:dim]), k) for e in exponents(dim, m) for k in range(dim)]


def monomial(s: np.ndarray, e) -> np.ndarray:
    """p_e(s) = prod s_i^e_i / e_i! for rows s [N, dim]."""
    v = np.ones(s.shape[0])
    for i, ei in enumerate(e):
        if ei:
            v = v * s[:, i] ** ei / math.factorial(ei)
    return v


def edge_integrals(xs: np.ndarray, xt: np.ndarray, eps: float, basis, nq: int) -> np.ndarray:
    """Xi[j, i] = integral over t in [0, 1] of phi_i(x_T + t r_j) . r_j,
    r_j = x_j - x_T, by nq-point Gauss-Legendre quadrature."""
    t, wq = np.polynomial.legendre.leggauss(nq)
    t = 0.5 * (t + 1.0)
    wq = 0.5 * wq
    r = xs - xt
    Xi = np.zeros((xs.shape[0], len(basis)))
    for tq, w in zip(t, wq):
        s = tq * r / eps
        for i, (e, k) in enumerate(basis):
            Xi[:, i] += w * monomial(s, e) * r[:, k]
    return Xi


def functionals(dim: int, basis, mask: int, eps: float) -> np.ndarray:
    """Rows of Phi(x_T) (gradient components) and (div Phi)(x_T)."""
    rows = []
    zero = (0,) * dim
    if mask & F_GRAD:
        for k in range(dim):
            rows.append([1.0 if (e == zero and c == k) else 0.0 for e, c in basis])
    if mask & F_LAPLACIAN:
        unit = [tuple(1 if i == k else 0 for i in range(dim)) for k in range(dim)]
        rows.append([1.0 / eps if e == unit[c] else 0.0 for e, c in basis])
    return np.array(rows)


def staggered_target(xs, xt, eps: float, p: int, m: int, mask: int):
    """(alpha [F, N], beta [F]) of one target."""
    dim = xs.shape[1]
    basis = vector_basis(dim, m)
    Xi = edge_integrals(xs, xt, eps, basis, m + 1)
    r = np.sqrt(np.sum(((xs - xt) / eps) ** 2, axis=1))
    w = np.where(r < 1.0, (1.0 - r) ** p, 0.0)
    sw = np.sqrt(w)
    # c = A_s^+ B_s rho = (W^1/2 Xi)^+ W^1/2 rho
    Rmap = np.linalg.pinv(sw[:, None] * Xi, rcond=RCOND) * sw[None, :]  # [Q_v, N]
    alpha = functionals(dim, basis, mask, eps) @ Rmap
    return alpha, -alpha.sum(axis=1)


def stencils_staggered(src, tgt, m: int, mask: int, p: int, eps, row_ptr, col):
    """Weights in the library's layout (target t owns F*row_ptr[t]...,
    entry f*N + j) and target weights beta [n_tgt, F]."""
    src = np.asarray(src, dtype=np.float64)
    tgt = np.asarray(tgt, dtype=np.float64)
    dim = src.shape[1]
    F = (dim if mask & F_GRAD else 0) + (1 if mask & F_LAPLACIAN else 0)
    w = np.zeros(F * int(row_ptr[-1]))
    beta = np.zeros((tgt.shape[0], F))
    for t in range(tgt.shape[0]):
        b, e = int(row_ptr[t]), int(row_ptr[t + 1])
        alpha, bt = staggered_target(src[col[b:e]], tgt[t], float(eps[t]), p, m, mask)
        w[F * b:F * e] = alpha.reshape(-1)
        beta[t] = bt
    return w, beta, F
