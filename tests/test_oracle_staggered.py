"""Pins of the staggered oracle (oracle/staggered.py) against what Section 2.4
and the mathematics fix:

* the quadrature edge integrals equal their closed form
  xi_(a,k)(x_j) = eps s_k p_a(s) / (|a| + 1), s = (x_j - x_T)/eps;
* the vector basis has exactly the circulating fields as its null space under
  edge integration: rank Xi = Q_s(m+1) - 1 (scalar polynomials of degree
  1..m+1), nullity = d Q_s(m) - rank;
* gradient and Laplacian are reproduced exactly for polynomials of degree
  <= m+1 (one degree above the vector order), including the paper's cubic
  manufactured pressure of Section 4.1 at m = 2;
* an independent derivation (least squares of rho_j = p_j - p(x_T) on the
  scalar monomials of degree 1..m+1, LAPACK lstsq, derivatives at x_T) gives
  the same stencils;
* the weights annihilate constants (sum alpha + beta = 0)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import staggered as S
from oracle.constrained import exponents
from tests import polytools as PT

GRAD_LAP = 2 | 4
HERE = os.path.dirname(os.path.abspath(__file__))


def case(dim, k, n_src=4000, n_tgt=12, seed=3):
    src = W.jittered_grid(n_src, dim, seed)
    g = W.rng(seed + 1)
    tgt = src[g.choice(n_src, size=n_tgt, replace=False)]
    rp, col, eps = oracle.knn(src, tgt, k, 1.5)
    return src, tgt, rp, col, eps


@pytest.mark.parametrize("dim,m", [(2, 1), (2, 3), (3, 2)])
def test_edge_integrals_closed_form(dim, m):
    src, tgt, rp, col, eps = case(dim, 30)
    basis = S.vector_basis(dim, m)
    xs, xt = src[col[rp[0]:rp[1]]], tgt[0]
    Xi = S.edge_integrals(xs, xt, eps[0], basis, m + 1)
    s = (xs - xt) / eps[0]
    ref = np.stack([eps[0] * s[:, k] * S.monomial(s, e) / (sum(e) + 1) for e, k in basis], axis=1)
    np.testing.assert_allclose(Xi, ref, rtol=1e-13, atol=1e-15 * np.abs(ref).max())


@pytest.mark.parametrize("dim,m", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_null_space_is_the_circulating_fields(dim, m):
    src, tgt, rp, col, eps = case(dim, 60)
    basis = S.vector_basis(dim, m)
    Xi = S.edge_integrals(src[col[rp[0]:rp[1]]], tgt[0], eps[0], basis, m + 1)
    sv = np.linalg.svd(Xi, compute_uv=False)
    rank = int((sv > 1e-11 * sv[0]).sum())
    assert rank == math.comb(m + 1 + dim, dim) - 1
    assert len(basis) - rank == dim * math.comb(m + dim, dim) - rank


def _check_reproduction(src, tgt, rp, col, eps, m, polys, dim):
    w, beta, F = S.stencils_staggered(src, tgt, m, GRAD_LAP, 4, eps, rp, col)
    worst = 0.0
    for q in polys:
        grads = [PT.deriv(q, i) for i in range(dim)]
        lap = PT.laplacian(q, dim)
        for t in range(len(tgt)):
            x = tgt[t:t + 1]
            u = PT.evaluate(q, src[col[rp[t]:rp[t + 1]]])
            ut = PT.evaluate(q, x)[0]
            exact = [PT.evaluate(g, x)[0] for g in grads] + [PT.evaluate(lap, x)[0]]
            a = w[F * rp[t]:F * rp[t + 1]].reshape(F, -1)
            for f in range(F):
                got = a[f] @ u + beta[t, f] * ut
                scale = np.abs(a[f] * u).sum() + abs(beta[t, f] * ut) + abs(exact[f])
                worst = max(worst, abs(got - exact[f]) / scale)
    return worst


@pytest.mark.parametrize("dim,m,k", [(2, 1, 16), (2, 2, 30), (2, 3, 45), (3, 1, 30), (3, 2, 60), (3, 3, 110)])
def test_reproduces_one_degree_above_the_order(dim, m, k):
    src, tgt, rp, col, eps = case(dim, k, n_src=6000 if dim == 2 else 20000)
    g = W.rng(50 + m)
    polys = [PT.random_poly(dim, m + 1, g) for _ in range(3)]
    assert _check_reproduction(src, tgt, rp, col, eps, m, polys, dim) <= 1e-10


def test_paper_cubic_pressure_field_at_order_2():
    """Section 4.1's cubic pressure is reproduced by the order-2 staggered
    stencils (gradient and Laplacian 6 + 6z, closed forms in the fixture)."""
    fx = json.load(open(os.path.join(HERE, "golden", "manufactured_fields.json")))["phi2"]
    phi = PT.from_terms(fx["field"])
    src, tgt, rp, col, eps = case(3, 60, n_src=20000)
    w, beta, F = S.stencils_staggered(src, tgt, 2, GRAD_LAP, 4, eps, rp, col)
    grad = [PT.from_terms(gk) for gk in fx["gradient"]]
    lap = PT.from_terms(fx["laplacian"])
    for t in range(len(tgt)):
        x = tgt[t:t + 1]
        u = PT.evaluate(phi, src[col[rp[t]:rp[t + 1]]])
        ut = PT.evaluate(phi, x)[0]
        a = w[F * rp[t]:F * rp[t + 1]].reshape(F, -1)
        exact = [PT.evaluate(gk, x)[0] for gk in grad] + [PT.evaluate(lap, x)[0]]
        for f in range(F):
            got = a[f] @ u + beta[t, f] * ut
            assert abs(got - exact[f]) <= 1e-10 * (np.abs(a[f] * u).sum() + abs(beta[t, f] * ut) + 1.0)


@pytest.mark.parametrize("dim,m,k", [(2, 2, 30), (3, 2, 60), (3, 3, 110)])
def test_matches_reduced_scalar_least_squares(dim, m, k):
    src, tgt, rp, col, eps = case(dim, k, n_src=6000 if dim == 2 else 20000)
    w, beta, F = S.stencils_staggered(src, tgt, m, GRAD_LAP, 4, eps, rp, col)
    ex = [tuple(int(v) for v in e[:dim]) for e in exponents(dim, m + 1)][1:]  # no constant
    for t in range(len(tgt)):
        xs = src[col[rp[t]:rp[t + 1]]]
        s = (xs - tgt[t]) / eps[t]
        r = np.linalg.norm(s, axis=1)
        sw = np.sqrt(np.where(r < 1, (1 - r) ** 4, 0.0))
        P = np.stack([S.monomial(s, e) for e in ex], axis=1)
        # lstsq map rho -> coefficients, then derivatives of the scalar fit at x_T
        Cmap = np.linalg.lstsq(sw[:, None] * P, np.diag(sw), rcond=None)[0]
        rows = []
        for kx in range(dim):
            rows.append([1.0 / eps[t] if e == tuple(1 if i == kx else 0 for i in range(dim)) else 0.0 for e in ex])
        rows.append([1.0 / eps[t] ** 2 if (sum(e) == 2 and max(e) == 2) else 0.0 for e in ex])
        ref = np.array(rows) @ Cmap
        a = w[F * rp[t]:F * rp[t + 1]].reshape(F, -1)
        err = np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)
        assert err.max() <= 1e-10, err
        np.testing.assert_allclose(beta[t], -ref.sum(axis=1), rtol=1e-9, atol=1e-10 * np.abs(ref).sum())


def test_constants_are_annihilated():
    src, tgt, rp, col, eps = case(3, 60, n_src=20000)
    w, beta, F = S.stencils_staggered(src, tgt, 2, GRAD_LAP, 4, eps, rp, col)
    for t in range(len(tgt)):
        a = w[F * rp[t]:F * rp[t + 1]].reshape(F, -1)
        assert np.all(np.abs(a.sum(axis=1) + beta[t]) <= 1e-12 * np.abs(a).sum(axis=1))
