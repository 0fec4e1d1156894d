"""Pins of the Neumann-constrained oracle (oracle/constrained.py) against what
Section 2.3 and the mathematics fix, not against itself:

* the constraint holds exactly: the normal-derivative stencil of the
  constrained fit returns h, whatever u is;
* polynomials of degree <= m with a consistent h are reproduced exactly by
  every functional (value, gradient, Laplacian);
* a zero normal gives the unconstrained stencil of the C oracle (Householder
  QR, a different algorithm);
* an independent null-space solution of the constrained least-squares problem
  (SVD of F^T, then unconstrained least squares) gives the same functional
  values;
* scaling the normal by s leaves alpha and divides beta by s."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import constrained as OC
from tests import polytools as PT

GRAD, VAL_GRAD_LAP = 2, 1 | 2 | 4


def case(dim, order, k, n_src=3000, n_tgt=24, seed=5):
    src = W.jittered_grid(n_src, dim, seed)
    tgt, nrm = W.boundary_points(n_tgt, dim, seed + 1)
    rp, col, eps = oracle.knn(src, tgt, k, 1.5)
    return src, tgt, nrm, rp, col, eps


@pytest.mark.parametrize("dim,order,k", [(2, 2, 20), (3, 2, 40), (3, 3, 60)])
def test_normal_derivative_returns_h(dim, order, k):
    src, tgt, nrm, rp, col, eps = case(dim, order, k)
    w, beta, F = OC.stencils_constrained(src, tgt, order, GRAD, 4, eps, rp, col, nrm)
    for t in range(len(tgt)):
        a = w[F * rp[t]:F * rp[t + 1]].reshape(F, -1)
        an = nrm[t] @ a
        assert np.linalg.norm(an) <= 1e-11 * np.linalg.norm(a)
        assert abs(nrm[t] @ beta[t] - 1.0) <= 1e-11


@pytest.mark.parametrize("dim,order,k", [(2, 3, 30), (3, 2, 40), (3, 3, 60)])
def test_polynomials_with_consistent_h_are_reproduced(dim, order, k):
    src, tgt, nrm, rp, col, eps = case(dim, order, k)
    w, beta, F = OC.stencils_constrained(src, tgt, order, VAL_GRAD_LAP, 4, eps, rp, col, nrm)
    g = W.rng(77)
    worst = 0.0
    for _ in range(4):
        q = PT.random_poly(dim, order, g)
        grads = [PT.deriv(q, i) for i in range(dim)]
        for t in range(len(tgt)):
            x = tgt[t:t + 1]
            u = PT.evaluate(q, src[col[rp[t]:rp[t + 1]]])
            h = sum(nrm[t, i] * PT.evaluate(grads[i], x)[0] for i in range(dim))
            exact = [PT.evaluate(q, x)[0]] + [PT.evaluate(gi, x)[0] for gi in grads] + \
                    [PT.evaluate(PT.laplacian(q, dim), x)[0]]
            a = w[F * rp[t]:F * rp[t + 1]].reshape(F, -1)
            for f in range(F):
                got = a[f] @ u + beta[t, f] * h
                scale = np.abs(a[f] * u).sum() + abs(beta[t, f] * h) + abs(exact[f])
                worst = max(worst, abs(got - exact[f]) / scale)
    assert worst <= 1e-10, worst


def test_zero_normal_is_the_unconstrained_stencil():
    src, tgt, nrm, rp, col, eps = case(3, 3, 60)
    w, beta, F = OC.stencils_constrained(src, tgt, 3, VAL_GRAD_LAP, 4, eps, rp, col, np.zeros_like(nrm))
    wq, st, Fq, _ = oracle.stencils(src, tgt, 3, "scalar", VAL_GRAD_LAP, 4, eps, rp, col)
    assert F == Fq and (st == 0).all() and not beta.any()
    for t in range(len(tgt)):
        a = w[F * rp[t]:F * rp[t + 1]].reshape(F, -1)
        b = wq[F * rp[t]:F * rp[t + 1]].reshape(F, -1)
        assert np.all(np.linalg.norm(a - b, axis=1) <= 1e-11 * np.linalg.norm(b, axis=1))


def test_null_space_solution_agrees():
    dim, order, k, p = 3, 2, 30, 4
    src, tgt, nrm, rp, col, eps = case(dim, order, k, n_tgt=10)
    w, beta, F = OC.stencils_constrained(src, tgt, order, VAL_GRAD_LAP, p, eps, rp, col, nrm)
    ex = OC.exponents(dim, order)
    g = W.rng(9)
    for t in range(len(tgt)):
        xs = src[col[rp[t]:rp[t + 1]]]
        s = (xs - tgt[t]) / eps[t]
        r = np.linalg.norm(s, axis=1)
        sw = np.sqrt(np.where(r < 1, (1 - r) ** p, 0.0))
        P = OC.basis(s, ex)
        lam = OC.functionals(dim, ex, VAL_GRAD_LAP, eps[t])
        Fv = np.zeros(len(ex))
        for kk in range(dim):
            Fv[1 + kk] = nrm[t, kk] / eps[t]
        u = g.standard_normal(len(xs))
        h = g.standard_normal()
        # particular solution of F^T c = h, null space of F^T from the SVD
        c0 = Fv * h / (Fv @ Fv)
        Z = np.linalg.svd(Fv[None, :])[2][1:].T
        tz = np.linalg.lstsq(sw[:, None] * (P @ Z), sw * (u - P @ c0), rcond=None)[0]
        c = c0 + Z @ tz
        a = w[F * rp[t]:F * rp[t + 1]].reshape(F, -1)
        got = a @ u + beta[t] * h
        ref = lam @ c
        assert np.all(np.abs(got - ref) <= 1e-10 * (np.abs(ref) + np.abs(a) @ np.abs(u) + np.abs(beta[t] * h)))


def test_normal_scaling():
    src, tgt, nrm, rp, col, eps = case(3, 2, 40)
    w1, b1, F = OC.stencils_constrained(src, tgt, 2, VAL_GRAD_LAP, 4, eps, rp, col, nrm)
    w2, b2, _ = OC.stencils_constrained(src, tgt, 2, VAL_GRAD_LAP, 4, eps, rp, col, 2.5 * nrm)
    np.testing.assert_allclose(w2, w1, rtol=1e-10, atol=1e-12 * np.abs(w1).max())
    np.testing.assert_allclose(b2, b1 / 2.5, rtol=1e-10, atol=1e-14)


def _mp_target(xs, xt, eps, p, order, mask, normal, dps=60):
    """The bordered system of Section 2.3 formed and solved in 60-digit
    arithmetic (mpmath), from the same FP64 inputs: an independent reference
    whose own error is negligible."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = dps
    dim = xs.shape[1]
    ex = [tuple(int(v) for v in e) for e in OC.exponents(dim, order)]
    Q, N = len(ex), len(xs)
    e = mpmath.mpf(float(eps))
    P, w = [], []
    for j in range(N):
        s = [(mpmath.mpf(float(xs[j, i])) - mpmath.mpf(float(xt[i]))) / e for i in range(dim)]
        r = mpmath.sqrt(mpmath.fsum(v * v for v in s))
        w.append((1 - r) ** p if r < 1 else mpmath.mpf(0))
        P.append([mpmath.fprod(s[i] ** a[i] / mpmath.factorial(a[i]) for i in range(dim)) for a in ex])
    con = bool(np.any(normal))
    K = mpmath.matrix(Q + 1, Q + 1)
    for a in range(Q):
        for b in range(a, Q):
            K[a, b] = K[b, a] = mpmath.fsum(w[j] * P[j][a] * P[j][b] for j in range(N))
    if con:
        for k in range(dim):
            a = ex.index(tuple(1 if i == k else 0 for i in range(3))[:3])
            K[a, Q] = K[Q, a] = mpmath.mpf(float(normal[k])) / e
    else:
        K[Q, Q] = 1
    rows = []
    if mask & 1:
        rows.append({(0, 0, 0): mpmath.mpf(1)})
    if mask & 2:
        rows += [{tuple(1 if i == k else 0 for i in range(3)): 1 / e} for k in range(dim)]
    if mask & 4:
        rows.append({tuple(2 if i == k else 0 for i in range(3)): 1 / e ** 2 for k in range(dim)})
    alpha = np.zeros((len(rows), N))
    beta = np.zeros(len(rows))
    for f, row in enumerate(rows):
        g = mpmath.lu_solve(K, mpmath.matrix([row.get(a, 0) for a in ex] + [0]))
        for j in range(N):
            alpha[f, j] = float(w[j] * mpmath.fsum(P[j][a] * g[a] for a in range(Q)))
        beta[f] = float(g[Q]) if con else 0.0
    return alpha, beta


@pytest.mark.parametrize("dim,order,k,pick", [(3, 4, 90, "worst"), (3, 4, 90, "constrained"), (2, 3, 30, "constrained")])
def test_matches_high_precision_solution(dim, order, k, pick):
    """Gate: 1e-12 of the row norm, relaxed to 2^-53 cond(W^1/2 P) where the
    local problem is worse conditioned than 1e4 (corner targets of a cube face
    with a one-sided neighbourhood reach 3e6 at order 4)."""
    src, tgt, nrm, rp, col, eps = case(dim, order, k, n_src=20000 if dim == 3 else 6000, n_tgt=40, seed=44)
    nrm[::7] = 0.0
    ex = OC.exponents(dim, order)
    conds = []
    for t in range(len(tgt)):
        s = (src[col[rp[t]:rp[t + 1]]] - tgt[t]) / eps[t]
        r = np.linalg.norm(s, axis=1)
        conds.append(np.linalg.cond(np.sqrt(np.where(r < 1, (1 - r) ** 4, 0.0))[:, None] * OC.basis(s, ex)))
    conds = np.array(conds)
    if pick == "worst":
        t = int(np.argmax(conds))
    else:
        t = int(np.flatnonzero(np.any(nrm != 0, axis=1))[0])
    xs = src[col[rp[t]:rp[t + 1]]]
    a, b = OC.constrained_target(xs, tgt[t], float(eps[t]), 4, order, VAL_GRAD_LAP, nrm[t])
    ra, rb = _mp_target(xs, tgt[t], eps[t], 4, order, VAL_GRAD_LAP, nrm[t])
    tol = max(1e-12, conds[t] * 2.0 ** -53)
    scale = np.hypot(np.linalg.norm(ra, axis=1), rb)
    assert np.all(np.linalg.norm(a - ra, axis=1) <= tol * scale), (conds[t], np.linalg.norm(a - ra, axis=1) / scale)
    assert np.all(np.abs(b - rb) <= tol * scale)
