"""Pins for the oracle's stencils, alpha = W P (P^T W P)^{-1} lambda
(Section 2.1 normal equations; Section 2.5 functionals on the basis).

Each test checks the oracle against something other than itself:
polynomial reproduction with closed-form derivatives (the definition of
order-m reproduction, Section 2.1), the paper's manufactured fields
(Section 4.1), sum rules, the unisolvent and five-point-Laplacian closed
forms, 40-digit mpmath evaluation of the defining formula, LAPACK's
minimum-norm solver, and basis invariance of the divergence-free span
(Section 2.2, including the paper's own 2D list)."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import divfree
from tests import polytools as pt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F_VALUE, F_GRAD, F_LAP, F_DIV = 1, 2, 4, 8


def knn_case(pts, k, eps_mult=1.5):
    return oracle.knn(pts, pts, k, eps_mult)


def rows_of(w, rp, t, F, C):
    n = rp[t + 1] - rp[t]
    return w[F * C * rp[t]: F * C * rp[t + 1]].reshape(F, n, C)


def interior(pts, margin):
    return np.where(np.all((pts > margin) & (pts < 1 - margin), axis=1))[0]


# --------------------------------------------------------------------------
# P1: polynomial reproduction of order m with closed-form derivatives
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim,order,k,n", [(2, 2, 12, 1000), (2, 4, 40, 4000), (3, 2, 30, 3000),
                                           (3, 3, 60, 8000), (3, 4, 100, 8000)])
def test_polynomial_reproduction(dim, order, k, n):
    pts = W.jittered_grid(n, dim, 100 + order)
    rp, col, eps = knn_case(pts, k)
    mask = F_VALUE | F_GRAD | F_LAP
    w, st, F, C = oracle.stencils(pts, pts, order, "scalar", mask, 4, eps, rp, col)
    assert not st.any()
    g = W.rng(2002)
    polys = [pt.random_poly(dim, order, g) for _ in range(4)]
    tsel = np.arange(0, n, max(1, n // 150))
    for q in polys:
        funcs = [q] + [pt.deriv(q, i) for i in range(dim)] + [pt.laplacian(q, dim)]
        qv = pt.evaluate(q, pts)
        for t in tsel:
            a = rows_of(w, rp, t, F, C)[:, :, 0]
            vals = qv[col[rp[t]:rp[t + 1]]]
            got = a @ vals
            want = np.array([pt.evaluate(f, pts[t:t + 1])[0] for f in funcs])
            scale = np.abs(a) @ np.abs(vals) + np.abs(want)
            assert np.all(np.abs(got - want) <= 1e-10 * scale), (t, got - want)


# --------------------------------------------------------------------------
# P2 + P3: moment conditions, range condition, sum rules
# --------------------------------------------------------------------------
def scaled_basis(dim, order, s):
    ex = W.monomial_exponents(dim, order)
    from math import factorial

    P = np.ones((s.shape[0], len(ex)))
    for a, e in enumerate(ex):
        for i in range(dim):
            P[:, a] *= s[:, i] ** e[i] / factorial(e[i])
    return P, ex


def test_moment_range_and_sum_rules():
    dim, order, k = 3, 3, 50
    pts = W.jittered_grid(5000, dim, 77)
    rp, col, eps = knn_case(pts, k)
    mask = F_VALUE | F_GRAD | F_LAP
    w, st, F, C = oracle.stencils(pts, pts, order, "scalar", mask, 4, eps, rp, col)
    for t in range(0, 5000, 97):
        nb = col[rp[t]:rp[t + 1]]
        s = (pts[nb] - pts[t]) / eps[t]
        r = np.sqrt((s * s).sum(1))
        wt = np.where(r < 1, (1 - r) ** 4, 0.0)
        P, ex = scaled_basis(dim, order, s)
        a = rows_of(w, rp, t, F, C)[:, :, 0]
        # lambda of value, d/dx_i, Laplacian on the scaled basis
        lam = np.zeros((F, len(ex)))
        lam[0, ex.index((0,) * dim)] = 1.0
        for i in range(dim):
            e = [0] * dim
            e[i] = 1
            lam[1 + i, ex.index(tuple(e))] = 1.0 / eps[t]
            e[i] = 2
            lam[1 + dim, ex.index(tuple(e))] += 1.0 / eps[t] ** 2
        mom = a @ P
        assert np.all(np.abs(mom - lam) <= 1e-11 * (np.abs(a) @ np.abs(P) + np.abs(lam)))
        # range: alpha in range(W P)
        WP = wt[:, None] * P
        for f in range(F):
            y, *_ = np.linalg.lstsq(WP, a[f], rcond=None)
            assert np.linalg.norm(WP @ y - a[f]) <= 1e-10 * np.linalg.norm(a[f])
        # sum rules
        d = pts[nb] - pts[t]
        assert abs(a[0].sum() - 1.0) < 1e-12
        for i in range(dim):
            assert abs(a[1 + i].sum()) <= 1e-12 * np.abs(a[1 + i]).sum()
            assert abs(a[1 + i] @ d[:, i] - 1.0) < 1e-11
        assert abs(a[1 + dim].sum()) <= 1e-12 * np.abs(a[1 + dim]).sum()


# --------------------------------------------------------------------------
# P4: the paper's manufactured fields (Section 4.1)
# --------------------------------------------------------------------------
def golden():
    with open(os.path.join(GOLDEN, "manufactured_fields.json")) as f:
        return json.load(f)


def test_golden_fields_closed_forms():
    """The hand-derived derivatives in the fixture match the printed fields."""
    G = golden()
    for name in ("v2", "v4"):
        comps = [pt.from_terms(c) for c in G[name]["components"]]
        for c in range(3):
            assert pt.same(pt.laplacian(comps[c], 3), pt.from_terms(G[name]["laplacian"][c]))
        assert pt.add(*[pt.deriv(comps[c], c) for c in range(3)]) == {}
    for name in ("phi2", "phi4"):
        phi = pt.from_terms(G[name]["field"])
        assert pt.same(pt.laplacian(phi, 3), pt.from_terms(G[name]["laplacian"]))
    phi = pt.from_terms(G["phi2"]["field"])
    for i in range(3):
        assert pt.same(pt.deriv(phi, i), pt.from_terms(G["phi2"]["gradient"][i]))


@pytest.mark.parametrize("name,order,k,n", [("v2", 2, 60, 8000), ("v4", 4, 170, 27000)])
def test_divfree_reproduces_manufactured_velocity(name, order, k, n):
    G = golden()[name]
    pts = W.jittered_grid(n, 3, 1003)
    tsel = interior(pts, 0.2)[::max(1, len(interior(pts, 0.2)) // 12)][:12]
    rp, col, eps = oracle.knn(pts, pts[tsel], k, 1.5)
    mask = F_VALUE | F_LAP | F_DIV
    w, st, F, C = oracle.stencils(pts, pts[tsel], order, "divfree", mask, 6 if order == 4 else 4, eps, rp, col)
    assert not st.any() and F == 7 and C == 3
    comps = [pt.from_terms(c) for c in G["components"]]
    laps = [pt.from_terms(c) for c in G["laplacian"]]
    for q, t in enumerate(tsel):
        a = rows_of(w, rp, q, F, C)
        nb = col[rp[q]:rp[q + 1]]
        V = np.stack([pt.evaluate(c, pts[nb]) for c in comps], 1)  # [N, 3]
        got = np.einsum("fjc,jc->f", a, V)
        x = pts[t:t + 1]
        want = np.array([pt.evaluate(c, x)[0] for c in comps] + [pt.evaluate(c, x)[0] for c in laps] + [0.0])
        scale = np.einsum("fjc,jc->f", np.abs(a), np.abs(V)) + np.abs(want)
        scale[6] = scale[3]  # identically-zero row: judged on the Laplacian's scale
        assert np.all(np.abs(got - want) <= 1e-10 * scale), (q, got - want)
        # divergence row: exactly zero on the divergence-free span
        assert np.abs(a[6]).max() <= 1e-12 * np.abs(a[3]).max()


@pytest.mark.parametrize("name,order,k,n", [("phi2", 3, 60, 8000), ("phi4", 3, 60, 8000), ("phi4", 4, 100, 8000)])
def test_scalar_reproduces_manufactured_pressure(name, order, k, n):
    G = golden()[name]
    pts = W.jittered_grid(n, 3, 1004)
    rp, col, eps = knn_case(pts, k)
    w, st, F, C = oracle.stencils(pts, pts, order, "scalar", F_GRAD | F_LAP, 4, eps, rp, col)
    phi = pt.from_terms(G["field"])
    funcs = [pt.deriv(phi, i) for i in range(3)] + [pt.from_terms(G["laplacian"])]
    pv = pt.evaluate(phi, pts)
    for t in range(0, n, 211):
        a = rows_of(w, rp, t, F, C)[:, :, 0]
        v = pv[col[rp[t]:rp[t + 1]]]
        got = a @ v
        want = np.array([pt.evaluate(f, pts[t:t + 1])[0] for f in funcs])
        assert np.all(np.abs(got - want) <= 1e-10 * (np.abs(a) @ np.abs(v) + np.abs(want)))


# --------------------------------------------------------------------------
# P5: unisolvent case N = Q, the weights do not depend on the kernel
# --------------------------------------------------------------------------
def test_unisolvent_independent_of_kernel():
    g = W.rng(5)
    src = g.uniform(size=(6, 2)) * 0.1 + 0.45
    tgt = np.array([[0.5, 0.5]])
    rp = np.array([0, 6], np.int64)
    col = np.arange(6, dtype=np.int32)
    eps = np.array([0.2])
    mask = F_VALUE | F_GRAD | F_LAP
    w4, _, F, _ = oracle.stencils(src, tgt, 2, "scalar", mask, 4, eps, rp, col)
    w6, _, _, _ = oracle.stencils(src, tgt, 2, "scalar", mask, 6, eps, rp, col)
    np.testing.assert_allclose(w4, w6, rtol=1e-11, atol=1e-11 * np.abs(w4).max())
    # textbook: alpha = P^{-T} lambda for plain monomials
    X = src - tgt
    P = np.stack([np.ones(6), X[:, 0], X[:, 1], X[:, 0] ** 2, X[:, 0] * X[:, 1], X[:, 1] ** 2], 1)
    lam = np.array([[1, 0, 0, 0, 0, 0], [0, 1, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0], [0, 0, 0, 2, 0, 2]], float)
    ref = np.linalg.solve(P.T, lam.T).T
    np.testing.assert_allclose(w4.reshape(F, 6), ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


# --------------------------------------------------------------------------
# P6: nine-point stencil on an exact grid reduces to a 2x2 closed form, and
# to the textbook five-point Laplacian as the corner weight vanishes
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p", [2, 4, 6, 40])
def test_grid_laplacian_closed_form(p):
    h = 0.1
    ax = np.arange(-1, 2) * h
    src = np.array([[x, y] for y in ax for x in ax]) + 0.5
    tgt = np.array([[0.5, 0.5]])
    rp, col, eps = oracle.knn(src, tgt, 9, 1.5)
    w, st, F, C = oracle.stencils(src, tgt, 2, "scalar", F_LAP, p, eps, rp, col)
    d = np.sqrt(((src[col] - tgt) ** 2).sum(1))
    e = eps[0]
    we, wc = (1 - h / e) ** p, (1 - np.sqrt(2) * h / e) ** p
    # alpha_j = w_j (mu0 + mu2 r_j^2): centre a0 = mu0, edge ae, corner ac;
    # a0 + 4 ae + 4 ac = 0 and ae + 2 ac = 1/h^2
    A = np.array([[1 + 4 * we + 4 * wc, 4 * we * h * h + 8 * wc * h * h],
                  [we + 2 * wc, we * h * h + 4 * wc * h * h]])
    mu0, mu2 = np.linalg.solve(A, [0.0, 1 / h ** 2])
    wts = np.where(d < 1e-12, 1.0, np.where(d < 1.2 * h, we, wc))
    ref = wts * (mu0 + mu2 * d * d)
    np.testing.assert_allclose(w, ref, rtol=1e-11, atol=1e-11 / h ** 2)
    if p == 40:
        five = np.where(d < 1e-12, -4, np.where(d < 1.2 * h, 1, 0)) / h ** 2
        np.testing.assert_allclose(w, five, atol=1e-5 / h ** 2)


# --------------------------------------------------------------------------
# P7: 40-digit evaluation of W P (P^T W P)^{-1} lambda
# --------------------------------------------------------------------------
def mp_stencil(src, x, nb, eps, p, dim, order, mask, basis, T=None):
    import mpmath as mp

    mp.mp.dps = 40
    ex = W.monomial_exponents(dim, order)
    exo = [tuple(e) for e in oracle.monomials(dim, order)]
    rows, wts = [], []
    for j in nb:
        s = [(mp.mpf(src[j, i]) - mp.mpf(x[i])) / mp.mpf(eps) for i in range(dim)]
        r = mp.sqrt(sum(v * v for v in s))
        wj = (1 - r) ** p if r < 1 else mp.mpf(0)
        pv = {}
        for e in set(ex) | set(exo):
            v = mp.mpf(1)
            for i in range(dim):
                v *= s[i] ** e[i] / mp.factorial(e[i])
            pv[e] = v
        if basis == "scalar":
            rows.append([pv[e] for e in exo])
            wts.append(wj)
        else:
            for c in range(dim):
                rows.append([sum(mp.mpf(T[a * dim + c, i]) * pv[exo[a]] for a in range(len(exo)) if T[a * dim + c, i] != 0)
                             for i in range(T.shape[1])])
                wts.append(wj)
    P = mp.matrix(rows)
    Wd = mp.diag(wts)
    A = P.T * Wd * P
    lam_rows = []
    ncol = P.cols
    ie = mp.mpf(1) / mp.mpf(eps)
    def dval(e_basis, beta):
        return ie ** sum(beta) if tuple(e_basis) == tuple(beta) else mp.mpf(0)
    if basis == "scalar":
        if mask & F_VALUE:
            lam_rows.append([dval(e, (0,) * dim) for e in exo])
        if mask & F_GRAD:
            for i in range(dim):
                b = [0] * dim; b[i] = 1
                lam_rows.append([dval(e, b) for e in exo])
        if mask & F_LAP:
            lam_rows.append([sum(dval(e, [2 if q == i else 0 for q in range(dim)]) for i in range(dim)) for e in exo])
    else:
        def comp_row(c, betas):
            return [sum(mp.mpf(T[a * dim + c, i]) * dval(exo[a], b) for a in range(len(exo)) for b in betas
                        if T[a * dim + c, i] != 0) for i in range(ncol)]
        if mask & F_LAP:
            for c in range(dim):
                lam_rows.append(comp_row(c, [[2 if q == i else 0 for q in range(dim)] for i in range(dim)]))
    out = []
    for lr in lam_rows:
        y = mp.lu_solve(A, mp.matrix(lr))
        a = Wd * P * y
        out.append([float(v) for v in a])
    return np.array(out)


@pytest.mark.parametrize("case", ["2d_m2", "3d_m3", "3d_divfree_m2"])
def test_mpmath_high_precision(case):
    if case == "2d_m2":
        dim, order, k, basis, mask, p, n = 2, 2, 12, "scalar", F_VALUE | F_GRAD | F_LAP, 4, 1000
    elif case == "3d_m3":
        dim, order, k, basis, mask, p, n = 3, 3, 40, "scalar", F_GRAD | F_LAP, 4, 3000
    else:
        dim, order, k, basis, mask, p, n = 3, 2, 30, "divfree", F_LAP, 4, 3000
    pts = W.jittered_grid(n, dim, 300)
    tsel = np.array([0, n // 3, n // 2 + 7])
    rp, col, eps = oracle.knn(pts, pts[tsel], k, 1.5)
    T = divfree.explicit_basis(dim, order) if basis == "divfree" else None
    w, st, F, C = oracle.stencils(pts, pts[tsel], order, basis, mask, p, eps, rp, col)
    for q, t in enumerate(tsel):
        nb = col[rp[q]:rp[q + 1]]
        ref = mp_stencil(pts, pts[t], nb, eps[q], p, dim, order, mask, basis, T)
        got = rows_of(w, rp, q, F, C).reshape(F, -1)
        for f in range(F):
            assert np.linalg.norm(got[f] - ref[f]) <= 1e-12 * np.linalg.norm(ref[f]), (case, q, f)


# --------------------------------------------------------------------------
# P8: any spanning set of the divergence-free space gives the same stencil
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim,order,k,n", [(2, 2, 12, 1000), (3, 2, 40, 4000), (3, 4, 120, 8000)])
def test_divfree_basis_invariance(dim, order, k, n):
    pts = W.jittered_grid(n, dim, 400)
    tsel = np.arange(0, n, n // 20)
    rp, col, eps = oracle.knn(pts, pts[tsel], k, 1.5)
    mask = F_VALUE | F_LAP | F_DIV
    bases = [divfree.nullspace_basis(dim, order), divfree.explicit_basis(dim, order)]
    if (dim, order) == (2, 2):
        bases.append(divfree.paper_2d_order2())
    assert all(b.shape[1] == divfree.dimension(dim, order) for b in bases)
    assert all(np.abs(divfree.divergence_matrix(dim, order) @ b).max() < 1e-12 for b in bases)
    outs = [oracle.stencils(pts, pts[tsel], order, "divfree", mask, 4, eps, rp, col, T=b) for b in bases]
    F, C = outs[0][2], outs[0][3]
    for q in range(len(tsel)):
        ref = rows_of(outs[0][0], rp, q, F, C).reshape(F, -1)
        for o in outs[1:]:
            got = rows_of(o[0], rp, q, F, C).reshape(F, -1)
            for f in range(F - 1):
                assert np.linalg.norm(got[f] - ref[f]) <= 1e-11 * np.linalg.norm(ref[f])
            assert np.abs(got[F - 1]).max() <= 1e-11 * np.abs(ref[dim]).max()


# --------------------------------------------------------------------------
# P9: LAPACK minimum-norm solver on the same weighted matrix
# --------------------------------------------------------------------------
def test_lapack_minimum_norm_cross_check():
    dim, order, k = 3, 4, 120
    pts = W.jittered_grid(8000, dim, 500)
    rp, col, eps = knn_case(pts, k)
    w, st, F, C = oracle.stencils(pts, pts, order, "scalar", F_LAP, 6, eps, rp, col)
    for t in range(0, 8000, 331):
        nb = col[rp[t]:rp[t + 1]]
        s = (pts[nb] - pts[t]) / eps[t]
        r = np.sqrt((s * s).sum(1))
        sw = np.sqrt(np.where(r < 1, (1 - r) ** 6, 0.0))
        P, ex = scaled_basis(dim, order, s)
        lam = np.zeros(len(ex))
        for i in range(dim):
            e = [0] * dim
            e[i] = 2
            lam[ex.index(tuple(e))] = 1 / eps[t] ** 2
        beta, *_ = np.linalg.lstsq((sw[:, None] * P).T, lam, rcond=None)
        ref = sw * beta
        got = rows_of(w, rp, t, F, C)[0, :, 0]
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


# --------------------------------------------------------------------------
# rank-deficient targets are flagged and get NaN weights
# --------------------------------------------------------------------------
def test_rank_deficient_flags():
    pts = W.jittered_grid(400, 2, 9)
    rp, col, eps = oracle.knn(pts, pts, 5, 1.5)  # N = 5 < Q = 6
    w, st, F, C = oracle.stencils(pts, pts, 2, "scalar", F_LAP, 4, eps, rp, col)
    assert st.all() and np.isnan(w).all()
    g = W.rng(4)
    flat = g.uniform(size=(500, 3))
    flat[:, 2] = 0.25  # coplanar cloud: z-monomials vanish
    rp, col, eps = oracle.knn(flat, flat, 30, 1.5)
    w, st, F, C = oracle.stencils(flat, flat, 2, "scalar", F_LAP, 4, eps, rp, col)
    assert st.all()


# --------------------------------------------------------------------------
# Duplicate points: repeated rows of the weighted sample matrix
# --------------------------------------------------------------------------
def test_duplicate_points():
    """Each point three times over.  Twelve neighbours are four distinct
    points, fewer than the six functions of order 2 in 2D: every target is
    rank deficient although N >= Q.  Thirty neighbours are the ten nearest
    distinct points three times; tripling every row triples the Gram, so each
    copy's weight is one third of the weight on the distinct cloud with ten
    neighbours (the same support radius), and the copies of a point sum to it."""
    base = W.jittered_grid(400, 2, 31)
    pts = np.repeat(base, 3, axis=0)
    mask = F_GRAD | F_LAP
    rp, col, eps = oracle.knn(pts, pts, 12, 1.5)
    w, st, F, C = oracle.stencils(pts, pts, 2, "scalar", mask, 4, eps, rp, col)
    assert (st == 1).all() and np.isnan(w).all()
    rp, col, eps = oracle.knn(pts, pts, 30, 1.5)
    w, st, F, C = oracle.stencils(pts, pts, 2, "scalar", mask, 4, eps, rp, col)
    brp, bcol, beps = oracle.knn(base, base, 10, 1.5)
    bw, bst, _, _ = oracle.stencils(base, base, 2, "scalar", mask, 4, beps, brp, bcol)
    assert not st.any() and not bst.any()
    for t in range(0, len(pts), 7):
        b = t // 3
        assert eps[t] == beps[b]
        a = rows_of(w, rp, t, F, C)[:, :, 0]
        src = col[rp[t]:rp[t + 1]] // 3
        summed = np.zeros((F, len(base)))
        np.add.at(summed.T, src, a.T)
        ref = rows_of(bw, brp, b, F, C)[:, :, 0]
        got = summed[:, bcol[brp[b]:brp[b + 1]]]
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        # the three copies of a point (adjacent: equal distances, ties by index) carry equal weights
        trip = a.reshape(F, -1, 3)
        assert np.array_equal(src.reshape(-1, 3), np.repeat(src[::3, None], 3, axis=1))
        assert np.abs(trip - trip[:, :, :1]).max() <= 1e-12 * np.abs(a).max()


# --------------------------------------------------------------------------
# P10: convergence of the stencils on refining clouds (Section 2.5: a
# derivative D^beta of an order-m fit converges as h^(m+1-|beta|))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim,order,k,sides", [(2, 2, 12, (20, 40, 80)), (2, 4, 30, (20, 40, 80)),
                                                (3, 2, 30, (10, 16, 24)), (3, 3, 50, (10, 16, 24))])
def test_convergence_order(dim, order, k, sides):
    """u = prod_d sin(pi x_d) (the paper's manufactured field of Section 4.2
    scaled to the unit box) on jittered grids of spacing h = 1/n: the RMS
    error of the x-derivative and Laplacian stencils over the targets in the
    middle of the box falls at least as h^(m+1-|beta|), with 0.3 of slack on
    the fitted log-log slope.  (The Laplacian of an even order can converge
    faster on these quasi-uniform clouds, so only the lower bound is held.)
    A wrong power of eps, a dropped term or a wrong functional changes the
    slope by a whole order or stops the convergence."""
    hs, eg, el = [], [], []
    for n in sides:
        pts = W.jittered_grid(n ** dim, dim, 7)
        rp, col, eps = knn_case(pts, k)
        w, st, F, C = oracle.stencils(pts, pts, order, "scalar", F_GRAD | F_LAP, 4, eps, rp, col)
        assert not st.any()
        u = np.prod(np.sin(np.pi * pts), axis=1)
        gx = np.pi * np.cos(np.pi * pts[:, 0]) * np.prod(np.sin(np.pi * pts[:, 1:]), axis=1)
        lap = -dim * np.pi ** 2 * u
        inner = np.where(np.all((pts > 0.3) & (pts < 0.7), axis=1))[0]
        g, lp = [], []
        for t in inner:
            a = rows_of(w, rp, t, F, C)[:, :, 0]
            v = u[col[rp[t]:rp[t + 1]]]
            g.append(a[0] @ v - gx[t])
            lp.append(a[F - 1] @ v - lap[t])
        hs.append(1.0 / n)
        eg.append(np.sqrt(np.mean(np.square(g))))
        el.append(np.sqrt(np.mean(np.square(lp))))
    slope_g = np.polyfit(np.log(hs), np.log(eg), 1)[0]
    slope_l = np.polyfit(np.log(hs), np.log(el), 1)[0]
    assert slope_g >= order - 0.3, (slope_g, eg)
    assert slope_l >= order - 1 - 0.3, (slope_l, el)
    assert eg[-1] < eg[0] and el[-1] < el[0]
