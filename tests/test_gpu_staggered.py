"""Staggered stencils on the GPU (FP64 Householder path, constant monomial
dropped) against the staggered oracle (vector basis, edge-integral sample
matrix, pseudo-inverse): weights and target weights per target and
functional row, gate 1e-10 of the row norm, relaxed to 4 cond 2^-53 for the
one-sided neighbourhoods of targets near the cloud's boundary (cond of the
weighted sample matrix of the scalar monomials of degree 1..m+1).  Also: the
stencils reproduce a polynomial of degree m+1 on the GPU side alone, and the
entry point refuses what it does not compute."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import staggered as S
from oracle.constrained import exponents
from tests import polytools as PT
from tests.gpu_helpers import ctx, dev, flush, host, require_gpu, row_errors

pytestmark = pytest.mark.gpu

TOL = 1e-10
GRAD_LAP = 2 | 4


def case(dim, k, n_tgt, seed):
    src = W.jittered_grid(6000 if dim == 2 else 20000, dim, seed)
    tgt = src[W.rng(seed + 1).choice(len(src), size=n_tgt, replace=False)]
    rp, col, eps = oracle.knn(src, tgt, k, 1.5)
    return src, tgt, rp, col, eps


def cond_reduced(src, tgt, rp, col, eps, dim, m):
    ex = [tuple(int(v) for v in e[:dim]) for e in exponents(dim, m + 1)][1:]
    out = np.empty(len(tgt))
    for t in range(len(tgt)):
        s = (src[col[rp[t]:rp[t + 1]]] - tgt[t]) / eps[t]
        r = np.linalg.norm(s, axis=1)
        sw = np.sqrt(np.where(r < 1, (1 - r) ** 4, 0.0))
        out[t] = np.linalg.cond(sw[:, None] * np.stack([S.monomial(s, e) for e in ex], axis=1))
    return out


@pytest.mark.parametrize("dim,m,k,n_tgt,qr", [(2, 1, 16, 300, -1), (2, 2, 30, 300, -1), (2, 3, 45, 257, -1),
                                              (3, 0, 12, 200, -1), (3, 1, 30, 300, -1), (3, 2, 60, 300, -1),
                                              (3, 3, 110, 130, -1), (3, 2, 60, 300, 1), (3, 2, 60, 300, 2),
                                              (3, 3, 110, 130, 1), (3, 3, 110, 130, 2), (2, 3, 45, 257, 2)])
def test_staggered_parity(dim, m, k, n_tgt, qr):
    """qr: the FP64 QR kernel's shape candidate (-1: the default)."""
    G = require_gpu()
    src, tgt, rp, col, eps = case(dim, k, n_tgt, 60 + m)
    flush(f"staggered dim={dim} m={m} k={k} n_tgt={n_tgt} qr shape {qr}")
    c = ctx()
    c.set_option(G.OPT_QR_SHAPE, qr)
    try:
        w, tw, st, _ = G.gmls_stencils_staggered(c, dev(src), dev(tgt), m, GRAD_LAP, 4, dev(eps), dev(rp), dev(col))
    finally:
        c.set_option(G.OPT_QR_SHAPE, -1)
    w, tw, st = host(w), host(tw), host(st)
    ow, ob, F = S.stencils_staggered(src, tgt, m, GRAD_LAP, 4, eps, rp, col)
    assert (st == 0).all()
    errs = row_errors(w, ow, rp, F, 1)
    # target weights relative to the norm of the functional row
    scale = np.array([[np.hypot(np.linalg.norm(ow[F * rp[t] + f * (rp[t + 1] - rp[t]):
                                                   F * rp[t] + (f + 1) * (rp[t + 1] - rp[t])]), ob[t, f])
                       for f in range(F)] for t in range(len(tgt))])
    berr = np.abs(tw - ob) / np.where(scale > 0, scale, 1.0)
    cond = cond_reduced(src, tgt, rp, col, eps, dim, m)
    tol = np.maximum(TOL, 4 * cond * 2.0 ** -53)[:, None]
    flush(f"  max rel err weights {errs.max():.3e} target weights {berr.max():.3e} max cond {cond.max():.2e}")
    assert np.all(errs <= tol) and np.all(berr <= tol)


@pytest.mark.parametrize("dim,m,k", [(2, 2, 30), (3, 2, 60)])
def test_staggered_reproduces_degree_m_plus_1(dim, m, k):
    """GPU stencils alone: gradient and Laplacian of random polynomials of
    degree m+1 at every target (closed forms), 1e-10 of the rounding scale."""
    G = require_gpu()
    src, tgt, rp, col, eps = case(dim, k, 400, 90)
    w, tw, st, _ = G.gmls_stencils_staggered(ctx(), dev(src), dev(tgt), m, GRAD_LAP, 4, dev(eps), dev(rp), dev(col))
    w, tw = host(w), host(tw)
    F = dim + 1
    g = W.rng(91)
    worst = 0.0
    for _ in range(3):
        q = PT.random_poly(dim, m + 1, g)
        exact = np.stack([PT.evaluate(PT.deriv(q, i), tgt) for i in range(dim)] +
                         [PT.evaluate(PT.laplacian(q, dim), tgt)], axis=1)
        u = PT.evaluate(q, src)
        ut = PT.evaluate(q, tgt)
        for t in range(len(tgt)):
            a = w[F * rp[t]:F * rp[t + 1]].reshape(F, -1)
            uj = u[col[rp[t]:rp[t + 1]]]
            got = a @ uj + tw[t] * ut[t]
            scale = np.abs(a * uj).sum(axis=1) + np.abs(tw[t] * ut[t]) + np.abs(exact[t])
            worst = max(worst, float((np.abs(got - exact[t]) / scale).max()))
    flush(f"  staggered reproduction worst {worst:.3e}")
    assert worst <= 1e-10


def test_staggered_refusals_and_empty():
    G = require_gpu()
    src, tgt, rp, col, eps = case(2, 16, 20, 5)
    args = (dev(eps), dev(rp), dev(col))
    for mask in (1 | 2, 8):  # value and divergence are not staggered functionals: GMLS_ERR_ARG
        with pytest.raises(G.GmlsError) as e:
            G.gmls_stencils_staggered(ctx(), dev(src), dev(tgt), 1, mask, 4, *args)
        assert e.value.status == 1
    src3, tgt3, rp3, col3, eps3 = case(3, 110, 10, 7)
    with pytest.raises(G.GmlsError) as e:  # degree 4 in 3-D: 34 columns, beyond the mixed pipeline
        G.gmls_stencils_staggered(ctx(), dev(src3), dev(tgt3), 3, GRAD_LAP, 4, dev(eps3), dev(rp3), dev(col3),
                                  prec=G.PREC_MIXED)
    assert e.value.status == G.GMLS_ERR_UNSUPPORTED
    with pytest.raises(G.GmlsError) as e:
        G.gmls_stencils_staggered(ctx(), dev(src), dev(tgt), 4, GRAD_LAP, 4, *args)
    assert e.value.status == G.GMLS_ERR_UNSUPPORTED
    empty = np.zeros((0, 2))
    w, tw, st, _ = G.gmls_stencils_staggered(ctx(), dev(src), dev(empty), 1, GRAD_LAP, 4, dev(np.zeros(0)),
                                             dev(np.zeros(1, dtype=np.int64)), dev(np.zeros(0, dtype=np.int32)))
    assert w.numel() == 0 and tw.shape[0] == 0 and st.numel() == 0


@pytest.mark.parametrize("dim,m,k,n_tgt", [(2, 1, 16, 300), (2, 2, 30, 300), (2, 3, 45, 257), (3, 1, 30, 300),
                                           (3, 2, 60, 300)])
def test_staggered_mixed_parity(dim, m, k, n_tgt):
    """The mixed pipeline with the constant column dropped: gate 1e-8
    (targets it hands to the FP64 fallback meet the FP64 gate anyway)."""
    G = require_gpu()
    src, tgt, rp, col, eps = case(dim, k, n_tgt, 70 + m)
    flush(f"staggered mixed dim={dim} m={m} k={k}")
    w, tw, st, rep = G.gmls_stencils_staggered(ctx(), dev(src), dev(tgt), m, GRAD_LAP, 4, dev(eps), dev(rp),
                                               dev(col), prec=G.PREC_MIXED, report=True)
    w, tw, st = host(w), host(tw), host(st)
    ow, ob, F = S.stencils_staggered(src, tgt, m, GRAD_LAP, 4, eps, rp, col)
    assert not (st == 1).any()
    errs = row_errors(w, ow, rp, F, 1)
    scale = np.array([[np.hypot(np.linalg.norm(ow[F * rp[t] + f * (rp[t + 1] - rp[t]):
                                                   F * rp[t] + (f + 1) * (rp[t + 1] - rp[t])]), ob[t, f])
                       for f in range(F)] for t in range(len(tgt))])
    berr = np.abs(tw - ob) / np.where(scale > 0, scale, 1.0)
    flush(f"  max rel err weights {errs.max():.3e} target weights {berr.max():.3e} fallback {rep['n_fallback']}")
    assert errs.max() <= 1e-8 and berr.max() <= 1e-8


def test_staggered_autotune_then_parity():
    """Tuning the staggered QR kernel (GMLS_TUNE_STAGGERED); the next call
    takes the tuned shapes and stays within the gate."""
    G = require_gpu()
    dim, m, k, n_tgt = 3, 2, 60, 300
    src, tgt, rp, col, eps = case(dim, k, n_tgt, 60 + m)
    c = G.Context(0)
    args = (dev(src), dev(tgt), m, GRAD_LAP, 4, dev(eps), dev(rp), dev(col))
    res = G.gmls_autotune(c, args[0], args[1], m, G.TUNE_STAGGERED, GRAD_LAP, 4, args[5], args[6], args[7], reps=1)
    flush(f"  {res}")
    assert sorted(res) == ["qr"]
    w, tw, st, _ = G.gmls_stencils_staggered(c, *args)
    w, tw = host(w), host(tw)
    ow, ob, F = S.stencils_staggered(src, tgt, m, GRAD_LAP, 4, eps, rp, col)
    cond = cond_reduced(src, tgt, rp, col, eps, dim, m)
    tol = np.maximum(TOL, 4 * cond * 2.0 ** -53)[:, None]
    assert np.all(row_errors(w, ow, rp, F, 1) <= tol)
    c.close()
