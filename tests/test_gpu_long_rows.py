"""Rows of more than 256 neighbours (Section 2.1: the neighbour set is every
particle inside the support, with no bound on its size).

A clustered cloud (a dense Gaussian blob in a uniform background) under a
fixed-radius search gives rows from a few dozen to several hundred
neighbours (up to about 800 at the centre of the blob; the background is
floored to 45, more than twice the 20 functions of order 3).  Every precision and scheme must match the FP64 oracle on the
GPU's own rows: the FP64 QR path factors the long rows chunk by chunk (a
tall-skinny QR), the mixed pipeline loops its moment and weight kernels over
them, and the wavefront and fused schemes hand them to the FP64 path."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import ctx, dev, flush, host, require_gpu, row_errors

pytestmark = pytest.mark.gpu

FP64_TOL, MIXED_TOL = 1e-10, 1e-8
_cache = {}


def cloud():
    if "c" not in _cache:
        g = W.rng(4242)
        pts = np.concatenate([g.normal(0.5, 0.04, size=(2500, 3)), g.uniform(size=(3500, 3))])
        rp, col, eps = oracle.radius(pts, pts, 0.05, 45)
        _cache["c"] = (pts, rp, col, eps)
    return _cache["c"]


def gpu_rows():
    """The GPU's own search (radius rows are sets; the oracle's stencils are
    taken on the GPU's row order)."""
    G = require_gpu()
    pts, rp, col, eps = cloud()
    s = dev(pts)
    grp, gcol, geps = G.gmls_neighbors(ctx(), s, s, G.SEARCH_RADIUS, radius=0.05, k_min=45)
    grp, gcol, geps = host(grp), host(gcol), host(geps)
    assert np.array_equal(grp, rp) and np.array_equal(geps, eps)
    return pts, grp, gcol, geps


def test_cloud_has_long_rows():
    pts, rp, col, eps = cloud()
    n = np.diff(rp)
    flush(f"rows: min {n.min()} median {int(np.median(n))} max {n.max()}, over 256: {(n > 256).sum()}")
    assert (n > 256).sum() >= 200 and n.max() >= 700 and (n <= 64).sum() >= 100


CASES = [("scalar", 2, 2 | 4), ("scalar", 3, 1 | 4), ("divfree", 2, 1 | 4 | 8)]


@pytest.mark.parametrize("prec,scheme", [("fp64", 0), ("mixed", 0), ("mixed", 1), ("mixed", 2), ("mixed", 4)],
                         ids=["fp64", "mixed-auto", "mixed-rows", "mixed-gram", "mixed-wave"])
@pytest.mark.parametrize("basis,order,mask", CASES, ids=["scalar2", "scalar3", "divfree2"])
def test_long_rows_match_oracle(basis, order, mask, prec, scheme):
    G = require_gpu()
    pts, rp, col, eps = gpu_rows()
    b = G.BASIS_SCALAR if basis == "scalar" else G.BASIS_DIVFREE
    p = G.PREC_FP64 if prec == "fp64" else G.PREC_MIXED
    c = ctx()
    c.set_option(G.OPT_MIXED_SCHEME, scheme)
    s = dev(pts)
    flush(f"long rows {basis} m={order} {prec} scheme {scheme}")
    try:
        gw, gst, rep = G.gmls_stencils(c, s, s, order, b, mask, 4, dev(eps), dev(rp), dev(col), prec=p, report=True)
    except G.GmlsError as e:
        if e.status == 5 and prec == "mixed":  # the scheme is not compiled for this basis/order
            return
        raise
    finally:
        c.set_option(G.OPT_MIXED_SCHEME, 0)
    gw, gst = host(gw), host(gst)
    w, st, F, C = oracle.stencils(pts, pts, order, basis, mask, 4, eps, rp, col)
    assert np.array_equal(gst == 1, st == 1)
    zero = (F - 1,) if basis == "divfree" and mask & 8 else ()
    errs = row_errors(gw, w, rp, F, C, zero_rows=zero)[st != 1]
    n = np.diff(rp)[st != 1]
    flush(f"  max rel err {errs.max():.3e} (rows > 256: {errs[n > 256].max():.3e}) fallback {rep['n_fallback']}")
    assert errs.max() <= (FP64_TOL if prec == "fp64" else MIXED_TOL)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_long_rows_shared_sets(prec):
    """A scalar and a divergence-free set on the same long rows in one call
    (shared factor in FP64, shared moments on the pipeline)."""
    G = require_gpu()
    pts, rp, col, eps = gpu_rows()
    p = G.PREC_FP64 if prec == "fp64" else G.PREC_MIXED
    s = dev(pts)
    sets = [(G.BASIS_SCALAR, G.F_GRAD | G.F_LAPLACIAN), (G.BASIS_DIVFREE, G.F_VALUE | G.F_LAPLACIAN | G.F_DIV)]
    flush(f"long rows shared sets {prec}")
    outs, _ = G.gmls_stencils_multi(ctx(), s, s, 2, 4, dev(eps), dev(rp), dev(col), sets, prec=p)
    for (basis, mask), (gw, gs) in zip(sets, outs):
        name = "scalar" if basis == G.BASIS_SCALAR else "divfree"
        w, st, F, C = oracle.stencils(pts, pts, 2, name, mask, 4, eps, rp, col)
        gs = host(gs)
        assert np.array_equal(gs == 1, st == 1)
        zero = (F - 1,) if name == "divfree" else ()
        errs = row_errors(host(gw), w, rp, F, C, zero_rows=zero)[st != 1]
        flush(f"  {name}: max rel err {errs.max():.3e}")
        assert errs.max() <= (FP64_TOL if prec == "fp64" else MIXED_TOL)


def test_long_rows_staggered_and_constrained():
    """The staggered (Section 2.4) and Neumann-constrained (Section 2.3) calls
    take long rows through the same chunked QR: the 80 longest rows and 40
    others against the (per-target, extended-precision) oracles."""
    G = require_gpu()
    from oracle import constrained as OC
    from oracle import staggered as OS

    pts, rp, col, eps = gpu_rows()
    n = np.diff(rp)
    sel = np.unique(np.concatenate([np.argsort(n)[-80:], np.arange(0, len(pts), len(pts) // 40)]))
    srp = np.zeros(len(sel) + 1, dtype=np.int64)
    srp[1:] = np.cumsum(n[sel])
    scol = np.concatenate([col[rp[t]:rp[t + 1]] for t in sel])
    s = dev(pts)
    nrm = np.zeros_like(pts)
    nrm[::3, 2] = 1.0  # every third target constrained, the others not

    def sub(w, F):
        return np.concatenate([w[F * rp[t]:F * rp[t + 1]] for t in sel])

    flush("long rows staggered")
    gw, gt, gst, _ = G.gmls_stencils_staggered(ctx(), s, s, 1, G.F_GRAD | G.F_LAPLACIAN, 4, dev(eps), dev(rp),
                                               dev(col), prec=G.PREC_FP64)
    ow, oaux, F = OS.stencils_staggered(pts, pts[sel], 1, G.F_GRAD | G.F_LAPLACIAN, 4, eps[sel], srp, scol)
    errs = row_errors(sub(host(gw), F), ow, srp, F, 1)
    flush(f"  max rel err {errs.max():.3e}")
    assert errs.max() <= FP64_TOL
    flush("long rows constrained")
    gw, gh, gst, _ = G.gmls_stencils_constrained(ctx(), s, s, 2, G.F_LAPLACIAN, 4, dev(eps), dev(rp), dev(col),
                                                 dev(nrm))
    ow, oh, F = OC.stencils_constrained(pts, pts[sel], 2, G.F_LAPLACIAN, 4, eps[sel], srp, scol, nrm[sel])
    errs = row_errors(sub(host(gw), F), ow, srp, F, 1)
    flush(f"  max rel err {errs.max():.3e}")
    assert errs.max() <= FP64_TOL


@pytest.mark.parametrize("cand", [1, 2])
@pytest.mark.parametrize("basis,order,mask", [("scalar", 3, 1 | 4), ("divfree", 2, 1 | 4 | 8)],
                         ids=["scalar3", "divfree2"])
def test_long_rows_every_qr_shape(basis, order, mask, cand):
    """The FP64 QR kernel's other shapes (fewer rows per lane, so that every
    bin's rows, and the long rows, are factored in more chunks)."""
    G = require_gpu()
    pts, rp, col, eps = gpu_rows()
    b = G.BASIS_SCALAR if basis == "scalar" else G.BASIS_DIVFREE
    c = ctx()
    c.set_option(G.OPT_QR_SHAPE, cand)
    s = dev(pts)
    flush(f"long rows {basis} m={order} fp64 QR shape {cand}")
    try:
        gw, gst, _ = G.gmls_stencils(c, s, s, order, b, mask, 4, dev(eps), dev(rp), dev(col), prec=G.PREC_FP64)
    finally:
        c.set_option(G.OPT_QR_SHAPE, -1)
    gw, gst = host(gw), host(gst)
    w, st, F, C = oracle.stencils(pts, pts, order, basis, mask, 4, eps, rp, col)
    assert np.array_equal(gst, st)
    zero = (F - 1,) if basis == "divfree" and mask & 8 else ()
    errs = row_errors(gw, w, rp, F, C, zero_rows=zero)[st != 1]
    flush(f"  max rel err {errs.max():.3e}")
    assert errs.max() <= FP64_TOL
