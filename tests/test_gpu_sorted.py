"""The search's cell-ordered source records (gmls_neighbors_sorted) and
stencils gathered from them (GMLS_OPT_SOURCE_STRIDE = 4).

A stencil depends only on the coordinates of its row entries, in row order
(Section 2.1), so stencils on (records, col_sorted) must equal those on
(coords, col) bit for bit.  The search side is checked against its own
definition: the rows are the ones gmls_neighbors returns (and the oracle's),
the records are the sources ordered by cell and index, the same on every
call, and col_sorted[j] points at the record of source col[j]."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import ctx, dev, flush, host, require_gpu, row_sorted

pytestmark = pytest.mark.gpu


def clouds():
    g = W.rng(31)
    return {
        "ramp": W.density_ramp(20000, 1004),
        "clustered": np.concatenate([g.normal(0.5, 0.02, size=(3000, 3)), g.uniform(size=(4000, 3))]),
        "grid2d": W.jittered_grid(4000, 2, 17),
    }


# (cloud, search, option overrides): the one-pass radius search writes
# positions as it goes; the two-pass, index-order and kNN searches and the
# rows deferred to the per-target kernels (floor, crowded cells) are
# translated afterwards
CASES = {
    "radius-onepass": ("ramp", ("radius", 30), {}),
    "radius-twopass": ("ramp", ("radius", 30), {"OPT_RADIUS_SCRATCH_MB": 0}),
    "radius-index": ("ramp", ("radius", 30), {"OPT_ROW_ORDER": 1}),
    "radius-clustered": ("clustered", ("radius", 10, 0.02), {}),
    "radius-floor": ("grid2d", ("radius", 25, 0.01), {}),
    "radius-long": ("grid2d", ("radius", 0, 0.15), {}),
    "knn-3d": ("ramp", ("knn", 60), {}),
    "knn-2d": ("grid2d", ("knn", 40), {}),
}
DEFAULTS = {"OPT_RADIUS_SCRATCH_MB": 8192, "OPT_ROW_ORDER": 0}


def search(G, c, x, spec, sorted_out):
    fn = G.gmls_neighbors_sorted if sorted_out else G.gmls_neighbors
    if spec[0] == "radius":
        r0 = spec[2] if len(spec) > 2 else W.radius_for_mean_count(len(x))
        return fn(c, x, x, G.SEARCH_RADIUS, radius=r0, k_min=spec[1])
    return fn(c, x, x, G.SEARCH_KNN, k=spec[1], eps_mult=1.5)


@pytest.mark.parametrize("case", list(CASES))
def test_sorted_search_rows_and_records(case):
    G = require_gpu()
    cloud, spec, opts = CASES[case]
    pts = clouds()[cloud]
    n, dim = pts.shape
    c = ctx()
    x = dev(pts)
    for k, v in opts.items():
        c.set_option(getattr(G, k), v)
    try:
        flush(f"sorted search {case}")
        rp, col, eps = [host(t) for t in search(G, c, x, spec, False)]
        srp, scol, seps, rec, pcol = [host(t) for t in search(G, c, x, spec, True)]
        rec2, pcol2 = [host(t) for t in search(G, c, x, spec, True)[3:]]
    finally:
        for k in opts:
            c.set_option(getattr(G, k), DEFAULTS[k])
    # the rows are those of gmls_neighbors
    assert np.array_equal(rp, srp) and np.array_equal(col, scol) and np.array_equal(eps, seps)
    # records: every source once, its coordinates, zeros past dim, by cell
    # then index, and the same on a second call
    idx = rec[:, 3].astype(np.int64)
    assert np.array_equal(rec[:, 3], idx.astype(np.float64))
    assert np.array_equal(np.sort(idx), np.arange(n))
    assert np.array_equal(rec[:, :dim], pts[idx]) and not rec[:, dim:3].any()
    assert np.array_equal(rec, rec2) and np.array_equal(pcol, pcol2)
    # col_sorted points at the record of every row entry
    assert pcol.min() >= 0 and pcol.max() < n
    assert np.array_equal(idx[pcol], col)
    # and the rows are the oracle's
    if spec[0] == "radius":
        r0 = spec[2] if len(spec) > 2 else W.radius_for_mean_count(n)
        orp, ocol, oeps = oracle.radius(pts, pts, r0, spec[1])
        assert np.array_equal(rp, orp) and np.array_equal(row_sorted(rp, col), row_sorted(orp, ocol))
    else:
        orp, ocol, oeps = oracle.knn(pts, pts, spec[1], 1.5)
        assert np.array_equal(rp, orp) and np.array_equal(col, ocol)


def test_sorted_search_foreign_targets():
    G = require_gpu()
    src = W.density_ramp(5000, 77)
    tgt = W.rng(9).uniform(-0.1, 1.1, size=(400, 3))
    r0 = W.radius_for_mean_count(5000)
    flush("sorted search, foreign targets")
    rp, col, eps, rec, pcol = [host(t) for t in G.gmls_neighbors_sorted(ctx(), dev(src), dev(tgt), G.SEARCH_RADIUS,
                                                                          radius=r0, k_min=20)]
    orp, ocol, oeps = oracle.radius(src, tgt, r0, 20)
    assert np.array_equal(rp, orp) and np.array_equal(row_sorted(rp, col), row_sorted(orp, ocol))
    assert np.array_equal(rec[:, 3].astype(np.int64)[pcol], col)


STENCIL_CASES = {
    # cloud, search, order, basis, mask, prec, scheme
    "c4-fp64": ("ramp", ("radius", 30), 3, "scalar", "lap", 0, 0),
    "c4-mixed-pipe": ("ramp", ("radius", 30), 3, "scalar", "lap", 1, 3),
    "c4-mixed-rows": ("ramp", ("radius", 30), 3, "scalar", "lap", 1, 1),
    "c4-clustered-pipe": ("clustered", ("radius", 10, 0.02), 2, "scalar", "lap_grad", 1, 3),
    "knn-div-fp64": ("ramp", ("knn", 60), 2, "divfree", "lap_div", 0, 0),
    "knn-div-pipe": ("ramp", ("knn", 60), 2, "divfree", "lap_div", 1, 3),
    "knn-order4-wave": ("ramp", ("knn", 60), 4, "scalar", "lap_grad", 1, 4),
    "2d-order4-fp64": ("grid2d", ("knn", 40), 4, "scalar", "all", 0, 0),
}


def masks(G):
    return {"lap": G.F_LAPLACIAN, "lap_grad": G.F_LAPLACIAN | G.F_GRAD, "lap_div": G.F_LAPLACIAN | G.F_DIV,
            "all": G.F_VALUE | G.F_GRAD | G.F_LAPLACIAN}


@pytest.mark.parametrize("case", list(STENCIL_CASES))
def test_stencils_on_records_bit_equal(case):
    G = require_gpu()
    cloud, spec, order, basis, mk, prec, scheme = STENCIL_CASES[case]
    pts = clouds()[cloud]
    c = ctx()
    x = dev(pts)
    b = G.BASIS_SCALAR if basis == "scalar" else G.BASIS_DIVFREE
    m = masks(G)[mk]
    rp, col, eps, rec, pcol = search(G, c, x, spec, True)
    c.set_option(G.OPT_MIXED_SCHEME, scheme)
    try:
        flush(f"stencils on records {case}: coords")
        w0, st0, r0 = G.gmls_stencils(c, x, x, order, b, m, 4, eps, rp, col, prec=prec, report=True)
        w0, st0 = host(w0), host(st0)
        c.set_option(G.OPT_SOURCE_STRIDE, 4)
        flush(f"stencils on records {case}: records")
        w1, st1, r1 = G.gmls_stencils(c, rec, x, order, b, m, 4, eps, rp, pcol, prec=prec, report=True)
        w1, st1 = host(w1), host(st1)
    finally:
        c.set_option(G.OPT_SOURCE_STRIDE, 0)
        c.set_option(G.OPT_MIXED_SCHEME, 0)
    assert np.array_equal(st0, st1)
    assert np.array_equal(w0.view(np.uint64), w1.view(np.uint64))
    assert r0["n_fallback"] == r1["n_fallback"] and r0["n_ok"] == r1["n_ok"]


def test_multi_staggered_constrained_on_records():
    """The other stencil calls take the stride too."""
    G = require_gpu()
    pts = clouds()["ramp"][:6000]
    c = ctx()
    x = dev(pts)
    rp, col, eps, rec, pcol = G.gmls_neighbors_sorted(c, x, x, G.SEARCH_KNN, k=60, eps_mult=1.5)
    sets = [(G.BASIS_SCALAR, G.F_GRAD | G.F_LAPLACIAN), (G.BASIS_DIVFREE, G.F_LAPLACIAN | G.F_DIV)]
    normals = np.zeros_like(pts)
    normals[:, 0] = 1.0
    nrm = dev(normals)

    def run(src, cc):
        outs = []
        for prec in (G.PREC_FP64, G.PREC_MIXED):
            ws, _ = G.gmls_stencils_multi(c, src, x, 2, 4, eps, rp, cc, sets, prec=prec)
            outs += [host(w) for w, _ in ws] + [host(s) for _, s in ws]
        w, tw, st, _ = G.gmls_stencils_staggered(c, src, x, 1, G.F_GRAD | G.F_LAPLACIAN, 4, eps, rp, cc,
                                                 prec=G.PREC_MIXED)
        outs += [host(w), host(tw), host(st)]
        w, hw, st, _ = G.gmls_stencils_constrained(c, src, x, 2, G.F_LAPLACIAN, 4, eps, rp, cc, nrm)
        outs += [host(w), host(hw), host(st)]
        return outs

    flush("multi/staggered/constrained: coords")
    a = run(x, col)
    c.set_option(G.OPT_SOURCE_STRIDE, 4)
    try:
        flush("multi/staggered/constrained: records")
        b = run(rec, pcol)
    finally:
        c.set_option(G.OPT_SOURCE_STRIDE, 0)
    for u, v in zip(a, b):
        assert u.dtype == v.dtype and np.array_equal(u.view(np.uint8), v.view(np.uint8))


def test_source_stride_arguments():
    G = require_gpu()
    pts = W.jittered_grid(500, 3, 3)
    c = G.Context(0)
    x = dev(pts)
    rp, col, eps, rec, pcol = G.gmls_neighbors_sorted(c, x, x, G.SEARCH_KNN, k=20, eps_mult=1.5)
    with pytest.raises(ValueError):  # records without the option
        G.gmls_stencils(c, rec, x, 2, G.BASIS_SCALAR, G.F_LAPLACIAN, 4, eps, rp, pcol)
    with pytest.raises(G.GmlsError):
        c.set_option(G.OPT_SOURCE_STRIDE, -1)
    c.set_option(G.OPT_SOURCE_STRIDE, 2)  # below dim: refused by the call
    with pytest.raises(G.GmlsError):
        G.gmls_stencils(c, dev(np.zeros((500, 2))), x, 2, G.BASIS_SCALAR, G.F_LAPLACIAN, 4, eps, rp, pcol)
    c.set_option(G.OPT_SOURCE_STRIDE, 5)  # any stride >= dim: padded records
    padded = np.zeros((500, 5))
    padded[:, :3] = pts
    padded[:, 3:] = np.nan  # never read
    w5, _, _ = G.gmls_stencils(c, dev(padded), x, 2, G.BASIS_SCALAR, G.F_LAPLACIAN, 4, eps, rp, col)
    c.set_option(G.OPT_SOURCE_STRIDE, 0)
    w3, _, _ = G.gmls_stencils(c, x, x, 2, G.BASIS_SCALAR, G.F_LAPLACIAN, 4, eps, rp, col)
    assert np.array_equal(host(w5).view(np.uint64), host(w3).view(np.uint64))
    with pytest.raises(G.GmlsError):  # aliasing outputs
        G.gmls_neighbors_sorted(c, x, x, G.SEARCH_KNN, k=20, col=col, col_sorted=col)
    c.close()
