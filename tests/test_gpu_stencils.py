"""GPU stencils vs the FP64 oracle on the same neighbour lists.

Gates (per target and functional row, ||a - b|| / ||b||): FP64 path 1e-10,
mixed path 1e-8.  Sizes span every row-count bin (N up to 256), ragged rows
from the radius search, and both bases."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import row_sorted, ctx, dev, flush, host, require_gpu, row_errors

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-8

CASES = {
    # name: (points, search, basis, order, mask, p)
    "c1_2d_m2": (lambda: W.make_points("c1_2d_m2"), ("knn", 12), "scalar", 2, 2 | 4, 4),
    "2d_m4": (lambda: W.jittered_grid(6000, 2, 1002), ("knn", 40), "scalar", 4, 1 | 2 | 4, 4),
    "3d_m2_grad": (lambda: W.jittered_grid(8000, 3, 1003), ("knn", 60), "scalar", 2, 2, 4),
    "3d_m3_radius": (lambda: W.density_ramp(12000, 1004), ("radius", 30), "scalar", 3, 4, 4),
    "3d_m4_k170": (lambda: W.jittered_grid(8000, 3, 1005), ("knn", 170), "scalar", 4, 2 | 4, 6),
    "3d_divfree_m2": (lambda: W.jittered_grid(8000, 3, 1003), ("knn", 60), "divfree", 2, 1 | 4 | 8, 4),
    "2d_divfree_m2": (lambda: W.jittered_grid(3000, 2, 7), ("knn", 20), "divfree", 2, 1 | 4 | 8, 4),
    "3d_divfree_m4": (lambda: W.jittered_grid(8000, 3, 1005), ("knn", 170), "divfree", 4, 4 | 8, 6),
    # the FP64 solve's second factor (of B) at 10 columns: its column sums
    # go through LDS (3-D order 3, 2-D order 4), where order 2 takes wave sums
    "3d_divfree_m3": (lambda: W.jittered_grid(6000, 3, 1006), ("knn", 100), "divfree", 3, 1 | 4 | 8, 4),
    "2d_divfree_m4": (lambda: W.jittered_grid(4000, 2, 1007), ("knn", 40), "divfree", 4, 1 | 4 | 8, 4),
    # fewer neighbours than scalar monomials (9 < 10, 30 < 35) but enough
    # rows for the divergence-free functions (27 >= 26, 90 >= 85): the
    # divergence-free sample matrix is factored itself
    "3d_divfree_m2_k9": (lambda: W.jittered_grid(3000, 3, 11), ("knn", 9), "divfree", 2, 1 | 4 | 8, 4),
    "3d_divfree_m4_k30": (lambda: W.jittered_grid(3000, 3, 12), ("knn", 30), "divfree", 4, 4 | 8, 6),
}

_cache = {}


def case_data(name):
    if name not in _cache:
        mk, search, basis, order, mask, p = CASES[name]
        pts = mk()
        if search[0] == "knn":
            rp, col, eps = oracle.knn(pts, pts, search[1], 1.5)
        else:
            rp, col, eps = oracle.radius(pts, pts, W.radius_for_mean_count(len(pts)), search[1])
        w, st, F, C = oracle.stencils(pts, pts, order, basis, mask, p, eps, rp, col)
        _cache[name] = (pts, rp, col, eps, w, st, F, C)
    return _cache[name]


def run_gpu(name, prec, sub=None):
    G = require_gpu()
    pts, rp, col, eps, w, st, F, C = case_data(name)
    _, _, basis, order, mask, p = CASES[name]
    b = G.BASIS_SCALAR if basis == "scalar" else G.BASIS_DIVFREE
    flush(f"stencils {name} prec={prec} n={len(pts)} nnz={len(col)}")
    s = dev(pts)
    gw, gst, rep = G.gmls_stencils(ctx(), s, s, order, b, mask, p, dev(eps), dev(rp), dev(col), prec=prec,
                                   report=True)
    return host(gw), host(gst), rep


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_matches_oracle(name):
    G = require_gpu()
    pts, rp, col, eps, w, st, F, C = case_data(name)
    gw, gst, rep = run_gpu(name, G.PREC_FP64)
    assert np.array_equal(gst, st)
    zero = (F - 1,) if CASES[name][2] == "divfree" and CASES[name][4] & 8 else ()
    errs = row_errors(gw, w, rp, F, C, zero_rows=zero)
    flush(f"  fp64 max rel err {errs.max():.3e}  p99 {np.percentile(errs, 99):.3e}")
    assert errs.max() <= FP64_TOL


def test_rank_deficient_targets_flagged():
    G = require_gpu()
    pts = W.jittered_grid(500, 2, 9)
    rp, col, eps = oracle.knn(pts, pts, 5, 1.5)  # N = 5 < Q = 6
    s = dev(pts)
    flush("rank deficient N<Q")
    gw, gst, rep = G.gmls_stencils(ctx(), s, s, 2, G.BASIS_SCALAR, 4, 4, dev(eps), dev(rp), dev(col),
                                   prec=G.PREC_FP64, report=True)
    assert (host(gst) == 1).all() and np.isnan(host(gw)).all()
    assert rep["n_rank_deficient"] == 500
    flat = W.rng(4).uniform(size=(600, 3))
    flat[:, 2] = 0.25
    rp, col, eps = oracle.knn(flat, flat, 30, 1.5)
    w, st, F, C = oracle.stencils(flat, flat, 2, "scalar", 4, 4, eps, rp, col)
    s = dev(flat)
    flush("rank deficient coplanar")
    gw, gst, _ = G.gmls_stencils(ctx(), s, s, 2, G.BASIS_SCALAR, 4, 4, dev(eps), dev(rp), dev(col),
                                 prec=G.PREC_FP64)
    assert np.array_equal(host(gst), st)


def test_empty_and_unsupported():
    G = require_gpu()
    s = dev(W.jittered_grid(100, 3, 1))
    e = dev(np.zeros(0))
    rp = dev(np.zeros(1, np.int64))
    c = dev(np.zeros(0, np.int32))
    flush("empty target set")
    gw, gst, _ = G.gmls_stencils(ctx(), s, s[:0], 2, G.BASIS_SCALAR, 4, 4, e, rp, c)
    assert gw.numel() == 0
    with pytest.raises(G.GmlsError):
        G.gmls_stencils(ctx(), s, s[:0], 2, G.BASIS_SCALAR, 8, 4, e, rp, c)  # divergence on scalar basis
    with pytest.raises(G.GmlsError):
        G.gmls_stencils(ctx(), s, s[:0], 2, G.BASIS_DIVFREE, 2, 4, e, rp, c)  # gradient on vector basis


def test_apply_matches_numpy():
    G = require_gpu()
    pts, rp, col, eps, w, st, F, C = case_data("3d_divfree_m2")
    field = W.rng(3).standard_normal((len(pts), C))
    flush("apply")
    out = host(G.gmls_apply(ctx(), dev(rp), dev(col), dev(w), F, C, dev(field)))
    ref = np.zeros((len(rp) - 1, F))
    for t in range(len(rp) - 1):
        n = rp[t + 1] - rp[t]
        a = w[F * C * rp[t]: F * C * rp[t + 1]].reshape(F, n, C)
        ref[t] = np.einsum("fjc,jc->f", a, field[col[rp[t]:rp[t + 1]]])
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_end_to_end_gpu_search_then_stencils():
    G = require_gpu()
    pts = W.density_ramp(20000, 1004)
    r0 = W.radius_for_mean_count(20000)
    s = dev(pts)
    flush("end to end radius + m3")
    rp, col, eps = G.gmls_neighbors(ctx(), s, s, G.SEARCH_RADIUS, radius=r0, k_min=30)
    gw, gst, _ = G.gmls_stencils(ctx(), s, s, 3, G.BASIS_SCALAR, 4, 4, eps, rp, col, prec=G.PREC_FP64)
    orp, ocol, oeps = oracle.radius(pts, pts, r0, 30)
    gcol = host(col)
    assert np.array_equal(host(rp), orp) and np.array_equal(row_sorted(orp, gcol), ocol)
    assert np.array_equal(host(eps), oeps)
    # the oracle's weights for the GPU's row order (radius rows are sets)
    w, st, F, C = oracle.stencils(pts, pts, 3, "scalar", 4, 4, oeps, orp, gcol)
    errs = row_errors(host(gw), w, orp, F, C)
    flush(f"  e2e max rel err {errs.max():.3e}")
    assert errs.max() <= FP64_TOL


def _nmono(dim, deg):
    from math import comb
    return comb(deg + dim, dim)


def scheme_compiled(name, scheme):
    """Whether a mixed scheme (1 rows, 2 moment Gram, 3 pipeline, 4 wavefront
    per target) exists for a case."""
    _, _, basis, order, _, _ = CASES[name]
    dim = case_data(name)[0].shape[1]
    if scheme == 1:
        return True
    if scheme == 4:
        return _nmono(dim, order) <= 35
    if scheme == 2:
        return _nmono(dim, 2 * order) <= 96
    # the pipeline: scalar bases of <= 20 monomials, divergence-free bases
    # whose scalar basis has <= 10
    return _nmono(dim, order) <= (20 if basis == "scalar" else 10)


def run_mixed(name, scheme, chunk=0):
    G = require_gpu()
    c = ctx()
    c.set_option(G.OPT_MIXED_SCHEME, scheme)
    c.set_option(G.OPT_PIPE_CHUNK, chunk)
    try:
        return run_gpu(name, G.PREC_MIXED)
    finally:
        c.set_option(G.OPT_MIXED_SCHEME, 0)
        c.set_option(G.OPT_PIPE_CHUNK, 0)


def check_mixed(name, gw, gst, rep):
    pts, rp, col, eps, w, st, F, C = case_data(name)
    # rank-deficient targets agree; everything else is OK or was recomputed
    assert np.array_equal(gst == 1, st == 1)
    assert np.isin(gst, [0, 1, 2, 3]).all()
    zero = (F - 1,) if CASES[name][2] == "divfree" and CASES[name][4] & 8 else ()
    errs = row_errors(gw, w, rp, F, C, zero_rows=zero)
    flush(f"  mixed max rel err {errs.max():.3e}  p99 {np.percentile(errs, 99):.3e}  "
          f"fallback {rep['n_fallback']} not-conv {rep['n_not_converged']} sweeps {rep['sweep_hist'][:6]} "
          f"cond_max {rep['cond_max']:.2e}")
    assert errs.max() <= MIXED_TOL
    # every target not rank deficient is counted once: converged, fallback or not converged
    n_live = int((st != 1).sum())
    assert sum(rep["sweep_hist"]) + rep["n_fallback"] + rep["n_not_converged"] == n_live
    # the report's counts are those of the statuses written
    assert rep["n_fallback"] == int((gst == 2).sum()) and rep["n_not_converged"] == int((gst == 3).sum())
    assert rep["n_rank_deficient"] == int((gst == 1).sum())
    if sum(rep["sweep_hist"]) > 0:  # condition numbers of the Grams the mixed kernels factored
        assert 0.0 < rep["cond_min"] <= rep["cond_max"] * (1 + 1e-6)
        assert rep["cond_min"] / 1.03 <= rep["cond_med"] <= rep["cond_max"] * 1.03


@pytest.mark.parametrize("scheme", [1, 2, 3, 4], ids=["rows", "gram", "pipe", "wave"])
@pytest.mark.parametrize("name", list(CASES))
def test_mixed_matches_oracle(name, scheme):
    G = require_gpu()
    if not scheme_compiled(name, scheme):
        with pytest.raises(G.GmlsError) as e:
            run_mixed(name, scheme)
        assert e.value.status == 5
        return
    check_mixed(name, *run_mixed(name, scheme))


def test_mixed_auto_scheme():
    require_gpu()
    check_mixed("3d_m3_radius", *run_mixed("3d_m3_radius", 0))


@pytest.mark.parametrize("chunk", [64, 1000, 4093])
def test_mixed_pipe_chunks(chunk):
    """Chunked pipeline: chunk boundaries inside and across row-count bins."""
    require_gpu()
    check_mixed("3d_m3_radius", *run_mixed("3d_m3_radius", 3, chunk))


@pytest.mark.parametrize("scheme", [1, 2, 3, 4], ids=["rows", "gram", "pipe", "wave"])
def test_mixed_forced_fallback_is_fp64_exact(scheme):
    G = require_gpu()
    c = ctx()
    c.set_option(G.OPT_FORCE_FALLBACK, 1)
    try:
        pts, rp, col, eps, w, st, F, C = case_data("3d_m3_radius")
        gw, gst, rep = run_mixed("3d_m3_radius", scheme)
    finally:
        c.set_option(G.OPT_FORCE_FALLBACK, 0)
    assert (gst == 2).all() and rep["n_fallback"] == len(st)
    errs = row_errors(gw, w, rp, F, C)
    flush(f"  forced fallback max rel err {errs.max():.3e}")
    assert errs.max() <= FP64_TOL


def test_divfree_pipe_forced_fallback_is_fp64_exact():
    """The divergence-free pipeline hands every target to the FP64 QR kernel."""
    G = require_gpu()
    c = ctx()
    c.set_option(G.OPT_FORCE_FALLBACK, 1)
    try:
        pts, rp, col, eps, w, st, F, C = case_data("3d_divfree_m2")
        gw, gst, rep = run_mixed("3d_divfree_m2", 3)
    finally:
        c.set_option(G.OPT_FORCE_FALLBACK, 0)
    assert (gst == 2).all() and rep["n_fallback"] == len(st)
    errs = row_errors(gw, w, rp, F, C, zero_rows=(F - 1,))
    flush(f"  divergence-free forced fallback max rel err {errs.max():.3e}")
    assert errs.max() <= FP64_TOL


def test_divfree_wave_forced_fallback_is_fp64_exact():
    """The wavefront kernel hands every divergence-free target to the FP64 QR kernel."""
    G = require_gpu()
    c = ctx()
    c.set_option(G.OPT_FORCE_FALLBACK, 1)
    try:
        pts, rp, col, eps, w, st, F, C = case_data("2d_divfree_m2")
        gw, gst, rep = run_mixed("2d_divfree_m2", 4)
    finally:
        c.set_option(G.OPT_FORCE_FALLBACK, 0)
    assert (gst == 2).all() and rep["n_fallback"] == len(st)
    errs = row_errors(gw, w, rp, F, C, zero_rows=(F - 1,))
    flush(f"  divergence-free wave forced fallback max rel err {errs.max():.3e}")
    assert errs.max() <= FP64_TOL


@pytest.mark.parametrize("name", ["3d_m4_k170", "3d_divfree_m4", "3d_m3_radius"])
def test_wave_reproducible(name):
    """Two calls of the wavefront kernel give identical bits (fixed reduction order)."""
    require_gpu()
    a = run_mixed(name, 4)
    b = run_mixed(name, 4)
    assert np.array_equal(a[0].view(np.uint64), b[0].view(np.uint64))
    assert np.array_equal(a[1], b[1])


@pytest.mark.parametrize("scheme", [1, 2, 3, 4], ids=["rows", "gram", "pipe", "wave"])
def test_mixed_near_coplanar_triggers_fallback(scheme):
    G = require_gpu()
    n = 4000
    pts = W.jittered_grid(n, 3, 13)
    # tilted near-plane: z - 0.3x - 0.2y is tiny, so the linear monomials are
    # nearly dependent in a way no diagonal (equilibration) scaling removes
    pts[:, 2] = 0.3 * pts[:, 0] + 0.2 * pts[:, 1] + 0.25 + (pts[:, 2] - 0.5) * 1e-4
    rp, col, eps = oracle.knn(pts, pts, 40, 1.5)
    w, st, F, C = oracle.stencils(pts, pts, 2, "scalar", 4, 4, eps, rp, col)
    s = dev(pts)
    flush(f"near-coplanar mixed scheme {scheme}")
    c = ctx()
    c.set_option(G.OPT_MIXED_SCHEME, scheme)
    try:
        gw, gst, rep = G.gmls_stencils(c, s, s, 2, G.BASIS_SCALAR, 4, 4, dev(eps), dev(rp), dev(col),
                                       prec=G.PREC_MIXED, report=True)
    finally:
        c.set_option(G.OPT_MIXED_SCHEME, 0)
    gw, gst = host(gw), host(gst)
    flush(f"  fallback {rep['n_fallback']} not-conv {rep['n_not_converged']} cond_max {rep['cond_max']:.2e}")
    assert rep["n_fallback"] + rep["n_not_converged"] > 0
    ok = st == 0
    assert np.array_equal(gst == 1, st == 1)
    errs = row_errors(gw, w, rp, F, C)
    assert errs[ok].max() <= MIXED_TOL


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_duplicate_points(prec):
    """Every point of the cloud three times over: with 12 neighbours a target
    sees 4 distinct points (fewer than the 6 functions of order 2 in 2D), so
    its weighted sample matrix is rank deficient although N >= Q; with 30 it
    sees 10 and the duplicated rows only weight them.  Statuses must equal the
    oracle's and the weights must be within the gate where defined."""
    G = require_gpu()
    base = W.jittered_grid(400, 2, 31)
    pts = np.repeat(base, 3, axis=0)
    p = G.PREC_FP64 if prec == "fp64" else G.PREC_MIXED
    s = dev(pts)
    for k in (12, 30):
        rp, col, eps = oracle.knn(pts, pts, k, 1.5)
        w, st, F, C = oracle.stencils(pts, pts, 2, "scalar", 2 | 4, 4, eps, rp, col)
        assert (st == 1).all() if k == 12 else (st == 0).all()
        flush(f"duplicate points k={k} prec={prec}")
        gw, gst, rep = G.gmls_stencils(ctx(), s, s, 2, G.BASIS_SCALAR, 2 | 4, 4, dev(eps), dev(rp), dev(col),
                                       prec=p, report=True)
        gw, gst = host(gw), host(gst)
        assert np.array_equal(gst == 1, st == 1)
        assert rep["n_rank_deficient"] == int((st == 1).sum())
        if k == 12:
            assert np.isnan(gw).all()
        else:
            errs = row_errors(gw, w, rp, F, C)
            assert errs.max() <= (FP64_TOL if prec == "fp64" else MIXED_TOL)
