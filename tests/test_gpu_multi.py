"""Several stencil sets on one neighbour list (gmls_stencils_multi).

A scalar and a divergence-free set of the same order share the moments and
the swept Gram in the wavefront scheme, the moments on the pipeline, and the
Householder factor in FP64; each set's result must be the one gmls_stencils
gives for it alone (bit for bit: the shared kernels run the same arithmetic
in the same order), and therefore within the gates of the oracle.  Other
combinations run the sets in turn."""
import numpy as np
import pytest

from tests.gpu_helpers import ctx, dev, flush, host, require_gpu, row_errors
from tests.test_gpu_stencils import FP64_TOL, MIXED_TOL, case_data

pytestmark = pytest.mark.gpu


def separate(G, pts, rp, col, eps, order, p, sets, prec):
    s = dev(pts)
    out = []
    for basis, mask in sets:
        w, st, _ = G.gmls_stencils(ctx(), s, s, order, basis, mask, p, dev(eps), dev(rp), dev(col), prec=prec)
        out.append((host(w), host(st)))
    return out


def multi(G, pts, rp, col, eps, order, p, sets, prec):
    s = dev(pts)
    outs, rep = G.gmls_stencils_multi(ctx(), s, s, order, p, dev(eps), dev(rp), dev(col), sets, prec=prec,
                                      report=True)
    got = [(host(w), host(st)) for w, st in outs]
    check_report(rep, [st for _, st in got])
    return got, rep


def check_report(rep, statuses):
    """The report counts (target, set) pairs by the statuses written, over
    every set of the call."""
    allst = np.concatenate(statuses)
    assert rep["n_targets"] == allst.size
    assert rep["n_rank_deficient"] == int((allst == 1).sum())
    assert rep["n_fallback"] == int((allst == 2).sum())
    assert rep["n_not_converged"] == int((allst == 3).sum())
    assert rep["n_ok"] == allst.size - rep["n_rank_deficient"]


@pytest.mark.parametrize("names", [("3d_m4_k170", "3d_divfree_m4"), ("3d_divfree_m4_k30", "3d_divfree_m4_k30")])
def test_shared_gram_equals_separate_calls(names):
    G = require_gpu()
    pts, rp, col, eps, _, _, _, _ = case_data(names[0])
    order, p = 4, 6
    sets = [(G.BASIS_SCALAR, G.F_GRAD | G.F_LAPLACIAN), (G.BASIS_DIVFREE, G.F_LAPLACIAN | G.F_DIV)]
    flush(f"shared Gram {names}")
    got, rep = multi(G, pts, rp, col, eps, order, p, sets, G.PREC_MIXED)
    ref = separate(G, pts, rp, col, eps, order, p, sets, G.PREC_MIXED)
    flush(f"  report {rep}")
    for (gw, gs), (rw, rs) in zip(got, ref):
        assert np.array_equal(gs, rs)
        assert np.array_equal(gw.view(np.uint64), rw.view(np.uint64))
    # and against the oracle, where it defines the stencils
    if names[0] == "3d_m4_k170":
        for (gw, gs), name, tol in zip(got, names, (MIXED_TOL, MIXED_TOL)):
            _, _, _, _, w, st, F, C = case_data(name)
            assert np.array_equal(gs == 1, st == 1)
            zero = (F - 1,) if C > 1 else ()
            assert row_errors(gw, w, rp, F, C, zero_rows=zero).max() <= tol
    else:  # 30 neighbours: the scalar basis (35) is rank deficient, the divergence-free one (85 of 90 rows) is not
        assert (got[0][1] == 1).all() and np.isnan(got[0][0]).all()
        _, _, _, _, w, st, F, C = case_data(names[1])
        assert (st == 0).all() and (got[1][1] == 2).all()
        assert row_errors(got[1][0], w, rp, F, C, zero_rows=(F - 1,)).max() <= FP64_TOL


@pytest.mark.parametrize("name", ["3d_divfree_m2", "2d_divfree_m2", "3d_divfree_m2_k9"])
def test_shared_pipeline_moments_equal_separate_calls(name):
    """Order 2: both sets on the pipeline, the divergence-free solve takes the
    scalar set's moments (bit-identical to separate calls, and the oracle)."""
    G = require_gpu()
    pts, rp, col, eps, w, st, F, C = case_data(name)
    sets = [(G.BASIS_DIVFREE, G.F_VALUE | G.F_LAPLACIAN | G.F_DIV), (G.BASIS_SCALAR, G.F_GRAD | G.F_LAPLACIAN)]
    flush(f"shared pipeline moments {name}")
    got, _ = multi(G, pts, rp, col, eps, 2, 4, sets, G.PREC_MIXED)
    ref = separate(G, pts, rp, col, eps, 2, 4, sets, G.PREC_MIXED)
    for (gw, gs), (rw, rs) in zip(got, ref):
        if name.endswith("_k9"):  # 9 < 10 neighbours: the bins of a separate divergence-free call differ
            assert np.array_equal(gs == 1, rs == 1)
        else:
            assert np.array_equal(gs, rs)
            assert np.array_equal(gw.view(np.uint64), rw.view(np.uint64))
    assert np.array_equal(got[0][1] == 1, st == 1)
    errs = row_errors(got[0][0], w, rp, F, C, zero_rows=(F - 1,))
    assert errs[st != 1].max() <= MIXED_TOL


@pytest.mark.parametrize("name,order,p", [("3d_divfree_m2", 2, 4), ("2d_divfree_m2", 2, 4),
                                          ("3d_divfree_m2_k9", 2, 4), ("3d_divfree_m4", 4, 6),
                                          ("3d_divfree_m4_k30", 4, 6)])
def test_fp64_shared_factor_equals_separate_calls(name, order, p):
    """FP64: one Householder factor per target serves the scalar and the
    divergence-free set; each set's weights and statuses are those of its own
    call bit for bit (the same steps in the same order), and the
    divergence-free set is within the FP64 gate of the oracle."""
    G = require_gpu()
    pts, rp, col, eps, w, st, F, C = case_data(name)
    dmask = G.F_VALUE | G.F_LAPLACIAN | G.F_DIV if order == 2 else G.F_LAPLACIAN | G.F_DIV
    sets = [(G.BASIS_SCALAR, G.F_GRAD | G.F_LAPLACIAN), (G.BASIS_DIVFREE, dmask)]
    flush(f"FP64 shared factor {name}")
    got, rep = multi(G, pts, rp, col, eps, order, p, sets, G.PREC_FP64)
    ref = separate(G, pts, rp, col, eps, order, p, sets, G.PREC_FP64)
    flush(f"  report {rep}")
    for (gw, gs), (rw, rs) in zip(got, ref):
        assert np.array_equal(gs, rs)
        assert np.array_equal(gw.view(np.uint64), rw.view(np.uint64))
    gw, gs = got[1]
    assert np.array_equal(gs == 1, st == 1)
    errs = row_errors(gw, w, rp, F, C, zero_rows=(F - 1,))
    assert errs[st != 1].max() <= FP64_TOL


def test_sets_in_turn_equal_separate_calls():
    """Two sets of one basis are not shared: they run one after the other."""
    G = require_gpu()
    pts, rp, col, eps, _, _, _, _ = case_data("3d_divfree_m2")
    sets = [(G.BASIS_SCALAR, G.F_VALUE | G.F_LAPLACIAN), (G.BASIS_SCALAR, G.F_GRAD)]
    for prec in (G.PREC_FP64, G.PREC_MIXED):
        flush(f"sets in turn prec={prec}")
        got, _ = multi(G, pts, rp, col, eps, 2, 4, sets, prec)
        ref = separate(G, pts, rp, col, eps, 2, 4, sets, prec)
        for (gw, gs), (rw, rs) in zip(got, ref):
            assert np.array_equal(gs, rs)
            assert np.array_equal(gw.view(np.uint64), rw.view(np.uint64))


def test_multi_rejects_bad_sets():
    G = require_gpu()
    pts, rp, col, eps, _, _, _, _ = case_data("3d_divfree_m2")
    with pytest.raises(G.GmlsError):
        multi(G, pts, rp, col, eps, 2, 4, [], G.PREC_MIXED)
    with pytest.raises(G.GmlsError):
        multi(G, pts, rp, col, eps, 2, 4, [(7, G.F_GRAD)], G.PREC_MIXED)
    with pytest.raises(G.GmlsError):
        multi(G, pts, rp, col, eps, 2, 4, [(G.BASIS_DIVFREE, G.F_GRAD)], G.PREC_MIXED)
