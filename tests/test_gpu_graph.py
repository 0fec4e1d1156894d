"""Capture-safe mode (GMLS_OPT_CAPTURE_SAFE): search + stencils captured into
one HIP graph and replayed.

Every replay is checked against the eager result of the normal mode, with
eager work (the output buffers are overwritten) and synchronisations between
the replays, and the last replay against the FP64 oracle (neighbour sets,
support radii, statuses and weights within the precision's gate).  The
capture-safe mode is also checked eagerly, and its deferred error reporting
(gmls_check) is checked on a capacity overflow."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_helpers import dev, flush, host, require_gpu, row_errors, row_sorted

FP64_TOL, MIXED_TOL = 1e-10, 1e-8

pytestmark = pytest.mark.gpu

N = 20000
K_MIN = 30


def case():
    pts = W.density_ramp(N, 1004)
    return pts, W.radius_for_mean_count(N)


def run_normal(G, c, x, r0, prec, scheme=0):
    c.set_option(G.OPT_MIXED_SCHEME, scheme)
    rp, col, eps = G.gmls_neighbors(c, x, x, G.SEARCH_RADIUS, radius=r0, k_min=K_MIN)
    w, st, _ = G.gmls_stencils(c, x, x, 3, G.BASIS_SCALAR, G.F_LAPLACIAN | G.F_GRAD, 4, eps, rp, col, prec=prec)
    return [host(v) for v in (rp, col, eps, w, st)]


@pytest.mark.parametrize("prec,scheme", [(0, 0), (1, 3), (1, 1), (1, 4)],
                         ids=["fp64", "mixed-pipe", "mixed-rows", "mixed-wave"])
def test_graph_replays_match_eager(prec, scheme):
    G = require_gpu()
    pts, r0 = case()
    s = torch.cuda.Stream()
    c = G.Context(0, stream=s)
    with torch.cuda.stream(s):
        x = dev(pts)
        flush(f"graph: eager reference prec={prec} scheme={scheme}")
        ref = run_normal(G, c, x, r0, prec, scheme)
        nnz = len(ref[1])
        F, C, _ = G.gmls_stencil_shape(3, 3, G.BASIS_SCALAR, G.F_LAPLACIAN | G.F_GRAD)
        col_buf = torch.empty(nnz + 4096, dtype=torch.int32, device="cuda")
        w_buf = torch.empty(F * C * nnz, dtype=torch.float64, device="cuda")
        st_buf = torch.empty(N, dtype=torch.uint8, device="cuda")
        c.set_option(G.OPT_CAPTURE_SAFE, 1)
        outs = {}

        def step():
            rp, col, eps = G.gmls_neighbors(c, x, x, G.SEARCH_RADIUS, radius=r0, k_min=K_MIN, col=col_buf)
            G.gmls_stencils(c, x, x, 3, G.BASIS_SCALAR, G.F_LAPLACIAN | G.F_GRAD, 4, eps, rp, col[:nnz], prec=prec,
                            weights=w_buf, status=st_buf)
            outs["rp"], outs["eps"] = rp, eps

        def compare(tag):
            s.synchronize()
            got = [host(outs["rp"]), host(col_buf[:nnz]), host(outs["eps"]), host(w_buf), host(st_buf)]
            for name, a, b in zip(("row_ptr", "col", "eps", "weights", "status"), got, ref):
                assert np.array_equal(a, b), f"{tag}: {name} differs"
            c.check()

        flush("graph: capture-safe eager")
        step()
        compare("capture-safe eager")
        g = torch.cuda.CUDAGraph()
        flush("graph: capture")
        with torch.cuda.graph(g, stream=s):
            step()
        for rep in range(3):
            # eager work between replays: clobber every output
            col_buf.fill_(-7)
            w_buf.fill_(float("nan"))
            st_buf.fill_(255)
            outs["eps"].fill_(-1.0)
            s.synchronize()
            flush(f"graph: replay {rep}")
            g.replay()
            compare(f"replay {rep}")
        flush("graph: last replay against the oracle")
        rp, col, eps = host(outs["rp"]), host(col_buf[:nnz]), host(outs["eps"])
        w, st = host(w_buf), host(st_buf)
    c.close()
    orp, ocol, oeps = oracle.radius(pts, pts, r0, K_MIN)
    assert np.array_equal(rp, orp) and np.array_equal(row_sorted(rp, col), ocol) and np.array_equal(eps, oeps)
    # the oracle's stencils on the replay's rows (radius rows are sets; the
    # weights follow the row order they are given)
    ow, ost, _, _ = oracle.stencils(pts, pts, 3, "scalar", G.F_LAPLACIAN | G.F_GRAD, 4, oeps, orp, col)
    assert np.array_equal(st == 1, ost == 1)
    errs = row_errors(w, ow, rp, F, C)[ost != 1]
    flush(f"  max rel err {errs.max():.3e}")
    assert errs.max() <= (FP64_TOL if prec == G.PREC_FP64 else MIXED_TOL)


def test_capture_safe_reports_capacity_through_check():
    G = require_gpu()
    pts, r0 = case()
    s = torch.cuda.Stream()
    c = G.Context(0, stream=s)
    with torch.cuda.stream(s):
        x = dev(pts)
        ref = run_normal(G, c, x, r0, 0)
        small = torch.full((len(ref[1]) // 2,), -3, dtype=torch.int32, device="cuda")
        c.set_option(G.OPT_CAPTURE_SAFE, 1)
        flush("capture-safe capacity overflow")
        rp, col, eps = G.gmls_neighbors(c, x, x, G.SEARCH_RADIUS, radius=r0, k_min=K_MIN, col=small)
        with pytest.raises(G.GmlsError) as e:
            c.check()
        assert e.value.status == G.GMLS_ERR_CAPACITY
        assert (host(small) == -3).all(), "col was written despite the overflow"
        assert host(rp)[-1] == len(ref[1])
        c.check()  # the record is cleared
    c.close()


@pytest.mark.parametrize("order,k,p,fp64", [(4, 170, 6, False), (2, 60, 4, False), (4, 170, 6, True)],
                         ids=["wave", "pipeline", "fp64"])
def test_graph_replays_shared_multi(order, k, p, fp64):
    """A kNN search and one gmls_stencils_multi call (scalar + divergence-free
    sets sharing the Gram, or in FP64 the QR factor) captured together and
    replayed, against eager."""
    G = require_gpu()
    prec = G.PREC_FP64 if fp64 else G.PREC_MIXED
    pts = W.jittered_grid(6000, 3, 1005)
    sets = [(G.BASIS_SCALAR, G.F_GRAD | G.F_LAPLACIAN), (G.BASIS_DIVFREE, G.F_LAPLACIAN | G.F_DIV)]
    s = torch.cuda.Stream()
    c = G.Context(0, stream=s)
    with torch.cuda.stream(s):
        x = dev(pts)
        flush(f"graph multi order={order}: eager reference")
        rp, col, eps = G.gmls_neighbors(c, x, x, G.SEARCH_KNN, k=k, eps_mult=1.5)
        ref = [(host(w), host(st)) for w, st in
               G.gmls_stencils_multi(c, x, x, order, p, eps, rp, col, sets, prec=prec)[0]]
        nnz = col.numel()
        col_buf = torch.empty(nnz, dtype=torch.int32, device="cuda")
        outs = []
        for basis, mask in sets:
            F, C, _ = G.gmls_stencil_shape(3, order, basis, mask)
            outs.append((torch.empty(F * C * nnz, dtype=torch.float64, device="cuda"),
                         torch.empty(len(pts), dtype=torch.uint8, device="cuda")))
        c.set_option(G.OPT_CAPTURE_SAFE, 1)
        gout = {}

        def step():
            rp_, col_, eps_ = G.gmls_neighbors(c, x, x, G.SEARCH_KNN, k=k, eps_mult=1.5, col=col_buf)
            G.gmls_stencils_multi(c, x, x, order, p, eps_, rp_, col_, sets, prec=prec, outputs=outs)
            gout["rp"] = rp_

        def compare(tag):
            s.synchronize()
            for (w, st), (rw, rst) in zip(outs, ref):
                assert np.array_equal(host(st), rst), tag
                assert np.array_equal(host(w).view(np.uint64), rw.view(np.uint64)), tag
            c.check()

        step()
        compare("capture-safe eager")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            step()
        for rep in range(3):
            for w, st in outs:
                w.fill_(float("nan"))
                st.fill_(255)
            s.synchronize()
            flush(f"graph multi: replay {rep}")
            g.replay()
            compare(f"replay {rep}")
        flush("graph multi: last replay against the oracle")
        rp, col = host(gout["rp"]), host(col_buf)
        got = [(host(w), host(st)) for w, st in outs]
    c.close()
    orp, ocol, oeps = oracle.knn(pts, pts, k, 1.5)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    for (basis, mask), (w, st) in zip(sets, got):
        name = "scalar" if basis == G.BASIS_SCALAR else "divfree"
        ow, ost, F, C = oracle.stencils(pts, pts, order, name, mask, p, oeps, orp, ocol)
        assert np.array_equal(st == 1, ost == 1)
        zero = (F - 1,) if name == "divfree" and mask & G.F_DIV else ()
        errs = row_errors(w, ow, rp, F, C, zero_rows=zero)[ost != 1]
        flush(f"  {name}: max rel err {errs.max():.3e}")
        assert errs.max() <= (FP64_TOL if fp64 else MIXED_TOL)


@pytest.mark.parametrize("knn", [False, True], ids=["radius", "knn"])
def test_graph_replays_sorted_records(knn):
    """gmls_neighbors_sorted (records and positions) and stencils gathered
    from the records (source stride 4) captured together: every replay equals
    the eager capture-safe run, and the stencils equal those of the index
    layout bit for bit."""
    G = require_gpu()
    pts, r0 = case()
    n = len(pts)
    spec = dict(mode=G.SEARCH_KNN, k=40, eps_mult=1.5) if knn else dict(mode=G.SEARCH_RADIUS, radius=r0,
                                                                         k_min=K_MIN)
    s = torch.cuda.Stream()
    c = G.Context(0, stream=s)
    with torch.cuda.stream(s):
        x = dev(pts)
        flush(f"graph sorted knn={knn}: index-layout reference")
        rp, col, eps = G.gmls_neighbors(c, x, x, **spec)
        ref_w, ref_st, _ = G.gmls_stencils(c, x, x, 3, G.BASIS_SCALAR, G.F_LAPLACIAN | G.F_GRAD, 4, eps, rp, col,
                                           prec=G.PREC_MIXED)
        ref = [host(v) for v in (rp, col, eps, ref_w, ref_st)]
        nnz = col.numel()
        F, C, _ = G.gmls_stencil_shape(3, 3, G.BASIS_SCALAR, G.F_LAPLACIAN | G.F_GRAD)
        col_buf = torch.empty(nnz + 4096, dtype=torch.int32, device="cuda")
        pcol_buf = torch.empty_like(col_buf)
        rec_buf = torch.empty((n, 4), dtype=torch.float64, device="cuda")
        w_buf = torch.empty(F * C * nnz, dtype=torch.float64, device="cuda")
        st_buf = torch.empty(n, dtype=torch.uint8, device="cuda")
        c.set_option(G.OPT_SOURCE_STRIDE, 4)
        # one normal call of each kind sizes the workspace
        rp_, col_, eps_, rec_, pcol_ = G.gmls_neighbors_sorted(c, x, x, **spec)
        G.gmls_stencils(c, rec_, x, 3, G.BASIS_SCALAR, G.F_LAPLACIAN | G.F_GRAD, 4, eps_, rp_, pcol_,
                        prec=G.PREC_MIXED)
        c.set_option(G.OPT_CAPTURE_SAFE, 1)
        outs = {}

        def step():
            rp2, col2, eps2, rec2, pcol2 = G.gmls_neighbors_sorted(c, x, x, col=col_buf, col_sorted=pcol_buf,
                                                                   records=rec_buf, **spec)
            G.gmls_stencils(c, rec2, x, 3, G.BASIS_SCALAR, G.F_LAPLACIAN | G.F_GRAD, 4, eps2, rp2,
                            pcol2[:nnz], prec=G.PREC_MIXED, weights=w_buf, status=st_buf)
            outs["rp"], outs["eps"] = rp2, eps2

        def snapshot():
            s.synchronize()
            return [host(outs["rp"]), host(col_buf[:nnz]), host(outs["eps"]), host(w_buf), host(st_buf),
                    host(pcol_buf[:nnz]), host(rec_buf)]

        flush("graph sorted: capture-safe eager")
        step()
        eager = snapshot()
        c.check()
        for name, a_, b_ in zip(("row_ptr", "col", "eps", "weights", "status"), eager, ref):
            assert np.array_equal(a_, b_), f"records vs index layout: {name} differs"
        idx = eager[6][:, 3].astype(np.int64)
        assert np.array_equal(idx[eager[5]], eager[1])
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            step()
        for rep in range(3):
            col_buf.fill_(-7)
            pcol_buf.fill_(-7)
            rec_buf.fill_(float("nan"))
            w_buf.fill_(float("nan"))
            st_buf.fill_(255)
            s.synchronize()
            flush(f"graph sorted: replay {rep}")
            g.replay()
            got = snapshot()
            for k_, (a_, b_) in enumerate(zip(got, eager)):
                assert np.array_equal(np.asarray(a_).view(np.uint8), np.asarray(b_).view(np.uint8)), \
                    f"replay {rep}: output {k_} differs"
            c.check()
    c.close()
