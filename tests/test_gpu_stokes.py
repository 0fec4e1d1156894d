"""Global Stokes operator on the GPU (gmls_assemble_stokes, gmls_spmv):

* the paper's quadratic manufactured solution (Section 4.1) with every
  stencil computed on the GPU: the assembled operator applied by gmls_spmv to
  the exact nodal values returns the right-hand side to rounding in every row;
* the GPU matrix equals the oracle's assembly of the same (GPU) stencils
  entry by entry (summed duplicates, sorted columns);
* gmls_spmv equals scipy's product on the same matrix, including the
  multiplier row, which is long enough (n > 8192 entries) for the block kernel;
* a too small capacity reports the size needed and writes nothing."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
import workloads as W
from oracle import stokes as OK
from tests.gpu_helpers import ctx, dev, flush, host, require_gpu
from tests.manufactured import exact_system

pytestmark = pytest.mark.gpu
F_GRAD, F_LAP = 2, 4


def gpu_system(n_side, k, seed, nu=1.0):
    G = require_gpu()
    pts, bnd, nrm = W.stokes_cloud(n_side, 3, seed)
    c = ctx()
    x = dev(pts)
    flush(f"stokes: n={len(pts)} k={k}: search + stencils")
    rp, col, eps = G.gmls_neighbors(c, x, x, G.SEARCH_KNN, k=k, eps_mult=1.5)
    vlap, s1, _ = G.gmls_stencils(c, x, x, 2, G.BASIS_DIVFREE, F_LAP, 4, eps, rp, col, prec=G.PREC_FP64)
    grad, s2, _ = G.gmls_stencils(c, x, x, 3, G.BASIS_SCALAR, F_GRAD, 4, eps, rp, col, prec=G.PREC_FP64)
    plap, plap_t, s3, _ = G.gmls_stencils_staggered(c, x, x, 2, F_LAP, 4, eps, rp, col)
    nt = dev(nrm)
    nlap, nlap_h, s4, _ = G.gmls_stencils_constrained(c, x, x, 3, F_LAP, 4, eps, rp, col, nt)
    for s_ in (s1, s2, s3, s4):
        assert (host(s_) == 0).all()
    flush("stokes: assembly")
    bt = dev(bnd)
    arp, acol, aval = G.gmls_assemble_stokes(c, rp, col, bt, nt, vlap, grad, plap, plap_t.reshape(-1).contiguous(),
                                             nlap, nlap_h.reshape(-1).contiguous(), nu=nu)
    st = dict(rp=host(rp), col=host(col), vlap=host(vlap), grad=host(grad), plap=host(plap),
              plap_t=host(plap_t).reshape(-1), nlap=host(nlap), nlap_h=host(nlap_h).reshape(-1))
    return pts, bnd, nrm, (arp, acol, aval), st


def to_scipy(arp, acol, aval):
    rp, cl, vl = host(arp), host(acol), host(aval)
    R = len(rp) - 1
    A = sp.csr_matrix((vl, cl, rp), shape=(R, R))
    A.sum_duplicates()
    A.sort_indices()
    return A


@pytest.mark.parametrize("nu", [1.0, 0.3])
def test_manufactured_solution_on_gpu(nu):
    G = require_gpu()
    pts, bnd, nrm, (arp, acol, aval), st = gpu_system(12, 80, 5, nu)
    x, rhs = exact_system(pts, bnd, nrm, st["nlap_h"], nu)
    flush("stokes: spmv")
    y = host(G.gmls_spmv(ctx(), arp, acol, aval, dev(x)))
    A = to_scipy(arp, acol, aval)
    scale = abs(A) @ np.abs(x) + np.abs(rhs)
    rel = np.abs(y - rhs) / scale
    flush(f"  manufactured residual: max {rel.max():.3e} over {len(rel)} rows")
    assert rel.max() <= 1e-9


def test_assembly_matches_oracle_and_spmv_matches_scipy():
    G = require_gpu()
    pts, bnd, nrm, (arp, acol, aval), st = gpu_system(20, 60, 7)
    n = len(pts)
    assert n > 8192  # the multiplier row goes to the long-row kernel
    flush("stokes: oracle assembly of the GPU stencils")
    B = OK.assemble(n, 3, st["rp"], st["col"], bnd, nrm, st["vlap"], st["grad"], st["plap"], st["plap_t"], st["nlap"],
                    st["nlap_h"])
    B.sum_duplicates()
    B.sort_indices()
    A = to_scipy(arp, acol, aval)
    assert np.array_equal(A.indptr, B.indptr) and np.array_equal(A.indices, B.indices)
    np.testing.assert_allclose(A.data, B.data, rtol=1e-14, atol=1e-14 * np.abs(B.data).max())
    xr = W.rng(3).standard_normal(A.shape[0])
    flush("stokes: spmv vs scipy")
    y1 = host(G.gmls_spmv(ctx(), arp, acol, aval, dev(xr)))
    y2 = host(G.gmls_spmv(ctx(), arp, acol, aval, dev(xr)))
    assert np.array_equal(y1, y2)  # fixed summation order
    ref = A @ xr
    scale = abs(A) @ np.abs(xr)
    assert (np.abs(y1 - ref) / scale).max() <= 1e-14


def test_capacity_error():
    G = require_gpu()
    pts, bnd, nrm = W.stokes_cloud(4, 2, 1)
    c = ctx()
    x = dev(pts)
    rp, col, eps = G.gmls_neighbors(c, x, x, G.SEARCH_KNN, k=12, eps_mult=1.5)
    n = len(pts)
    z = lambda m: torch.zeros(m, dtype=torch.float64, device="cuda")
    st = G.StokesStencils(n, 2, 0, *[G._ptr(t).value for t in (rp, col, dev(bnd), dev(nrm), z(4 * col.numel()),
                                                              z(2 * col.numel()), z(col.numel()), z(n),
                                                              z(col.numel()), z(n))])
    import ctypes
    a_rp = torch.empty(3 * n + 2, dtype=torch.int64, device="cuda")
    a_col = torch.full((8,), -5, dtype=torch.int32, device="cuda")
    a_val = torch.full((8,), 7.0, dtype=torch.float64, device="cuda")
    nnz = ctypes.c_int64()
    rc = G.load_library().gmls_assemble_stokes(c._h, ctypes.byref(st), 1.0, G._ptr(a_rp), G._ptr(a_col),
                                               G._ptr(a_val), 8, ctypes.byref(nnz))
    assert rc == G.GMLS_ERR_CAPACITY and nnz.value > 8
    assert (host(a_col) == -5).all() and (host(a_val) == 7.0).all()
