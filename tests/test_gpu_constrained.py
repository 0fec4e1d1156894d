"""Neumann-constrained stencils on the GPU (FP64 Householder path) against the
constrained oracle: alpha and beta per target and functional row, gate 1e-10
relative to the row norm.  Also: a zero normal reproduces gmls_stencils
exactly, the mixed precision is refused, and an empty target set is a no-op.

Targets on a cube face near an edge or corner see a one-sided neighbourhood;
at order 4 in 3-D the weighted sample matrix W^1/2 P reaches cond 3e6 there,
and any FP64 method (the GPU's Householder QR, the oracle's extended-precision
solve) is then only accurate to O(cond 2^-53).  The gate per target is
therefore max(1e-10, 4 cond 2^-53), which is the plain 1e-10 gate up to cond
2.2e5 (every target of the order <= 3 cases)."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import constrained as OC
from tests.gpu_helpers import ctx, dev, flush, host, require_gpu, row_errors

pytestmark = pytest.mark.gpu

TOL = 1e-10
MASK = 1 | 2 | 4  # value, gradient, Laplacian


def case(dim, n_src, n_tgt, k, seed):
    src = W.jittered_grid(n_src, dim, seed)
    tgt, nrm = W.boundary_points(n_tgt, dim, seed + 1)
    return src, tgt, nrm, oracle.knn(src, tgt, k, 1.5)


@pytest.mark.parametrize("dim,order,k,n_tgt", [(2, 2, 16, 300), (2, 4, 40, 257), (3, 2, 30, 300),
                                               (3, 3, 55, 321), (3, 4, 90, 130)])
def test_constrained_parity(dim, order, k, n_tgt):
    G = require_gpu()
    src, tgt, nrm, (rp, col, eps) = case(dim, 6000 if dim == 2 else 20000, n_tgt, k, 40 + order)
    nrm[::7] = 0.0  # some unconstrained targets in the same launch
    flush(f"constrained dim={dim} m={order} k={k} n_tgt={n_tgt}")
    w, hw, st, _ = G.gmls_stencils_constrained(ctx(), dev(src), dev(tgt), order, MASK, 4, dev(eps), dev(rp),
                                               dev(col), dev(nrm))
    w, hw, st = host(w), host(hw), host(st)
    ow, ob, F = OC.stencils_constrained(src, tgt, order, MASK, 4, eps, rp, col, nrm)
    assert (st == 0).all()
    errs = row_errors(w, ow, rp, F, 1)
    ex = OC.exponents(dim, order)
    cond = np.empty(len(tgt))
    for t in range(len(tgt)):
        sc = (src[col[rp[t]:rp[t + 1]]] - tgt[t]) / eps[t]
        r = np.linalg.norm(sc, axis=1)
        cond[t] = np.linalg.cond(np.sqrt(np.where(r < 1, (1 - r) ** 4, 0.0))[:, None] * OC.basis(sc, ex))
    tol = np.maximum(TOL, 4 * cond * 2.0 ** -53)[:, None]
    # beta relative to the norm of the whole functional row [alpha, beta]
    # (the gradient component along the normal has alpha = 0, beta = 1/n_k)
    scale = np.array([[np.hypot(np.linalg.norm(ow[F * rp[t] + f * (rp[t + 1] - rp[t]):
                                                   F * rp[t] + (f + 1) * (rp[t + 1] - rp[t])]), ob[t, f])
                       for f in range(F)] for t in range(len(tgt))])
    berr = np.abs(hw - ob) / np.where(scale > 0, scale, 1.0)
    flush(f"  max rel err alpha {errs.max():.3e} beta {berr.max():.3e}  max cond {cond.max():.2e}; "
          f"at cond <= 1e5: alpha {errs[cond <= 1e5].max():.3e}")
    assert np.all(errs <= tol) and np.all(berr <= tol)
    assert not hw[::7].any()


def test_zero_normals_equal_plain_stencils():
    G = require_gpu()
    src, tgt, nrm, (rp, col, eps) = case(3, 20000, 400, 60, 3)
    args = (ctx(), dev(src), dev(tgt), 3)
    w0, st0, _ = G.gmls_stencils(*args, G.BASIS_SCALAR, MASK, 4, dev(eps), dev(rp), dev(col), prec=G.PREC_FP64)
    w1, hw, st1, _ = G.gmls_stencils_constrained(*args, MASK, 4, dev(eps), dev(rp), dev(col),
                                                 dev(np.zeros_like(nrm)))
    assert np.array_equal(host(w0), host(w1)) and np.array_equal(host(st0), host(st1))
    assert not host(hw).any()


def test_constrained_mixed_is_refused_and_empty_is_noop():
    G = require_gpu()
    src, tgt, nrm, (rp, col, eps) = case(2, 3000, 50, 16, 8)
    with pytest.raises(G.GmlsError) as e:
        G.gmls_stencils_constrained(ctx(), dev(src), dev(tgt), 2, MASK, 4, dev(eps), dev(rp), dev(col), dev(nrm),
                                    prec=G.PREC_MIXED)
    assert e.value.status == G.GMLS_ERR_UNSUPPORTED
    empty = np.zeros((0, 2))
    w, hw, st, _ = G.gmls_stencils_constrained(ctx(), dev(src), dev(empty), 2, MASK, 4, dev(np.zeros(0)),
                                               dev(np.zeros(1, dtype=np.int64)), dev(np.zeros(0, dtype=np.int32)),
                                               dev(empty))
    assert w.numel() == 0 and hw.shape[0] == 0 and st.numel() == 0
