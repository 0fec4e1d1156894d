"""Pin of the Stokes assembly oracle (oracle/stokes.py) with the paper's
quadratic manufactured solution of Section 4.1: velocity v2 (divergence
free), pressure phi2 (cubic), both closed forms in tests/golden/.  With the
oracle's stencils (divergence-free order 2 vector Laplacian, scalar order 3
gradient, staggered order 2 Laplacian, Neumann-constrained order 3 Laplacian)
every one of them is exact on these fields, so the assembled operator applied
to the exact nodal values must return the right-hand side built from
f = -nu Laplacian v2 + grad phi2 and its divergence (Laplacian phi2) to
rounding, in every row: interior and boundary velocity and pressure rows and
the zero-mean multiplier row.  A wrong sign or a missing h-weight in the
boundary coupling fails the boundary pressure rows."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import constrained as OC
from oracle import staggered as OS
from oracle import stokes as OK
from tests.manufactured import exact_system

F_GRAD, F_LAP = 2, 4


def oracle_stencils(pts, nrm, rp, col, eps):
    vlap, st1, _, _ = oracle.stencils(pts, pts, 2, "divfree", F_LAP, 4, eps, rp, col)
    grad, st2, _, _ = oracle.stencils(pts, pts, 3, "scalar", F_GRAD, 4, eps, rp, col)
    plap, plap_t, _ = OS.stencils_staggered(pts, pts, 2, F_LAP, 4, eps, rp, col)
    nlap, nlap_h, _ = OC.stencils_constrained(pts, pts, 3, F_LAP, 4, eps, rp, col, nrm)
    assert (st1 == 0).all() and (st2 == 0).all()
    return vlap, grad, plap, plap_t[:, 0], nlap, nlap_h[:, 0]


@pytest.mark.parametrize("nu", [1.0, 0.3])
def test_manufactured_solution_residual(nu):
    pts, bnd, nrm = W.stokes_cloud(8, 3, 11)
    rp, col, eps = oracle.knn(pts, pts, 80, 1.5)
    vlap, grad, plap, plap_t, nlap, nlap_h = oracle_stencils(pts, nrm, rp, col, eps)
    A = OK.assemble(len(pts), 3, rp, col, bnd, nrm, vlap, grad, plap, plap_t, nlap, nlap_h, nu)
    x, rhs = exact_system(pts, bnd, nrm, nlap_h, nu)
    r = A @ x - rhs
    scale = abs(A) @ np.abs(x) + np.abs(rhs)
    rel = np.abs(r) / scale
    assert rel.max() <= 1e-9, (rel.max(), int(np.argmax(rel)))


def test_row_structure():
    pts, bnd, nrm = W.stokes_cloud(5, 2, 3)
    n, d = pts.shape
    rp, col, eps = oracle.knn(pts, pts, 20, 1.5)
    N = np.diff(rp)
    z = lambda m: np.zeros(m)
    A = OK.assemble(n, d, rp, col, bnd, nrm, z(d * d * rp[-1]), z(d * rp[-1]), z(rp[-1]), z(n), z(rp[-1]), z(n))
    A.eliminate_zeros()
    nnz_row = np.diff(A.indptr)
    for I in range(n):
        if bnd[I]:
            assert list(nnz_row[I * d:(I + 1) * d]) == [1] * d
            assert nnz_row[d * n + I] == 1  # only the multiplier survives with zero weights
        else:
            assert nnz_row[d * n + I] == 1
    assert nnz_row[-1] == n and A[d * n + n, d * n + n] == 0
