"""Global Stokes operator of Section 3.2 from stencils, plain numpy/scipy --
TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module (through the ``oracle`` package); the
product library never calls it and shares no code with it.

Section 3.2 assembles the stencils into the block system
[K G 0; N L 1; 0 1 0] [v; phi; lambda] = [b; g; 0].  Unknowns and rows are
ordered v_(J,c) at J*d + c, phi_J at d*n + J, lambda at d*n + n.  With nu the
viscosity, the Stokes equations -nu Laplacian v + grad phi = f, div v = 0, the
pressure Poisson equation Laplacian phi = div f, v = w and the Neumann data
h = n.f + nu n.Laplacian v on the boundary (Section 3.2 with Section 2.3's
constrained solution: Laplacian phi(x_I) = sum_j L^n phi_j + beta_I h_I):

  interior velocity (I, c):  K = -nu L^v (vector Laplacian), G = grad
  boundary velocity (I, c):  K = identity
  interior pressure I:       L = staggered Laplacian, plus its target weight
                             on phi_I, and 1 in the multiplier column
  boundary pressure I:       N = nu beta_I n_I . L^v, L = constrained
                             Laplacian, 1 in the multiplier column
  multiplier row:            1 for every phi_J (zero-mean pressure)

Readings: the multiplier row's diagonal is 0 (the printed corner entry is
read as a typesetting slip); the boundary coupling N carries the h-weight
beta_I, as in the equation the block is derived from.  Entries with the same
column in one row are summed.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def assemble(n, dim, row_ptr, col, boundary, normals, vlap, grad, plap, plap_t, nlap, nlap_h, nu=1.0):
    """CSR matrix (scipy) of the block system; stencil arrays in the library's
    layouts (target t owns F*C*row_ptr[t]..., entry (f*N + j)*C + c)."""
    d = dim
    rows, cols, vals = [], [], []
    pc = d * n  # column of phi_0
    lam = d * n + n
    for I in range(n):
        b, e = int(row_ptr[I]), int(row_ptr[I + 1])
        N = e - b
        J = np.asarray(col[b:e], dtype=np.int64)
        Lv = np.asarray(vlap[d * d * b:d * d * e]).reshape(d, N, d)  # [c, j, c']
        if boundary[I]:
            for c in range(d):
                rows.append([I * d + c]); cols.append([I * d + c]); vals.append([1.0])
            nL = np.einsum("c,cjk->jk", np.asarray(normals[I], dtype=np.float64), Lv)  # n_I . L^v
            r = pc + I
            rows.append(np.full(N * d, r)); cols.append((J[:, None] * d + np.arange(d)[None, :]).ravel())
            vals.append((nu * nlap_h[I] * nL).ravel())
            rows.append(np.full(N, r)); cols.append(pc + J); vals.append(np.asarray(nlap[b:e]))
            rows.append([r]); cols.append([lam]); vals.append([1.0])
        else:
            G = np.asarray(grad[d * b:d * e]).reshape(d, N)
            for c in range(d):
                r = I * d + c
                rows.append(np.full(N * d, r)); cols.append((J[:, None] * d + np.arange(d)[None, :]).ravel())
                vals.append((-nu * Lv[c]).ravel())
                rows.append(np.full(N, r)); cols.append(pc + J); vals.append(G[c])
            r = pc + I
            rows.append(np.full(N, r)); cols.append(pc + J); vals.append(np.asarray(plap[b:e]))
            rows.append([r]); cols.append([pc + I]); vals.append([plap_t[I]])
            rows.append([r]); cols.append([lam]); vals.append([1.0])
    rows.append(np.full(n, lam)); cols.append(pc + np.arange(n)); vals.append(np.ones(n))
    R = d * n + n + 1
    A = sp.coo_matrix((np.concatenate([np.asarray(v, dtype=np.float64) for v in vals]),
                       (np.concatenate([np.asarray(v, dtype=np.int64) for v in rows]),
                        np.concatenate([np.asarray(v, dtype=np.int64) for v in cols]))), shape=(R, R))
    return A.tocsr()
