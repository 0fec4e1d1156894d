"""Neumann-constrained GMLS stencils, plain numpy -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module (through the ``oracle`` package); the
product library never calls it and shares no code with it.

Definition (Section 2.3, the bordered system of the constrained local
problem): for target T with neighbours j, scaled Taylor basis
p_a(x) = prod_i ((x_i - xT_i)/eps)^a_i / a_i! (Section 2.1), weights
w_j = (1 - r_j/eps)^p (r_j < eps), and outward normal n, the fit c minimises
sum_j w_j (u_j - p(x_j).c)^2 subject to n . grad(p(x).c)|_{x_T} = h.  Its
Lagrange system is

    [A    F] [c ]   [P^T W u]        A = P^T W P,
    [F^T  0] [mu] = [h      ],       F = grad p(x_T)^T n.

A functional lambda applied to the fit is lambda^T c = alpha.u + beta h.  With
K the bordered matrix (symmetric) and [g; gamma] = K^-1 [lambda; 0]:
lambda^T c = g^T P^T W u + gamma h, so alpha = W P g and beta = gamma.  Each
target is one dense (Q+1)x(Q+1) solve by Gaussian elimination with partial
pivoting; nothing is blocked, fused or reordered.

Precision: A = P^T W P squares the conditioning of the weighted sample matrix,
so an FP64 solve of the bordered system loses about cond(A) * 2^-53 relative
accuracy (1e-10 at order 3 in 3-D), the size of the parity gate itself.  The
basis, the Gram matrix and the elimination are therefore carried in x87
extended precision (numpy.longdouble, 64-bit significand), which leaves the
oracle's own error near 1e-13; the results are returned in FP64.

A zero normal leaves the target unconstrained: alpha = W P A^-1 lambda,
beta = 0.
"""
from __future__ import annotations

import math

import numpy as np

F_VALUE, F_GRAD, F_LAPLACIAN = 1, 2, 4


def exponents(dim: int, order: int) -> np.ndarray:
    """Monomial exponents of total degree <= order: graded, and within a
    degree descending powers of x, then of y."""
    out = []
    for deg in range(order + 1):
        if dim == 1:
            out.append((deg, 0, 0))
        elif dim == 2:
            for a in range(deg, -1, -1):
                out.append((a, deg - a, 0))
        else:
            for a in range(deg, -1, -1):
                for b in range(deg - a, -1, -1):
                    out.append((a, b, deg - a - b))
    return np.array(out, dtype=np.int64)


def basis(s: np.ndarray, ex: np.ndarray) -> np.ndarray:
    """P[j, a] = prod_i s_ji^a_i / a_i! for scaled offsets s [N, dim]."""
    dim = s.shape[1]
    P = np.ones((s.shape[0], len(ex)), dtype=s.dtype)
    for a, e in enumerate(ex):
        for i in range(dim):
            if e[i]:
                P[:, a] *= s[:, i] ** int(e[i]) / math.factorial(int(e[i]))
    return P


def functionals(dim: int, ex: np.ndarray, mask: int, eps: float) -> np.ndarray:
    """Rows lambda_f[a] = (D_f p_a)(x_T) in the order value, gradient,
    Laplacian (Section 2.5: derivatives act on the basis at x_T)."""
    rows = []
    unit = [tuple(1 if i == k else 0 for i in range(3)) for k in range(3)]
    two = [tuple(2 if i == k else 0 for i in range(3)) for k in range(3)]
    exl = [tuple(e) for e in ex]
    if mask & F_VALUE:
        rows.append([1.0 if e == (0, 0, 0) else 0.0 for e in exl])
    if mask & F_GRAD:
        for k in range(dim):
            rows.append([1.0 / eps if e == unit[k] else 0.0 for e in exl])
    if mask & F_LAPLACIAN:
        rows.append([sum(1.0 / eps**2 for k in range(dim) if e == two[k]) for e in exl])
    return np.array(rows)


def _solve(K: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """K x = rhs by Gaussian elimination with partial pivoting, in the dtype
    of K (the bordered matrix is symmetric indefinite, so pivoting is needed)."""
    K = K.copy()
    x = rhs.copy()
    n = K.shape[0]
    for k in range(n):
        piv = k + int(np.argmax(np.abs(K[k:, k])))
        if piv != k:
            K[[k, piv]] = K[[piv, k]]
            x[[k, piv]] = x[[piv, k]]
        if K[k, k] == 0:
            raise np.linalg.LinAlgError("singular bordered system")
        m = K[k + 1:, k] / K[k, k]
        K[k + 1:, k:] -= np.outer(m, K[k, k:])
        x[k + 1:] -= np.outer(m, x[k])
    for k in range(n - 1, -1, -1):
        x[k] = (x[k] - K[k, k + 1:] @ x[k + 1:]) / K[k, k]
    return x


def constrained_target(xs: np.ndarray, xt: np.ndarray, eps: float, p: int, order: int, mask: int,
                       normal: np.ndarray):
    """(alpha [F, N], beta [F]) of one target from its neighbours xs [N, dim]."""
    LD = np.longdouble
    dim = xs.shape[1]
    ex = exponents(dim, order)
    eps_l = LD(eps)
    s = (xs.astype(LD) - xt.astype(LD)) / eps_l
    r = np.sqrt(np.sum(s * s, axis=1))
    w = np.where(r < 1, (1 - r) ** p, LD(0))
    P = basis(s, ex)
    A = P.T @ (w[:, None] * P)
    lam = functionals(dim, ex, mask, eps_l).astype(LD)
    Q = len(ex)
    if not np.any(normal):
        g = _solve(A, lam.T.copy())  # [Q, F]
        return (w[:, None] * (P @ g)).T.astype(np.float64), np.zeros(lam.shape[0])
    Fv = np.zeros(Q, dtype=LD)
    for k in range(dim):
        e = tuple(1 if i == k else 0 for i in range(3))
        a = [tuple(v) for v in ex].index(e)
        Fv[a] = LD(normal[k]) / eps_l
    K = np.zeros((Q + 1, Q + 1), dtype=LD)
    K[:Q, :Q] = A
    K[:Q, Q] = Fv
    K[Q, :Q] = Fv
    rhs = np.zeros((Q + 1, lam.shape[0]), dtype=LD)
    rhs[:Q, :] = lam.T
    sol = _solve(K, rhs)  # [Q+1, F]
    g, gamma = sol[:Q, :], sol[Q, :]
    return (w[:, None] * (P @ g)).T.astype(np.float64), gamma.astype(np.float64)


def stencils_constrained(src, tgt, order: int, mask: int, p: int, eps, row_ptr, col, normals):
    """Weights in the library's layout (target t owns F*row_ptr[t]..., entry
    f*N + j) and beta [n_tgt, F]."""
    src = np.asarray(src, dtype=np.float64)
    tgt = np.asarray(tgt, dtype=np.float64)
    normals = np.asarray(normals, dtype=np.float64)
    n_tgt = tgt.shape[0]
    F = functionals(src.shape[1], exponents(src.shape[1], order), mask, 1.0).shape[0]
    w = np.zeros(F * int(row_ptr[-1]))
    beta = np.zeros((n_tgt, F))
    for t in range(n_tgt):
        b, e = int(row_ptr[t]), int(row_ptr[t + 1])
        alpha, bt = constrained_target(src[col[b:e]], tgt[t], float(eps[t]), p, order, mask, normals[t])
        w[F * b:F * e] = alpha.reshape(-1)
        beta[t] = bt
    return w, beta, F
