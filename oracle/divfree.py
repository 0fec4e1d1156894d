"""Divergence-free vector polynomial bases for the oracle (Section 2.2).

A vector polynomial of degree <= m is written in the coefficients of
``p_a e_c`` (scaled monomial ``p_a`` of the oracle's ordering, component
``c``); the coefficient row index is ``a*dim + c``.  Because
``d/ds_c (s^a/a!) = s^(a-e_c)/(a-e_c)!``, the divergence maps ``p_a e_c`` to
the monomial ``p_(a-e_c)`` with coefficient exactly one (zero when
``a_c = 0``).  The space of divergence-free fields is the kernel of that
integer matrix; its dimension is ``dim*C(m+dim, dim) - C(m-1+dim, dim)``.

``nullspace_basis`` is the oracle's basis: an orthonormal kernel basis from
an SVD.  ``explicit_basis`` is an independent +-1 construction (each field is
one monomial in one component, balanced by at most one monomial in the first
component) and ``paper_2d_order2`` is the nine-field list the paper prints for
d = 2, m = 2; they exist to pin the oracle's basis by span (any spanning set
yields the same stencil).
"""
from __future__ import annotations

from math import comb

import numpy as np


def _monomials(dim, order):
    from . import monomials

    return monomials(dim, order)


def dimension(dim: int, order: int) -> int:
    return dim * comb(order + dim, dim) - (comb(order - 1 + dim, dim) if order >= 1 else 0)


def divergence_matrix(dim: int, order: int) -> np.ndarray:
    """Integer matrix ``[C(m-1+d,d), d*C(m+d,d)]`` of the divergence map."""
    ex = _monomials(dim, order)
    low = _monomials(dim, order - 1) if order >= 1 else np.zeros((0, dim), np.int32)
    index = {tuple(e): i for i, e in enumerate(low)}
    D = np.zeros((len(low), len(ex) * dim))
    for a, e in enumerate(ex):
        for c in range(dim):
            if e[c] >= 1:
                b = list(e)
                b[c] -= 1
                D[index[tuple(b)], a * dim + c] = 1.0
    return D


def nullspace_basis(dim: int, order: int) -> np.ndarray:
    """Orthonormal basis of the divergence-free fields, ``[d*Q_s, Q_d]``."""
    D = divergence_matrix(dim, order)
    n = D.shape[1]
    if D.shape[0] == 0:
        return np.eye(n)
    _, s, vt = np.linalg.svd(D)
    rank = int(np.sum(s > 1e-10 * s[0]))
    return np.ascontiguousarray(vt[rank:].T)


def explicit_basis(dim: int, order: int) -> np.ndarray:
    """+-1 basis, ``[d*Q_s, Q_d]``: for every monomial p_b and component
    c >= 1 the field p_b e_c - p_(b - e_c + e_x) e_x (second term only when
    b_c >= 1), plus p_g e_x for every g with g_x = 0."""
    ex = _monomials(dim, order)
    index = {tuple(e): i for i, e in enumerate(ex)}
    cols = []
    for deg in range(order + 1):
        for a, e in enumerate(ex):
            if sum(e) != deg:
                continue
            for c in range(1, dim):
                v = np.zeros(len(ex) * dim)
                v[a * dim + c] = 1.0
                if e[c] >= 1:
                    b = list(e)
                    b[c] -= 1
                    b[0] += 1
                    v[index[tuple(b)] * dim + 0] = -1.0
                cols.append(v)
            if e[0] == 0:
                v = np.zeros(len(ex) * dim)
                v[a * dim + 0] = 1.0
                cols.append(v)
    return np.stack(cols, axis=1)


def paper_2d_order2() -> np.ndarray:
    """The nine divergence-free fields listed for d = 2, m = 2 in Section 2.2,
    in the scaled-monomial coefficients (x^2 = 2 p_(2,0), xy = p_(1,1),
    y^2 = 2 p_(0,2))."""
    ex = _monomials(2, 2)
    index = {tuple(e): i for i, e in enumerate(ex)}

    def field(*terms):
        v = np.zeros(len(ex) * 2)
        for coef, e, c in terms:
            v[index[e] * 2 + c] += coef
        return v

    fields = [
        field((1, (0, 0), 0)),                      # (1, 0)
        field((1, (0, 0), 1)),                      # (0, 1)
        field((1, (0, 1), 0)),                      # (y, 0)
        field((1, (1, 0), 1)),                      # (0, x)
        field((1, (1, 0), 0), (-1, (0, 1), 1)),     # (x, -y)
        field((2, (0, 2), 0)),                      # (y^2, 0)
        field((2, (2, 0), 1)),                      # (0, x^2)
        field((2, (2, 0), 0), (-2, (1, 1), 1)),     # (x^2, -2xy)
        field((-2, (1, 1), 0), (2, (0, 2), 1)),     # (-2xy, y^2)
    ]
    return np.stack(fields, axis=1)
