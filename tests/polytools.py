"""Tiny exact polynomial helpers for the tests: a polynomial is a dict
{exponent tuple: coefficient}.  Derivatives are the textbook rules for
monomials; nothing here is shared with the oracle or the GPU path."""
from __future__ import annotations

import numpy as np


def from_terms(terms, dim=3):
    p = {}
    for coef, e in terms:
        e = tuple(e[:dim])
        p[e] = p.get(e, 0.0) + float(coef)
    return p


def deriv(p, axis, times=1):
    out = p
    for _ in range(times):
        q = {}
        for e, c in out.items():
            if e[axis] == 0:
                continue
            ne = list(e)
            ne[axis] -= 1
            ne = tuple(ne)
            q[ne] = q.get(ne, 0.0) + c * e[axis]
        out = q
    return out


def add(*ps):
    q = {}
    for p in ps:
        for e, c in p.items():
            q[e] = q.get(e, 0.0) + c
    return {e: c for e, c in q.items() if c != 0.0}


def laplacian(p, dim):
    return add(*[deriv(p, i, 2) for i in range(dim)])


def evaluate(p, x):
    """Values at points x [n, dim]; also returns the sum of |terms| (the
    rounding scale of the evaluation)."""
    x = np.atleast_2d(x)
    v = np.zeros(x.shape[0])
    for e, c in p.items():
        t = np.full(x.shape[0], c)
        for i, a in enumerate(e):
            t = t * x[:, i] ** a
        v = v + t
    return v


def same(p, q, tol=0.0):
    keys = set(p) | set(q)
    return all(abs(p.get(k, 0.0) - q.get(k, 0.0)) <= tol for k in keys)


def random_poly(dim, degree, rng):
    p = {}
    for deg in range(degree + 1):
        def rec(prefix, left, k):
            if k == dim - 1:
                p[tuple(prefix + [left])] = rng.standard_normal()
                return
            for a in range(left, -1, -1):
                rec(prefix + [a], left - a, k + 1)
        rec([], deg, 0)
    return p
