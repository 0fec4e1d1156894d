"""Seeded synthetic point clouds, workload descriptions and test fields.

This module is shared by the CPU oracle tests and the GPU path.  It holds no
GMLS arithmetic: only random draws, grid layouts and the parameters of the
five benchmark workloads (point counts, search rules, basis order, kernel
power, functionals).

Point clouds follow the paper's manufactured-solution setting (Section 4:
quasi-uniform particles in a box), reshaped to the benchmark sizes:

* ``jittered_grid``: ``n`` nodes per side with ``n`` the smallest integer such
  that ``n**dim >= n_points``; spacing ``h = 1/n``; nodes at ``(i + 1/2) h`` in
  lexicographic order with x fastest; every coordinate jittered by
  ``U(-h/4, h/4)``; the first ``n_points`` nodes are kept.
* ``density_ramp``: points in ``[0,1]^3`` with density proportional to
  ``1 + 3x`` (a 4x variation along x), by rejection sampling in batches of
  ``2**22`` uniform draws; a draw ``u`` is kept when an independent uniform
  ``a`` satisfies ``a < (1 + 3 u_x) / 4``.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng",
    "jittered_grid",
    "density_ramp",
    "radius_for_mean_count",
    "WORKLOADS",
    "boundary_points",
    "stokes_cloud",
    "make_points",
    "random_poly_coeffs",
    "monomial_exponents",
]


def rng(seed: int) -> np.random.Generator:
    """PCG64 generator for ``seed`` (every input here is drawn from one)."""
    return np.random.Generator(np.random.PCG64(seed))


def jittered_grid(n_points: int, dim: int, seed: int, jitter: float = 0.25) -> np.ndarray:
    """Jittered uniform grid in ``[0,1]^dim``; float64 array ``[n_points, dim]``."""
    if n_points <= 0:
        return np.zeros((0, dim))
    n = 1
    while n ** dim < n_points:
        n += 1
    h = 1.0 / n
    axes = np.arange(n, dtype=np.float64)
    # 'ij' meshgrid flattens with the last axis fastest; reversing the axes
    # gives columns (x, y, z) with x fastest: index = ix + n*iy + n*n*iz.
    mesh = np.meshgrid(*([axes] * dim), indexing="ij")
    nodes = np.stack([m.reshape(-1) for m in mesh][::-1], axis=1)
    pts = (nodes + 0.5) * h
    g = rng(seed)
    pts = pts + g.uniform(-jitter * h, jitter * h, size=pts.shape)
    return np.ascontiguousarray(pts[:n_points])


def boundary_points(n_points: int, dim: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Points uniform on the boundary of [0,1]^dim (a face chosen uniformly,
    then a uniform point on it) and their outward unit normals."""
    g = rng(seed)
    face = g.integers(0, 2 * dim, size=n_points)
    pts = g.uniform(0.0, 1.0, size=(n_points, dim))
    nrm = np.zeros((n_points, dim))
    axis, side = face // 2, face % 2
    pts[np.arange(n_points), axis] = side.astype(np.float64)
    nrm[np.arange(n_points), axis] = np.where(side == 1, 1.0, -1.0)
    return np.ascontiguousarray(pts), nrm


def stokes_cloud(n_side: int, dim: int, seed: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Particles of [-1,1]^dim: a jittered n_side^dim grid inside (nodes
    (i + 1/2) h - 1, h = 2/n_side, jitter U(-h/4, h/4)), then on every face
    an n_side^(dim-1) grid of the same nodes jittered within the face.
    Returns (points, boundary flag uint8, outward unit normals)."""
    g = rng(seed)
    h = 2.0 / n_side
    ax = (np.arange(n_side) + 0.5) * h - 1.0
    inner = np.stack(np.meshgrid(*([ax] * dim), indexing="ij"), -1).reshape(-1, dim)[:, ::-1].copy()
    inner += g.uniform(-h / 4, h / 4, size=inner.shape)
    faces, nrms = [], []
    grid = np.stack(np.meshgrid(*([ax] * (dim - 1)), indexing="ij"), -1).reshape(-1, dim - 1)
    for axis in range(dim):
        for side in (-1.0, 1.0):
            f = np.zeros((len(grid), dim))
            others = [k for k in range(dim) if k != axis]
            f[:, others] = grid + g.uniform(-h / 4, h / 4, size=grid.shape)
            f[:, axis] = side
            nv = np.zeros((len(grid), dim))
            nv[:, axis] = side
            faces.append(f)
            nrms.append(nv)
    pts = np.concatenate([inner] + faces)
    nrm = np.concatenate([np.zeros_like(inner)] + nrms)
    bnd = np.concatenate([np.zeros(len(inner), np.uint8), np.ones(len(pts) - len(inner), np.uint8)])
    return np.ascontiguousarray(pts), bnd, np.ascontiguousarray(nrm)


def density_ramp(n_points: int, seed: int, batch: int = 1 << 22) -> np.ndarray:
    """Points in ``[0,1]^3`` with density proportional to ``1 + 3x``."""
    g = rng(seed)
    out = []
    have = 0
    while have < n_points:
        u = g.uniform(0.0, 1.0, size=(batch, 3))
        a = g.uniform(0.0, 1.0, size=batch)
        keep = u[a < (1.0 + 3.0 * u[:, 0]) / 4.0]
        out.append(keep)
        have += keep.shape[0]
    return np.ascontiguousarray(np.concatenate(out, axis=0)[:n_points])


def radius_for_mean_count(n_points: int, count_at_x0: float = 40.0) -> float:
    """Radius whose ball holds ``count_at_x0`` points on average at x = 0 for
    the ``1 + 3x`` density (normalised by its integral 2.5) in 3D."""
    return (count_at_x0 * 2.5 / (n_points * 4.0 * math.pi / 3.0)) ** (1.0 / 3.0)


# Functional bit mask (row order in the output: value, gradient, Laplacian,
# divergence).
F_VALUE, F_GRAD, F_LAPLACIAN, F_DIV = 1, 2, 4, 8

# The five benchmark workloads.  "search" is either ("knn", k, eps_mult) or
# ("radius", r0, k_min).  "bases" lists (basis, order, functional mask); all
# bases of a workload share one neighbour list.
WORKLOADS = {
    "c1_2d_m2": dict(
        n=1000, dim=2, seed=1001, gen="grid", search=("knn", 12, 1.5), p=4,
        bases=[("scalar", 2, F_GRAD | F_LAPLACIAN)], modes=("fp64",),
    ),
    "c2_2d_m4": dict(
        n=100_000, dim=2, seed=1002, gen="grid", search=("knn", 40, 1.5), p=4,
        bases=[("scalar", 4, F_VALUE | F_GRAD | F_LAPLACIAN)], modes=("fp64",),
        poly_seed=2002,
    ),
    "c3_3d_divfree_m2": dict(
        n=1_000_000, dim=3, seed=1003, gen="grid", search=("knn", 60, 1.5), p=4,
        bases=[("divfree", 2, F_LAPLACIAN), ("scalar", 2, F_GRAD)],
        modes=("mixed", "fp64"),
    ),
    "c4_3d_m3_uneven": dict(
        n=2_000_000, dim=3, seed=1004, gen="ramp",
        search=("radius", radius_for_mean_count(2_000_000), 30), p=4,
        bases=[("scalar", 3, F_LAPLACIAN)], modes=("mixed", "fp64"),
    ),
    "c5_3d_m4": dict(
        n=500_000, dim=3, seed=1005, gen="grid", search=("knn", 170, 1.5), p=6,
        bases=[("scalar", 4, F_GRAD | F_LAPLACIAN), ("divfree", 4, F_LAPLACIAN | F_DIV)],
        modes=("mixed", "fp64"),
    ),
    # the two variants of the pressure side (Sections 2.3 and 2.4), FP64 QR
    # path: staggered gradient + Laplacian of vector order 2 on the C4 cloud
    # and search, and Neumann-constrained Laplacian stencils (scalar order 3)
    # for 60 000 points on the faces of the unit cube (outward normals) with
    # kNN rows into the C3 cloud
    "s4_3d_staggered_m2": dict(
        n=2_000_000, dim=3, seed=1004, gen="ramp",
        search=("radius", radius_for_mean_count(2_000_000), 30), p=4,
        bases=[("staggered", 2, F_GRAD | F_LAPLACIAN)], modes=("mixed", "fp64"),
    ),
    "n3_3d_neumann_m3": dict(
        n=1_000_000, dim=3, seed=1003, gen="grid", targets=("boundary", 60_000, 1103),
        search=("knn", 80, 1.5), p=4,
        bases=[("neumann", 3, F_LAPLACIAN)], modes=("fp64",),
    ),
}


def make_points(name: str, n: int | None = None, seed: int | None = None) -> np.ndarray:
    """Point cloud of workload ``name`` (optionally resized or reseeded)."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    seed = w["seed"] if seed is None else seed
    if w["gen"] == "grid":
        return jittered_grid(n, w["dim"], seed)
    return density_ramp(n, seed)


def monomial_exponents(dim: int, degree: int) -> list[tuple[int, ...]]:
    """All exponent tuples of total degree <= ``degree`` (graded, then
    lexicographic descending).  Used to draw random test polynomials."""
    out = []
    for deg in range(degree + 1):
        def rec(prefix, left, k):
            if k == dim - 1:
                out.append(tuple(prefix + [left]))
                return
            for a in range(left, -1, -1):
                rec(prefix + [a], left - a, k + 1)
        rec([], deg, 0)
    return out


def random_poly_coeffs(dim: int, degree: int, count: int, seed: int) -> tuple[list, np.ndarray]:
    """``count`` random polynomials of total degree <= ``degree`` with N(0,1)
    coefficients on the plain monomials ``x^a y^b (z^c)``; returns the
    exponent list and a ``[count, n_monomials]`` coefficient array."""
    ex = monomial_exponents(dim, degree)
    c = rng(seed).standard_normal((count, len(ex)))
    return ex, c
