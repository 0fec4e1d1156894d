"""Pins for the oracle's neighbour search (support ball of Section 2.1).

The oracle's brute-force search is checked against the definition written
with numpy sorts on tiny clouds, its bucket grid against its brute force
(including exact-grid ties, degenerate extents and targets outside the
cloud), and both against scipy's k-d tree on jittered clouds."""
import numpy as np
import pytest

import oracle
import workloads as W


def d2_np(src, x):
    d = src - x
    s = d[:, 0] * d[:, 0]
    for i in range(1, src.shape[1]):
        s = s + d[:, i] * d[:, i]
    return s


def knn_definition(src, tgt, k):
    rows = []
    for x in tgt:
        d2 = d2_np(src, x)
        order = np.lexsort((np.arange(len(src)), d2))
        rows.append(order[:k])
    return np.array(rows)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("k", [1, 5, 17])
def test_knn_brute_matches_definition(dim, k):
    g = W.rng(11 + dim)
    src = g.uniform(size=(300, dim))
    tgt = np.concatenate([src[:40], g.uniform(-0.2, 1.2, size=(20, dim))])
    rp, col, eps = oracle.knn(src, tgt, k, 1.5, use_grid=False)
    ref = knn_definition(src, tgt, k)
    assert np.array_equal(col.reshape(-1, k), ref)
    dk = np.sqrt(np.array([d2_np(src, x)[r[-1]] for x, r in zip(tgt, ref)]))
    assert np.array_equal(eps, 1.5 * dk)


def test_knn_exact_grid_ties_lexicographic():
    # unjittered grid: many equal distances, resolved by source index
    n = 12
    ax = (np.arange(n) + 0.5) / n
    src = np.stack(np.meshgrid(ax, ax, indexing="ij"), -1).reshape(-1, 2)[:, ::-1].copy()
    for k in (5, 9, 13, 21):
        _, col, _ = oracle.knn(src, src, k, 1.5, use_grid=False)
        assert np.array_equal(col.reshape(-1, k), knn_definition(src, src, k))
        _, colg, _ = oracle.knn(src, src, k, 1.5, use_grid=True)
        assert np.array_equal(colg, col)


@pytest.mark.parametrize("case", ["grid2d", "grid3d", "ramp", "plane", "cluster"])
def test_knn_grid_equals_brute(case):
    g = W.rng(7)
    if case == "grid2d":
        src = W.jittered_grid(3000, 2, 5)
    elif case == "grid3d":
        src = W.jittered_grid(4000, 3, 6)
    elif case == "ramp":
        src = W.density_ramp(4000, 9)
    elif case == "plane":
        src = g.uniform(size=(3000, 3))
        src[:, 2] = 0.5
    else:
        src = np.concatenate([g.normal(0.3, 0.01, size=(1500, 3)), g.uniform(size=(1500, 3))])
    tgt = np.concatenate([src[::7], g.uniform(-0.3, 1.3, size=(50, src.shape[1]))])
    for k in (1, 12, 60):
        _, cb, eb = oracle.knn(src, tgt, k, 1.5, use_grid=False)
        _, cg, eg = oracle.knn(src, tgt, k, 1.5, use_grid=True)
        assert np.array_equal(cb, cg)
        assert np.array_equal(eb, eg)


def test_knn_matches_kdtree():
    from scipy.spatial import cKDTree

    src = W.jittered_grid(20000, 3, 1003)
    tgt = src[::13]
    k = 60
    _, col, eps = oracle.knn(src, tgt, k, 1.5)
    dist, idx = cKDTree(src).query(tgt, k=k)
    assert np.array_equal(np.sort(col.reshape(-1, k), 1), np.sort(idx, 1))
    np.testing.assert_allclose(eps, 1.5 * dist[:, -1], rtol=1e-14)


def radius_definition(src, tgt, r0, k_min):
    rows, eps = [], []
    for x in tgt:
        d2 = d2_np(src, x)
        order = np.lexsort((np.arange(len(src)), d2))
        inside = order[d2[order] < r0 * r0]
        if len(inside) >= k_min:
            rows.append(np.sort(inside))
            eps.append(r0)
        else:
            rows.append(np.sort(order[:k_min]))
            eps.append(0.5 * (np.sqrt(d2[order[k_min - 1]]) + np.sqrt(d2[order[k_min]])))
    return rows, np.array(eps)


@pytest.mark.parametrize("use_grid", [False, True])
def test_radius_matches_definition(use_grid):
    src = W.density_ramp(3000, 21)
    g = W.rng(3)
    tgt = np.concatenate([src[:200], g.uniform(-0.1, 1.1, size=(30, 3))])
    r0 = W.radius_for_mean_count(3000)
    k_min = 30
    rp, col, eps = oracle.radius(src, tgt, r0, k_min, use_grid=use_grid)
    rows, ref_eps = radius_definition(src, tgt, r0, k_min)
    assert np.array_equal(np.diff(rp), [len(r) for r in rows])
    assert np.array_equal(col, np.concatenate(rows))
    assert np.array_equal(eps, ref_eps)
    # both branches of the floor rule are exercised
    assert (np.diff(rp) == k_min).any() and (np.diff(rp) > k_min).any()


def test_radius_grid_equals_brute_ramp():
    n = 20000
    src = W.density_ramp(n, 1004)
    tgt = src[::5]
    r0 = W.radius_for_mean_count(n)
    a = oracle.radius(src, tgt, r0, 30, use_grid=False)
    b = oracle.radius(src, tgt, r0, 30, use_grid=True)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    counts = np.diff(a[0])
    # density ramp: interior counts span roughly 40 (x = 0) to 160 (x = 1)
    assert counts.min() >= 30 and 150 < counts.max() < 260
