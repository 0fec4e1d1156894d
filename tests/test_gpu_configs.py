"""The five workload configurations at full size, in the launch configuration
bench.py uses (search over the whole cloud, then stencils over every target).

Parity is checked on sampled targets that the oracle computes one by one:
128 random targets plus the longest and shortest rows and the first and last
targets.  Neighbour rows must be identical (bit-exact indices and ε);
weights must meet the gates (FP64 path 1e-10, mixed 1e-8, per target and
functional row).  Configuration C2 also checks a property at every target:
the GPU weights, applied by gmls_apply, reproduce the derivatives of random
degree-4 polynomials (closed form) to 1e-10 of the rounding scale."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests import polytools as PT
from tests.gpu_helpers import ctx, dev, flush, host, require_gpu, row_errors, row_sorted

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-8}
_cache = {}


def search(name):
    """GPU neighbour lists of a configuration, checked against the oracle on
    the sampled targets (cached per configuration)."""
    if name in _cache:
        return _cache[name]
    G = require_gpu()
    w = W.WORKLOADS[name]
    pts = W.make_points(name)
    n = len(pts)
    s = dev(pts)
    flush(f"[{name}] search n={n} {w['search']}")
    if w["search"][0] == "knn":
        k, mult = w["search"][1], w["search"][2]
        rp, col, eps = G.gmls_neighbors(ctx(), s, s, G.SEARCH_KNN, k=k, eps_mult=mult)
    else:
        r0, kmin = w["search"][1], w["search"][2]
        rp, col, eps = G.gmls_neighbors(ctx(), s, s, G.SEARCH_RADIUS, radius=r0, k_min=kmin)
    rph, epsh = host(rp), host(eps)
    lens = np.diff(rph)
    g = W.rng(777)
    sample = set(g.choice(n, size=min(128, n), replace=False).tolist())
    sample |= {int(np.argmax(lens)), int(np.argmin(lens)), 0, n - 1}
    sample = np.array(sorted(sample))
    # the sampled rows, gathered on the device
    idx = np.concatenate([np.arange(rph[t], rph[t + 1]) for t in sample])
    colh = host(col[torch.from_numpy(idx).cuda()])
    srp = np.zeros(len(sample) + 1, dtype=np.int64)
    srp[1:] = np.cumsum(lens[sample])
    if w["search"][0] == "knn":
        orp, ocol, oeps = oracle.knn(pts, pts[sample], k, mult)
    else:
        orp, ocol, oeps = oracle.radius(pts, pts[sample], r0, kmin)
    assert np.array_equal(srp, orp), "row lengths differ from the oracle"
    if w["search"][0] == "knn":
        assert np.array_equal(colh, ocol), "neighbour indices differ from the oracle"
    else:  # radius rows are sets (cell order on the GPU, index order in the oracle)
        assert np.array_equal(row_sorted(srp, colh), ocol), "neighbour sets differ from the oracle"
    assert np.array_equal(epsh[sample], oeps), "support radii differ from the oracle"
    flush(f"  search ok: nnz={col.numel()} rows {lens.min()}..{lens.max()}")
    _cache[name] = (pts, s, rp, col, eps, rph, sample, srp, colh, epsh[sample])
    return _cache[name]


def sampled_weights(wt, rph, sample, F, C):
    idx = np.concatenate([np.arange(F * C * rph[t], F * C * rph[t + 1]) for t in sample])
    return host(wt[torch.from_numpy(idx).cuda()])


# the five configurations (targets = sources, plain scalar / divergence-free bases)
CONFIGS = {name: w for name, w in W.WORKLOADS.items()
           if "targets" not in w and all(b[0] in ("scalar", "divfree") for b in w["bases"])}
CASES = [(name, bi, mode) for name, w in CONFIGS.items() for bi in range(len(w["bases"])) for mode in w["modes"]]


@pytest.mark.parametrize("name,bi,mode", CASES, ids=[f"{n}-b{b}-{m}" for n, b, m in CASES])
def test_config_sampled_parity(name, bi, mode):
    G = require_gpu()
    w = W.WORKLOADS[name]
    pts, s, rp, col, eps, rph, sample, srp, scol, seps = search(name)
    basis, order, mask = w["bases"][bi]
    b = G.BASIS_SCALAR if basis == "scalar" else G.BASIS_DIVFREE
    prec = G.PREC_MIXED if mode == "mixed" else G.PREC_FP64
    flush(f"[{name}] stencils {basis} m={order} mask={mask} {mode}")
    wt, st, rep = G.gmls_stencils(ctx(), s, s, order, b, mask, w["p"], eps, rp, col, prec=prec, report=True)
    F, C, _ = G.gmls_stencil_shape(w["dim"], order, b, mask)
    gw = sampled_weights(wt, rph, sample, F, C)
    gst = host(st)[sample]
    del wt
    ow, ost, _, _ = oracle.stencils(pts, pts[sample], order, basis, mask, w["p"], seps, srp, scol)
    assert np.array_equal(gst == 1, ost == 1), "rank-deficient flags differ"
    zero = (F - 1,) if basis == "divfree" and mask & G.F_DIV else ()
    errs = row_errors(gw, ow, srp, F, C, zero_rows=zero)
    ok = ost != 1
    flush(f"  max rel err {errs[ok].max():.3e}  fallback {rep['n_fallback']} not-conv {rep['n_not_converged']} "
          f"rank-def {rep['n_rank_deficient']} stencil {rep['t_stencil_ms']:.1f} ms")
    assert errs[ok].max() <= TOL[mode]


def test_c2_polynomial_reproduction_every_target():
    """C2 at full size: Laplacian, gradient and value stencils reproduce 8
    random degree-4 polynomials at every target (Section 2.1: exactness on
    the polynomial space of the order)."""
    G = require_gpu()
    name = "c2_2d_m4"
    w = W.WORKLOADS[name]
    pts, s, rp, col, eps, rph, sample, srp, scol, seps = search(name)
    basis, order, mask = w["bases"][0]
    F, C, _ = G.gmls_stencil_shape(2, order, G.BASIS_SCALAR, mask)
    wt, st, _ = G.gmls_stencils(ctx(), s, s, order, G.BASIS_SCALAR, mask, w["p"], eps, rp, col,
                                prec=G.PREC_FP64)
    assert (host(st) == 0).all()
    absw = wt.abs()
    g = W.rng(w["poly_seed"])
    worst = 0.0
    for _ in range(8):
        poly = PT.random_poly(2, 4, g)
        u = PT.evaluate(poly, pts)
        exact = np.stack([PT.evaluate(poly, pts),
                          PT.evaluate(PT.deriv(poly, 0), pts), PT.evaluate(PT.deriv(poly, 1), pts),
                          PT.evaluate(PT.laplacian(poly, 2), pts)], axis=1)
        out = host(G.gmls_apply(ctx(), rp, col, wt, F, C, dev(u)))
        # rounding scale of each stencil sum: sum_j |alpha_j u_j|
        scale = host(G.gmls_apply(ctx(), rp, col, absw, F, C, dev(np.abs(u))))
        rel = np.abs(out - exact) / np.maximum(scale, 1e-300)
        worst = max(worst, float(rel.max()))
    flush(f"  C2 reproduction: worst relative residual {worst:.3e} over {len(pts)} targets x {F} rows")
    assert worst <= 1e-10
