"""The allocation-free SpMV (gmls_spmv_noalloc) against gmls_spmv through the
C ABI: the same kernels and summation order, so y must be bit for bit the
same, on two calls in a row (the second on a smaller matrix, with the
scratch holding the first call's long-row list), on a matrix with short rows
and rows longer than the 8192 entries a wavefront takes (the long-row list
lives in the scratch).  Also checked against a float64 product on the host,
and the host-side size limit."""
import numpy as np
import pytest
import torch

from tests.gpu_helpers import dev, flush, host, require_gpu

pytestmark = pytest.mark.gpu


def csr(n_rows, n_cols, long_rows, seed):
    g = np.random.default_rng(seed)
    lens = g.integers(0, 300, size=n_rows)
    lens[long_rows] = g.integers(8193, 30000, size=len(long_rows))
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    col = g.integers(0, n_cols, size=int(rp[-1])).astype(np.int32)
    val = g.standard_normal(int(rp[-1]))
    x = g.standard_normal(n_cols)
    return rp, col, val, x


def host_product(rp, col, val, x):
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    y = np.zeros(len(rp) - 1)
    np.add.at(y, rows, val * x[col])
    scale = np.zeros(len(rp) - 1)
    np.add.at(scale, rows, np.abs(val * x[col]))
    return y, scale


def test_noalloc_spmv_equals_spmv():
    G = require_gpu()
    c = G.Context(0)
    cases = [(100_000, 50_000, [3, 777, 60_000, 99_999], 1), (40_000, 9_000, [5, 39_998], 2)]
    for n_rows, n_cols, long_rows, seed in cases:  # the second call is smaller
        rp, col, val, x = csr(n_rows, n_cols, long_rows, seed)
        flush(f"noalloc spmv rows={n_rows} nnz={rp[-1]} long rows={len(long_rows)}")
        d = [dev(a) for a in (rp, col, val, x)]
        y_ref = host(G.gmls_spmv(c, *d))
        y_out = torch.full((n_rows,), float("nan"), dtype=torch.float64, device="cuda")
        y_na = host(G.gmls_spmv_noalloc(c, *d, y_out))
        assert np.array_equal(y_na.view(np.uint64), y_ref.view(np.uint64))
        yh, scale = host_product(rp, col, val, x)
        assert np.all(np.abs(y_na - yh) <= 1e-13 * scale + 1e-300)
    # more rows than the scratch holds: refused on the host
    too_many = torch.zeros(G.NOALLOC_SPMV_MAX_ROWS + 2, dtype=torch.int64, device="cuda")
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(G.GmlsError) as e:
        G.gmls_spmv_noalloc(c, too_many, torch.zeros(1, dtype=torch.int32, device="cuda"), one, one,
                            torch.empty(G.NOALLOC_SPMV_MAX_ROWS + 1, dtype=torch.float64, device="cuda"))
    assert e.value.status == 1
    c.close()
