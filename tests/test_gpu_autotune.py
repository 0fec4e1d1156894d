"""Autotuner of the mixed pipeline's row shapes (gmls_autotune).

Every compiled row shape (lanes per target x rows per lane, three per
row-count bin) gives stencils within the mixed gate of the oracle; the
autotuner keeps one compiled shape per (kernel, non-empty bin), later calls
use it and still pass the gate; the table survives a JSON round trip, and
files that are not in the format, or name a shape that is not compiled, are
refused without changing the table."""
import json

import numpy as np
import pytest

from tests.gpu_helpers import ctx, dev, flush, host, require_gpu, row_errors
from tests.test_gpu_stencils import CASES, MIXED_TOL, case_data, run_gpu

pytestmark = pytest.mark.gpu


def zero_rows(name, F):
    return (F - 1,) if CASES[name][2] == "divfree" and CASES[name][4] & 8 else ()


@pytest.mark.parametrize("cand", [0, 1, 2])
@pytest.mark.parametrize("name", ["3d_m3_radius", "3d_divfree_m2", "2d_m4"])
def test_every_row_shape_matches_oracle(name, cand):
    G = require_gpu()
    c = ctx()
    c.set_option(G.OPT_PIPE_SHAPE, cand)
    try:
        gw, gst, rep = run_gpu(name, G.PREC_MIXED)  # the automatic scheme is the pipeline here
    finally:
        c.set_option(G.OPT_PIPE_SHAPE, -1)
    pts, rp, col, eps, w, st, F, C = case_data(name)
    assert np.array_equal(gst == 1, st == 1)
    errs = row_errors(gw, w, rp, F, C, zero_rows=zero_rows(name, F))
    flush(f"  shape {cand}: max rel err {errs.max():.3e}")
    assert errs.max() <= MIXED_TOL


def test_pipe_shape_option_is_validated():
    G = require_gpu()
    for bad in (3, -2, 0.5):
        with pytest.raises(G.GmlsError):
            ctx().set_option(G.OPT_PIPE_SHAPE, bad)


def test_autotune_then_stencils_and_json_round_trip(tmp_path):
    G = require_gpu()
    name = "3d_m3_radius"
    pts, rp, col, eps, w, st, F, C = case_data(name)
    _, _, _, order, mask, p = CASES[name]
    n = np.diff(rp)
    bins = sorted({int((m + 63) // 64) for m in n[n >= 20]})  # scalar order 3: rank deficient below 20
    c = G.Context(0)
    s, de, drp, dcol = dev(pts), dev(eps), dev(rp), dev(col)
    flush(f"autotune {name} bins {bins}")
    res = G.gmls_autotune(c, s, s, order, G.BASIS_SCALAR, mask, p, de, drp, dcol, reps=2)
    flush(f"  {res}")
    for kname in ("moments", "weights"):
        assert sorted(res[kname]) == bins
        for b, e in res[kname].items():
            assert e["chosen"] in e["ms"] and len(e["ms"]) == 3
            assert all(v > 0 for v in e["ms"].values())
            assert min(e["ms"].values()) == e["ms"][e["chosen"]]
    gw, gst, _ = G.gmls_stencils(c, s, s, order, G.BASIS_SCALAR, mask, p, de, drp, dcol, prec=G.PREC_MIXED)
    errs = row_errors(host(gw), w, rp, F, C)
    assert errs.max() <= MIXED_TOL

    path = tmp_path / "tune.json"
    G.gmls_autotune_save(c, str(path))
    doc = json.loads(path.read_text())
    assert doc["libgmls_autotune"] == 1
    assert len(doc["entries"]) == 2 * len(bins)
    for e in doc["entries"]:
        assert (e["dim"], e["order"], e["basis"]) == (3, order, 0)
        assert (e["lanes"], e["rows_per_lane"]) == res[e["kernel"]][e["bin"]]["chosen"]
    c2 = G.Context(0)
    G.gmls_autotune_load(c2, str(path))
    path2 = tmp_path / "tune2.json"
    G.gmls_autotune_save(c2, str(path2))
    assert path2.read_text() == path.read_text()

    # refused files leave the table as it was
    bad = tmp_path / "bad.json"
    entry = doc["entries"][0]
    bad.write_text(json.dumps({"libgmls_autotune": 1, "entries": [dict(entry, lanes=7, rows_per_lane=9)]}))
    with pytest.raises(G.GmlsError):
        G.gmls_autotune_load(c2, str(bad))
    bad.write_text('{"something": 1}')
    with pytest.raises(G.GmlsError):
        G.gmls_autotune_load(c2, str(bad))
    with pytest.raises(G.GmlsError):
        G.gmls_autotune_load(c2, str(tmp_path / "missing.json"))
    G.gmls_autotune_save(c2, str(path2))
    assert path2.read_text() == path.read_text()
    c.close()
    c2.close()


def test_autotune_refuses_what_it_cannot_tune():
    G = require_gpu()
    pts, rp, col, eps, w, st, F, C = case_data("3d_m4_k170")
    _, _, _, order, mask, p = CASES["3d_m4_k170"]
    c = G.Context(0)
    s, de, drp, dcol = dev(pts), dev(eps), dev(rp), dev(col)
    with pytest.raises(G.GmlsError) as e:  # scalar order 4 in 3D runs the wavefront kernel, not the pipeline
        G.gmls_autotune(c, s, s, order, G.BASIS_SCALAR, mask, p, de, drp, dcol)
    assert e.value.status == G.GMLS_ERR_UNSUPPORTED
    with pytest.raises(G.GmlsError) as e:
        G.gmls_autotune(c, s, s, order, G.BASIS_SCALAR, mask, p, de, drp, dcol, reps=0)
    assert e.value.status == 1
    c.close()
