"""Autotuner of the per-bin kernel shapes (gmls_autotune).

Every compiled candidate of every tunable kernel gives stencils within the
oracle's gate: the pipeline's row shapes (lanes per target x rows per lane)
and the wavefront kernel's variants (occupancy, moments per LDS round) in
mixed precision, the FP64 QR kernel's shapes (rows per lane, with longer rows
factored in chunks, and persistent waves per CU) in FP64, for single bases
and for the shared kernels of gmls_stencils_multi.  The autotuner keeps one
candidate per (kernel, non-empty bin), later calls use it and still pass the
gate; the table survives a JSON round trip, and files that are not in the
format, or name a shape that is not compiled, are refused without changing
the table."""
import json

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import ctx, dev, flush, host, require_gpu, row_errors
from tests.test_gpu_stencils import CASES, FP64_TOL, MIXED_TOL, case_data, run_gpu

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
    assert sorted(res) == ["moments", "qr", "weights"]  # the pipeline (mixed) and the QR kernel (FP64)
    for kname in ("moments", "weights", "qr"):
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
    assert len(doc["entries"]) == 3 * len(bins)
    for e in doc["entries"]:
        assert (e["dim"], e["order"], e["basis"]) == (3, order, 0)
        shape = (e["rows_per_lane"], e["waves_per_simd"], e["waves_per_cu"]) if e["kernel"] == "qr" else \
            (e["lanes"], e["rows_per_lane"])
        assert shape == res[e["kernel"]][e["bin"]]["chosen"]
    c2 = G.Context(0)
    G.gmls_autotune_load(c2, str(path))
    path2 = tmp_path / "tune2.json"
    G.gmls_autotune_save(c2, str(path2))
    assert path2.read_text() == path.read_text()

    # refused files leave the table as it was
    bad = tmp_path / "bad.json"
    entry = [e for e in doc["entries"] if e["kernel"] == "moments"][0]
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


def test_autotune_arguments():
    G = require_gpu()
    pts, rp, col, eps, w, st, F, C = case_data("3d_m3_radius")
    _, _, _, order, mask, p = CASES["3d_m3_radius"]
    c = G.Context(0)
    s, de, drp, dcol = dev(pts), dev(eps), dev(rp), dev(col)
    with pytest.raises(G.GmlsError) as e:
        G.gmls_autotune(c, s, s, order, G.BASIS_SCALAR, mask, p, de, drp, dcol, reps=0)
    assert e.value.status == 1
    with pytest.raises(G.GmlsError) as e:  # not a basis
        G.gmls_autotune(c, s, s, order, 5, mask, p, de, drp, dcol)
    assert e.value.status == 1
    with pytest.raises(G.GmlsError) as e:  # staggered: gradient and Laplacian only
        G.gmls_autotune(c, s, s, 2, G.TUNE_STAGGERED, G.F_VALUE, p, de, drp, dcol)
    assert e.value.status == 1
    with pytest.raises(G.GmlsError) as e:  # shared: a mask beyond bits 0-7
        G.gmls_autotune(c, s, s, order, G.TUNE_SHARED, 1 << 9, p, de, drp, dcol)
    assert e.value.status == 1
    for opt in (G.OPT_WAVE_SHAPE, G.OPT_QR_SHAPE):
        for bad in (3, -2, 0.5):
            with pytest.raises(G.GmlsError):
                c.set_option(opt, bad)
    c.close()


# ---- the wavefront kernel's variants and the QR kernel's shapes ----

@pytest.mark.parametrize("cand", [0, 1, 2])
@pytest.mark.parametrize("name", ["3d_m4_k170", "3d_divfree_m4"])
def test_every_wave_variant_matches_oracle(name, cand):
    """Scalar order 4 and divergence-free order 4 in 3D run the wavefront
    kernel (the automatic mixed scheme): every variant within the gate."""
    G = require_gpu()
    c = ctx()
    c.set_option(G.OPT_WAVE_SHAPE, cand)
    try:
        gw, gst, rep = run_gpu(name, G.PREC_MIXED)
    finally:
        c.set_option(G.OPT_WAVE_SHAPE, -1)
    pts, rp, col, eps, w, st, F, C = case_data(name)
    assert np.array_equal(gst == 1, st == 1)
    errs = row_errors(gw, w, rp, F, C, zero_rows=zero_rows(name, F))
    flush(f"  wave variant {cand}: max rel err {errs.max():.3e}")
    assert errs.max() <= MIXED_TOL


@pytest.mark.parametrize("cand", [0, 1, 2])
@pytest.mark.parametrize("name", ["3d_m3_radius", "3d_divfree_m2", "2d_m4", "3d_m4_k170"])
def test_every_qr_shape_matches_oracle(name, cand):
    """Fewer rows per lane than the bin's row count: the rows are factored
    in chunks (tall-skinny QR); every shape within the FP64 gate."""
    G = require_gpu()
    c = ctx()
    c.set_option(G.OPT_QR_SHAPE, cand)
    try:
        gw, gst, rep = run_gpu(name, G.PREC_FP64)
    finally:
        c.set_option(G.OPT_QR_SHAPE, -1)
    pts, rp, col, eps, w, st, F, C = case_data(name)
    assert np.array_equal(gst, st)
    errs = row_errors(gw, w, rp, F, C, zero_rows=zero_rows(name, F))
    flush(f"  qr shape {cand}: max rel err {errs.max():.3e}")
    assert errs.max() <= FP64_TOL


_shared = {}


def shared_case():
    """A scalar and a divergence-free set of order 4 on 170-neighbour rows
    (the high-order configuration's shape, on 4000 points)."""
    if "c" not in _shared:
        pts = W.jittered_grid(4000, 3, 1006)
        rp, col, eps = oracle.knn(pts, pts, 170, 1.5)
        ms, mv = 2 | 4, 4 | 8
        ws, sts, Fs, Cs = oracle.stencils(pts, pts, 4, "scalar", ms, 6, eps, rp, col)
        wv, stv, Fv, Cv = oracle.stencils(pts, pts, 4, "divfree", mv, 6, eps, rp, col)
        _shared["c"] = (pts, rp, col, eps, ms, mv, (ws, sts, Fs, Cs), (wv, stv, Fv, Cv))
    return _shared["c"]


def check_shared(G, outs, fp64):
    pts, rp, col, eps, ms, mv, os_, ov = shared_case()
    for (w, st), (ow, ost, F, C), div in zip(outs, (os_, ov), (False, True)):
        w, st = host(w), host(st)
        if fp64:
            assert np.array_equal(st, ost)
        else:
            assert np.array_equal(st == 1, ost == 1)
        zero = (F - 1,) if div else ()
        errs = row_errors(w, ow, rp, F, C, zero_rows=zero)[ost != 1]
        flush(f"  {'divfree' if div else 'scalar'}: max rel err {errs.max():.3e}")
        assert errs.max() <= (FP64_TOL if fp64 else MIXED_TOL)


@pytest.mark.parametrize("kind,cand", [("wave", 0), ("wave", 1), ("wave", 2), ("qr", 0), ("qr", 1), ("qr", 2)])
def test_shared_kernels_every_shape(kind, cand):
    G = require_gpu()
    pts, rp, col, eps, ms, mv, _, _ = shared_case()
    c = ctx()
    s = dev(pts)
    opt = G.OPT_WAVE_SHAPE if kind == "wave" else G.OPT_QR_SHAPE
    c.set_option(opt, cand)
    try:
        flush(f"shared {kind} candidate {cand}")
        outs, _ = G.gmls_stencils_multi(c, s, s, 4, 6, dev(eps), dev(rp), dev(col),
                                        [(G.BASIS_SCALAR, ms), (G.BASIS_DIVFREE, mv)],
                                        prec=G.PREC_MIXED if kind == "wave" else G.PREC_FP64)
    finally:
        c.set_option(opt, -1)
    check_shared(G, outs, kind == "qr")


def test_autotune_shared_and_wave_json(tmp_path):
    """Tuning the shared kernels (wave and QR) and a single basis on the
    wavefront kernel; later calls use the table and pass the gate; the new
    kernels' entries survive a JSON round trip and bad ones are refused."""
    G = require_gpu()
    pts, rp, col, eps, ms, mv, _, _ = shared_case()
    c = G.Context(0)
    s, de, drp, dcol = dev(pts), dev(eps), dev(rp), dev(col)
    flush("autotune shared order 4")
    res = G.gmls_autotune(c, s, s, 4, G.TUNE_SHARED, ms | (mv << 4), 6, de, drp, dcol, reps=2)
    flush(f"  {res}")
    assert sorted(res) == ["qr", "wave"]
    bins = sorted({int((m + 63) // 64) for m in np.diff(rp)})
    for kname in ("wave", "qr"):
        assert sorted(res[kname]) == bins
        for b, e in res[kname].items():
            assert min(e["ms"].values()) == e["ms"][e["chosen"]] > 0
    sets = [(G.BASIS_SCALAR, ms), (G.BASIS_DIVFREE, mv)]
    for prec in (G.PREC_MIXED, G.PREC_FP64):
        outs, _ = G.gmls_stencils_multi(c, s, s, 4, 6, de, drp, dcol, sets, prec=prec)
        check_shared(G, outs, prec == G.PREC_FP64)
    flush("autotune scalar order 4 (wavefront kernel)")
    res1 = G.gmls_autotune(c, s, s, 4, G.BASIS_SCALAR, ms, 6, de, drp, dcol, reps=1)
    assert sorted(res1) == ["qr", "wave"]

    path = tmp_path / "tune.json"
    G.gmls_autotune_save(c, str(path))
    doc = json.loads(path.read_text())
    kinds = {(e["basis"], e["kernel"]) for e in doc["entries"]}
    assert kinds == {(3, "wave"), (3, "qr"), (0, "wave"), (0, "qr")}
    for e in doc["entries"]:
        r = res if e["basis"] == 3 else res1
        shape = (e["waves_per_simd"], e["lds_round"]) if e["kernel"] == "wave" else \
            (e["rows_per_lane"], e["waves_per_simd"], e["waves_per_cu"])
        assert shape == r[e["kernel"]][e["bin"]]["chosen"]
    c2 = G.Context(0)
    G.gmls_autotune_load(c2, str(path))
    path2 = tmp_path / "tune2.json"
    G.gmls_autotune_save(c2, str(path2))
    assert path2.read_text() == path.read_text()
    wave = [e for e in doc["entries"] if e["kernel"] == "wave"][0]
    qr = [e for e in doc["entries"] if e["kernel"] == "qr"][0]
    bad = tmp_path / "bad.json"
    for entry in (dict(wave, lds_round=7), dict(qr, waves_per_cu=5), dict(qr, kernel="solve"),
                  dict(wave, bin=5)):
        bad.write_text(json.dumps({"libgmls_autotune": 1, "entries": [entry]}).replace('},', '},\n'))
        with pytest.raises(G.GmlsError):
            G.gmls_autotune_load(c2, str(bad))
    G.gmls_autotune_save(c2, str(path2))
    assert path2.read_text() == path.read_text()
    c.close()
    c2.close()
