"""Benchmark: GMLS stencil generation on one MI355X.

Workload (default): 2,000,000 points in [0,1]^3 with density rising 4x along
x, fixed-radius neighbour search (radius giving 40 neighbours on average at
x = 0, 160 at x = 1, floored to the 30 nearest), scalar Taylor basis of
order 3 (20 functions), kernel (1 - r/eps)^4, Laplacian functional.

One step = the whole hot path over the batch: cell-list build and neighbour
search (gmls_neighbors) followed by stencil generation (gmls_stencils),
captured once into a HIP graph (capture-safe mode) and replayed; eager steps
with per-phase HIP events give the phase times and the roofline figures.
Inputs are resident in HBM before timing starts.  The same process checks
sampled outputs against the FP64 CPU oracle (parity gate) and times the
oracle on a bounded sample of the same workload on the host cores.

Prints ONE JSON line (see the end of main()).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

# Algorithmic work per stencil, the conventional count (scalar basis with Q
# functions, F functional rows, N neighbours): symmetric Gram N*Q*(Q+1),
# Cholesky Q^3/3, two triangular solves per row 2*F*Q^2, weights 2*N*Q*F.
# Bytes: the CSR row (4N), the weights (8*F*C*N) and per-target scalars
# (row_ptr, eps, coordinates: 64).  The moment form of the Gram does N*2*NM
# flops (NM = monomials of degree <= 2m) instead of N*Q*(Q+1); the
# conventional count is the one credited.
def _binom(n, k):
    from math import comb
    return comb(n, k)


def alg_flops_workload(nnz, n_tgt, dim, bases):
    """Conventional count over the bases of a configuration: the scalar Gram
    N*Qs*(Qs+1) once per target (shared by bases on one neighbour list), then
    per basis Q^3/3 + 2FQ^2 and 2*R*Qs*F for the weights (R = N scalar, d*N
    vector); the vector basis adds the congruence 4*Qd^2 and 2*F*Qd*d*Qs.
    The staggered basis counts its Qs = Q columns (no constant monomial), the
    Neumann-constrained basis the scalar ones."""
    qs_max = max(b["Qs"] for b in bases)
    total = nnz * qs_max * (qs_max + 1)
    for b in bases:
        qs = b["Qs"]
        Q, F = b["Q"], b["F"]
        total += n_tgt * (Q ** 3 / 3.0 + 2 * F * Q * Q)
        if b["name"] != "divfree":
            total += 2 * nnz * qs * F
        else:
            total += 2 * dim * nnz * qs * F + n_tgt * (4 * Q * Q + 2 * F * Q * dim * qs)
    return total


def alg_bytes_workload(nnz, n_tgt, dim, bases):
    return 4 * nnz + 64 * n_tgt + sum(8 * b["F"] * b["C"] * nnz for b in bases)


DEFAULT_WORKLOAD = "c4_3d_m3_uneven"
DESCRIBE = {
    "c1_2d_m2": "1000 jittered-grid points in 2D, kNN 12, scalar order 2, gradient + Laplacian",
    "c2_2d_m4": "100k jittered-grid points in 2D, kNN 40, scalar order 4, value + gradient + Laplacian",
    "c3_3d_divfree_m2": "1M jittered-grid points in 3D, kNN 60, div-free order 2 vector Laplacian + "
                        "scalar order 2 gradient",
    "c4_3d_m3_uneven": "2M points, density 1+3x, radius search (k_min 30), scalar order 3, Laplacian",
    "c5_3d_m4": "500k jittered-grid points in 3D, kNN 170, p=6, scalar order 4 gradient + Laplacian and "
                "div-free order 4 vector Laplacian + divergence",
    "s4_3d_staggered_m2": "the C4 cloud and radius search, staggered gradient + Laplacian of vector order 2",
    "n3_3d_neumann_m3": "60k points on the faces of the unit cube with outward normals, kNN 80 into 1M "
                        "jittered-grid points, Neumann-constrained scalar order 3 Laplacian (FP64)",
}


PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp64_TFs": 78.6,
    "fp32_TFs": 157.3,
}

# Sources of the stencil-phase kernels; a traffic figure measured with
# hardware counters is reported only while these are unchanged.
# device code of the stencil-phase kernels (and their launch shapes)
STENCIL_SOURCES = ["stencil_pipe.hpp", "stencil_mixed64.hpp", "stencil_mixed.hpp", "stencil_fp64.hpp",
                   "qr_kernel.hpp", "stencil_bins.hip", "basis.hpp", "common.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stencils_c4.txt")


def stencil_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in STENCIL_SOURCES:
        with open(os.path.join(ROOT, "paper_2104_14447_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec_name):
    """HBM bytes per step of the stencil phase from the committed counter
    summary, if it was taken on the current kernel sources and precision."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != stencil_source_hash() or kv.get("precision") != prec_name:
        return None
    try:
        return float(kv["hbm_bytes_per_step"])
    except (KeyError, ValueError):
        return None


def copy_probe():
    """A plain device-to-device copy of known size, for scaling HBM counters."""
    import torch
    n = 1 << 27  # 1 GiB of float64
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 8 * n, "copy_probe_bytes_written": 8 * n, "launches": 3}))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", choices=["mixed", "fp64", "auto"], default="auto")
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=list(W.WORKLOADS),
                    help="configuration (default: the 2M-point uneven radius workload)")
    ap.add_argument("--n", type=int, default=0, help="points (default: the configuration's size)")
    ap.add_argument("--sample", type=int, default=256, help="targets checked against the oracle")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target duration of the oracle timing leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scheme", type=int, default=0,
                    help="mixed scheme: 0 auto, 1 fused/rows residual, 2 fused/moment Gram, 3 pipeline, 4 wavefront per target")
    ap.add_argument("--chunk", type=int, default=0, help="pipeline chunk (targets; 0 = whole batch)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="mixed pipeline: keep the default row shapes instead of autotuning them first")
    ap.add_argument("--tune-cache", default="",
                    help="autotune table (JSON): loaded if the file exists, else written after tuning")
    ap.add_argument("--copy-probe", action="store_true", help="run a 1 GiB device copy (counter scaling) and exit")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager calls instead of HIP graph replays of search + stencils")
    ap.add_argument("--stokes", type=int, default=0, metavar="N_SIDE",
                    help="time the global Stokes operator build on a [-1,1]^3 cloud of N_SIDE^3 interior "
                         "particles instead")
    return ap.parse_args()


def stokes_main(args):
    """The global Stokes operator of the paper's scheme on [-1,1]^3: search,
    the four stencil families (FP64), assembly and operator application,
    each timed with HIP events; the manufactured quadratic solution's
    residual is the correctness gate."""
    import torch

    import paper_2104_14447_amd as G
    from tests.manufactured import exact_system  # closed forms of the paper's manufactured solution

    n_side, k = args.stokes, 80
    # mixed precision for the families the mixed kernels cover (vector
    # Laplacian, gradient, staggered Laplacian); the constrained boundary
    # stencils are FP64 in either case
    prec = G.PREC_FP64 if args.prec == "fp64" else G.PREC_MIXED
    pts, bnd, nrm = W.stokes_cloud(n_side, 3, 2024)
    n = len(pts)
    c = G.Context(0)
    x, bt, nt = (torch.from_numpy(a).cuda() for a in (pts, bnd, nrm))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    times = {"search": [], "stencils": [], "assembly": [], "spmv": []}
    for it in range(args.warmup + args.steps):
        ev[0].record()
        rp, col, eps = G.gmls_neighbors(c, x, x, G.SEARCH_KNN, k=k, eps_mult=1.5)
        ev[1].record()
        vlap, _, _ = G.gmls_stencils(c, x, x, 2, G.BASIS_DIVFREE, G.F_LAPLACIAN, 4, eps, rp, col, prec=prec)
        grad, _, _ = G.gmls_stencils(c, x, x, 3, G.BASIS_SCALAR, G.F_GRAD, 4, eps, rp, col, prec=prec)
        plap, plap_t, _, _ = G.gmls_stencils_staggered(c, x, x, 2, G.F_LAPLACIAN, 4, eps, rp, col, prec=prec)
        nlap, nlap_h, _, _ = G.gmls_stencils_constrained(c, x, x, 3, G.F_LAPLACIAN, 4, eps, rp, col, nt)
        ev[2].record()
        arp, acol, aval = G.gmls_assemble_stokes(c, rp, col, bt, nt, vlap, grad, plap, plap_t.reshape(-1),
                                                 nlap, nlap_h.reshape(-1))
        ev[3].record()
        if it == 0:
            xs, rhs = exact_system(pts, bnd, nrm, nlap_h.reshape(-1).cpu().numpy(), 1.0)
            xd = torch.from_numpy(xs).cuda()
            y = torch.empty_like(xd)
        for _ in range(10):
            G.gmls_spmv(c, arp, acol, aval, xd, y)
        ev[4].record()
        torch.cuda.synchronize()
        if it >= args.warmup:
            for key, a_, b_ in (("search", 0, 1), ("stencils", 1, 2), ("assembly", 2, 3)):
                times[key].append(ev[a_].elapsed_time(ev[b_]))
            times["spmv"].append(ev[3].elapsed_time(ev[4]) / 10)
        print(f"# stokes step {it} done", file=sys.stderr, flush=True)
    yh = y.cpu().numpy()
    # rounding scale of each row: |A| |x| + |rhs|, the product on the GPU
    scale = G.gmls_spmv(c, arp, acol, aval.abs(), xd.abs()).cpu().numpy() + np.abs(rhs)
    resid = float((np.abs(yh - rhs) / scale).max())
    t = {k_: float(np.median(v)) for k_, v in times.items()}
    total = t["search"] + t["stencils"] + t["assembly"]
    nnz = int(acol.numel())
    spmv_bytes = nnz * 12 + (len(xs) + 1) * 8 + 2 * len(xs) * 8
    pname = "fp64" if prec == G.PREC_FP64 else "mixed"
    line = {"metric": f"Stokes operator build (search + 4 stencil families ({pname}) + assembly), particles/s",
            "value": round(n / (total * 1e-3), 1), "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(total, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if pname == "fp64" else "f32+f64", "data": "synthetic",
            "config": {"precision": pname, "workload": f"[-1,1]^3 cloud: {n_side}^3 jittered interior + {n - n_side ** 3} boundary "
                                   f"particles, kNN {k}; div-free m2 vector Laplacian, scalar m3 gradient, "
                                   f"staggered m2 Laplacian, Neumann m3 Laplacian",
                       "n_particles": n, "rows": len(xs), "nnz": nnz, "phase_ms": t,
                       "manufactured_residual": resid, "gate": resid <= (1e-9 if pname == "fp64" else 1e-7),
                       "spmv_GBs": round(spmv_bytes / (t["spmv"] * 1e-3) / 1e9, 1)}}
    print(json.dumps(line))


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.stokes:
        stokes_main(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not a launched path)"}))
        sys.exit(2)
    import torch

    import paper_2104_14447_amd as G

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    G.load_library()
    dev = torch.device("cuda:0")
    ctx = G.Context(0)
    ctx.set_option(G.OPT_MIXED_SCHEME, args.scheme)
    ctx.set_option(G.OPT_PIPE_CHUNK, args.chunk)

    name = args.workload
    wl = W.WORKLOADS[name]
    dim, p = wl["dim"], wl["p"]
    n = args.n if args.n else wl["n"]
    knn = wl["search"][0] == "knn"
    if knn:
        k, mult = wl["search"][1], wl["search"][2]
        spec = dict(mode=G.SEARCH_KNN, k=k, eps_mult=mult)
    else:
        r0 = wl["search"][1] if n == wl["n"] else W.radius_for_mean_count(n)
        k_min = wl["search"][2]
        spec = dict(mode=G.SEARCH_RADIUS, radius=r0, k_min=k_min)
    t0 = time.time()
    pts = W.make_points(name, n=n)
    print(f"# generated {n} points in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    x = torch.from_numpy(pts).to(dev)
    # targets: the sources themselves, or points on the domain boundary with
    # outward normals (Neumann-constrained stencils)
    nrm = None
    if wl.get("targets"):
        _, n_b, seed_b = wl["targets"]
        tpts, nrm_h = W.boundary_points(n_b, dim, seed_b)
        xt = torch.from_numpy(tpts).to(dev)
        nrm = torch.from_numpy(nrm_h).to(dev)
    else:
        tpts, nrm_h, xt = pts, None, x
    n_t = len(tpts)
    bases = []
    for basis, order, mask in wl["bases"]:
        b = G.BASIS_DIVFREE if basis == "divfree" else G.BASIS_SCALAR
        F, C, Q = G.gmls_stencil_shape(dim, order, b, mask)
        if basis == "staggered":  # scalar monomials of degree 1..order+1
            F, C, Q = (dim if mask & G.F_GRAD else 0) + (1 if mask & G.F_LAPLACIAN else 0), 1, \
                _binom(order + 1 + dim, dim) - 1
        Qs = Q if basis != "divfree" else _binom(order + dim, dim)
        bases.append(dict(name=basis, b=b, order=order, mask=mask, F=F, C=C, Q=Q, Qs=Qs))

    def stencils(c, bs, eps_, rp_, col_, weights=None, status=None, aux=None, report=False):
        """One basis of the configuration through its entry point; `aux`
        receives the h-weights (constrained) or target weights (staggered)."""
        if bs["name"] == "staggered":
            return G.gmls_stencils_staggered(c, x, xt, bs["order"], bs["mask"], p, eps_, rp_, col_, prec=prec,
                                             weights=weights, t_weights=aux, status=status, report=report)
        if bs["name"] == "neumann":
            return G.gmls_stencils_constrained(c, x, xt, bs["order"], bs["mask"], p, eps_, rp_, col_, nrm,
                                               prec=prec, weights=weights, h_weights=aux, status=status,
                                               report=report)
        w_, st_, r_ = G.gmls_stencils(c, x, xt, bs["order"], bs["b"], bs["mask"], p, eps_, rp_, col_, prec=prec,
                                      weights=weights, status=status, report=report)
        return w_, None, st_, r_

    precs = {"mixed": G.PREC_MIXED, "fp64": G.PREC_FP64}
    if args.prec == "auto":
        prec_name = "mixed" if "mixed" in wl["modes"] else "fp64"
    else:
        prec_name = args.prec
    prec = precs[prec_name]

    # buffers reused across steps (no allocation inside the timed region)
    rp, col, eps = G.gmls_neighbors(ctx, x, xt, **spec)
    nnz = col.numel()
    col_buf = torch.empty(int(nnz * 1.05) + 1024, dtype=torch.int32, device=dev)
    for bs in bases:
        bs["w"] = torch.empty(bs["F"] * bs["C"] * nnz, dtype=torch.float64, device=dev)
        bs["st"] = torch.empty(n_t, dtype=torch.uint8, device=dev)
        bs["aux"] = torch.empty((n_t, bs["F"]), dtype=torch.float64, device=dev)

    # ---- autotune the mixed pipeline's row shapes (before any timing) ----
    tune_summary = "off"
    tune_path = None
    if prec == G.PREC_MIXED and not args.no_autotune:
        if args.tune_cache and os.path.exists(args.tune_cache):
            G.gmls_autotune_load(ctx, args.tune_cache)
            tune_summary = {"loaded": args.tune_cache}
            tune_path = args.tune_cache
        else:
            tune_summary = {}
            t0 = time.time()
            for bs in bases:
                if bs["name"] == "neumann":
                    continue
                # staggered stencils run the scalar pipeline of order + 1
                order_t, b_t = (bs["order"] + 1, G.BASIS_SCALAR) if bs["name"] == "staggered" \
                    else (bs["order"], bs["b"])
                try:
                    res = G.gmls_autotune(ctx, x, xt, order_t, b_t, bs["mask"], p, eps, rp, col, reps=3)
                except G.GmlsError as e:
                    if e.status != G.GMLS_ERR_UNSUPPORTED:  # not the pipeline: nothing to tune
                        raise
                    continue
                tune_summary[bs["name"]] = {k: {b: "%dx%d" % v["chosen"] for b, v in d.items()}
                                            for k, d in res.items()}
            print(f"# autotune: {tune_summary} ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
            if tune_summary:
                if args.tune_cache:
                    tune_path = args.tune_cache
                else:
                    fd, tune_path = tempfile.mkstemp(suffix=".json")
                    os.close(fd)
                G.gmls_autotune_save(ctx, tune_path)
            else:
                tune_summary = "no pipeline in this configuration"

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # a scalar and a divergence-free basis of one order on the same neighbour
    # lists go through one gmls_stencils_multi call (the library shares their
    # Gram where the scheme allows)
    shared = len(bases) == 2 and sorted(b["name"] for b in bases) == ["divfree", "scalar"] and \
        bases[0]["order"] == bases[1]["order"]

    def all_stencils(c, eps_, rp_, col_, wkey, stkey, auxkey, report=False):
        if shared:
            outs = [(bs[wkey], bs[stkey]) for bs in bases]
            return [G.gmls_stencils_multi(c, x, xt, bases[0]["order"], p, eps_, rp_, col_,
                                          [(bs["b"], bs["mask"]) for bs in bases], prec=prec, outputs=outs,
                                          report=report)[1]]
        return [stencils(c, bs, eps_, rp_, col_, weights=bs[wkey], status=bs[stkey], aux=bs[auxkey],
                         report=report)[3] for bs in bases]

    def step(report=False):
        ev0.record()
        rp_, col_, eps_ = G.gmls_neighbors(ctx, x, xt, col=col_buf, **spec)
        ev1.record()
        reps = all_stencils(ctx, eps_, rp_, col_, "w", "st", "aux", report=report)
        return rp_, col_, eps_, reps

    # ---- eager steps: per-phase GPU times (HIP events on the library's stream) ----
    for i in range(args.warmup):
        step()
        print(f"# warmup step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stencil_ms, search_ms = [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        out = step(report=True)
        stencil_ms.append(sum(r["t_stencil_ms"] + r["t_fallback_ms"] for r in out[3]))
        search_ms.append(ev0.elapsed_time(ev1))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_eager = 1e3 * t_total / args.steps
    rp_t, col_t, eps_t, reps = out
    print(f"# eager: {args.steps} steps: {ms_eager:.3f} ms/step; stencil kernels "
          f"{np.mean(stencil_ms):.3f} ms; search {np.mean(search_ms):.3f} ms; reports {reps}",
          file=sys.stderr, flush=True)
    ms_per_step = ms_eager

    # ---- the timed unit: one HIP graph replay of search + stencils ----
    graph = not args.no_graph
    if graph:
        gs = torch.cuda.Stream()
        gctx = G.Context(0, stream=gs)
        gctx.set_option(G.OPT_MIXED_SCHEME, args.scheme)
        if tune_path:
            G.gmls_autotune_load(gctx, tune_path)  # the same row shapes as the eager steps
        with torch.cuda.stream(gs):
            # one normal call of each kind sizes the context's workspace
            rpw, colw, epsw = G.gmls_neighbors(gctx, x, xt, **spec)
            for bs in bases:
                stencils(gctx, bs, epsw, rpw, colw)
            if shared:
                G.gmls_stencils_multi(gctx, x, xt, bases[0]["order"], p, epsw, rpw, colw,
                                      [(bs["b"], bs["mask"]) for bs in bases], prec=prec)
            gcol = torch.empty(nnz + 1024, dtype=torch.int32, device=dev)
            for bs in bases:
                bs["gw"] = torch.empty(bs["F"] * bs["C"] * nnz, dtype=torch.float64, device=dev)
                bs["gst"] = torch.empty(n_t, dtype=torch.uint8, device=dev)
                bs["gaux"] = torch.empty((n_t, bs["F"]), dtype=torch.float64, device=dev)
            gctx.set_option(G.OPT_CAPTURE_SAFE, 1)
            gout = {}

            def gstep():
                rp_, col_, eps_ = G.gmls_neighbors(gctx, x, xt, col=gcol, **spec)
                all_stencils(gctx, eps_, rp_, col_[:nnz], "gw", "gst", "gaux")
                gout["rp"], gout["eps"] = rp_, eps_

            gstep()  # capture-safe eager run (no allocation happens in the capture)
            hg = torch.cuda.CUDAGraph()
            with torch.cuda.graph(hg, stream=gs):
                gstep()
        for i in range(args.warmup):
            hg.replay()
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for i in range(args.steps):
            hg.replay()
        torch.cuda.synchronize()
        ms_per_step = 1e3 * (time.perf_counter() - t_start) / args.steps
        gctx.check()
        print(f"# graph: {args.steps} replays: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)
        # the parity gate below checks the replayed outputs
        rp_t, col_t, eps_t = gout["rp"], gcol[:nnz], gout["eps"]
        for bs in bases:
            bs["w"], bs["st"], bs["aux"] = bs["gw"], bs["gst"], bs["gaux"]

    if tune_path and not args.tune_cache:
        os.remove(tune_path)

    # ---- the CPU-baseline leg: the only part of this file that uses the
    # oracle.  It checks sampled outputs of the timed run against it (the
    # parity gate) and, unless --no-cpu-baseline, times it on the host ----
    def cpu_baseline_leg():
        import oracle

        rph = rp_t.cpu().numpy()
        epsh = eps_t.cpu().numpy()
        g = W.rng(424242)
        sample = np.sort(g.choice(n_t, size=min(args.sample, n_t), replace=False))
        idx = torch.from_numpy(np.concatenate([np.arange(rph[t], rph[t + 1]) for t in sample])).cuda()
        scol = col_t[idx].cpu().numpy()
        srp = np.zeros(len(sample) + 1, dtype=np.int64)
        srp[1:] = np.cumsum(np.diff(rph)[sample])
        if knn:
            orp, ocol, oeps = oracle.knn(pts, tpts[sample], k, mult)
        else:
            orp, ocol, oeps = oracle.radius(pts, tpts[sample], r0, k_min)
        if knn:
            same_rows = np.array_equal(scol, ocol)
        else:  # radius rows are sets: cell order on the GPU, index order in the oracle
            rows = np.repeat(np.arange(len(srp) - 1), np.diff(srp))
            same_rows = np.array_equal(srp, orp) and np.array_equal(scol[np.lexsort((scol, rows))], ocol)
        search_ok = np.array_equal(srp, orp) and same_rows and np.array_equal(epsh[sample], oeps)
        seps = epsh[sample]
        max_err = 0.0
        status_ok = True
        for bs in bases:
            F, C = bs["F"], bs["C"]
            widx = torch.from_numpy(np.concatenate([np.arange(F * C * rph[t], F * C * rph[t + 1])
                                                    for t in sample])).cuda()
            wh = bs["w"][widx].cpu().numpy()
            sth = bs["st"].cpu().numpy()[sample]
            if bs["name"] == "staggered":
                from oracle import staggered as OS
                ow, oaux, _ = OS.stencils_staggered(pts, tpts[sample], bs["order"], bs["mask"], p, seps, srp, scol)
                ost = np.zeros(len(sample), dtype=np.uint8)
            elif bs["name"] == "neumann":
                from oracle import constrained as OC
                ow, oaux, _ = OC.stencils_constrained(pts, tpts[sample], bs["order"], bs["mask"], p, seps, srp, scol,
                                                      nrm_h[sample])
                ost = np.zeros(len(sample), dtype=np.uint8)
            else:
                ow, ost, _, _ = oracle.stencils(pts, tpts[sample], bs["order"], bs["name"], bs["mask"], p, seps, srp,
                                                scol)
                oaux = None
            status_ok = status_ok and np.array_equal(sth == 1, ost == 1)
            if oaux is not None:  # target weights / h-weights, relative to the row norms
                gaux = bs["aux"].cpu().numpy()[sample]
                for q in range(len(sample)):
                    b_ = ow[F * srp[q]:F * srp[q + 1]].reshape(F, -1)
                    den = np.hypot(np.linalg.norm(b_, axis=1), oaux[q])
                    max_err = max(max_err, float((np.abs(gaux[q] - oaux[q]) / np.where(den > 0, den, 1.0)).max()))
            zero = F - 1 if bs["name"] == "divfree" and bs["mask"] & G.F_DIV else -1
            for q in range(len(sample)):
                if ost[q] == 1:
                    continue
                a = wh[F * C * srp[q]:F * C * srp[q + 1]].reshape(F, -1)
                b_ = ow[F * C * srp[q]:F * C * srp[q + 1]].reshape(F, -1)
                den = np.linalg.norm(b_, axis=1)
                if zero >= 0:
                    den[zero] = den[0]
                max_err = max(max_err, float((np.linalg.norm(a - b_, axis=1) / den).max()))
        tol = 1e-8 if prec_name == "mixed" else 1e-10
        gate = bool(search_ok and status_ok and max_err <= tol)
        print(f"# parity: search {'ok' if search_ok else 'MISMATCH'}; max rel err {max_err:.3e} (gate {tol:g})",
              file=sys.stderr, flush=True)


        cpu = None
        if not args.no_cpu_baseline and all(bs["name"] in ("scalar", "divfree") for bs in bases) and n_t == n:
            threads = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16), 16)

            def oracle_run(m):
                sub = np.arange(m)
                if knn:
                    a_rp, a_col, a_eps = oracle.knn(pts, pts[sub], k, mult, use_grid=True, nthreads=threads)
                else:
                    a_rp, a_col, a_eps = oracle.radius(pts, pts[sub], r0, k_min, use_grid=True, nthreads=threads)
                for bs in bases:
                    oracle.stencils(pts, pts[sub], bs["order"], bs["name"], bs["mask"], p, a_eps, a_rp, a_col,
                                    nthreads=threads)

            # calibrate on 1/64 of the targets, then size the sample for ~cpu_seconds
            m = max(1000, n // 64)
            t1 = time.perf_counter()
            oracle_run(m)
            dt = time.perf_counter() - t1
            m2 = int(min(n, max(m, m * args.cpu_seconds / max(dt, 1e-3))))
            t1 = time.perf_counter()
            oracle_run(m2)
            dt = time.perf_counter() - t1
            what = "all" if m2 == n else f"the first {m2} of the"
            cpu = {"value": round(m2 / dt, 1), "unit": "stencils/s", "cores": threads, "kind": "oracle",
                   "sample": f"{what} {n} targets of the same point cloud: bucket-grid neighbour search + "
                             f"Householder-QR stencils in FP64, {dt:.1f} s wall on {threads} threads"}

        return gate, max_err, len(sample), cpu

    gate, max_err, n_sample, cpu = cpu_baseline_leg()

    # ---- roofline of the stencil phase (its kernels timed by HIP events on
    # the library's stream, inside the timed steps) ----
    flops = alg_flops_workload(nnz, n_t, dim, bases)
    t_sten = float(np.mean(stencil_ms)) * 1e-3
    achieved_tf = flops / t_sten / 1e12
    peak_tf = PEAK["fp32_TFs"] if prec_name == "mixed" else PEAK["fp64_TFs"]
    traffic = measured_traffic(prec_name) if name == DEFAULT_WORKLOAD and n == wl["n"] else None
    roofline = {"bound": "alu", "achieved": round(achieved_tf, 3), "peak": peak_tf, "unit": "TFLOP/s",
                "frac": round(achieved_tf / peak_tf, 4), "traffic": traffic,
                "kernel": "stencil phase: moments, solve and weights kernels of every row-count bin + FP64 "
                          "fallback (one launch sequence per basis per step)",
                "alg_flops_per_step": flops, "alg_bytes_per_step": alg_bytes_workload(nnz, n_t, dim, bases),
                "kernel_ms": round(t_sten * 1e3, 4),
                "frac_of_fp64_peak": round(achieved_tf / PEAK["fp64_TFs"], 4),
                "search_ms": round(float(np.mean(search_ms)), 4)}

    value = n_t / (ms_per_step * 1e-3)
    line = {
        "metric": "GMLS stencils/sec (3D, order 3, uneven nbrs); mixed vs FP64 at <=1e-8 rel err",
        "value": round(value, 1),
        "unit": "stencils/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec_name == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{name}: {DESCRIBE[name]}",
                   "n_points": n, "n_targets": n_t, "nnz": int(nnz), "precision": prec_name,
                   "search": wl["search"][0] + (f" k={k}" if knn else f" r={r0:.6f} k_min={k_min}"),
                   "mixed_scheme": ["auto", "fused, rows residual", "fused, moment Gram",
                                    "pipeline", "wavefront per target"][args.scheme],
                   "autotune": tune_summary,
                   "bases_call": "gmls_stencils_multi (one call for both bases)" if shared else "gmls_stencils per basis",
                   "parity_gate": gate, "parity_max_rel_err": max_err, "parity_sample": int(n_sample),
                   "timed_unit": "HIP graph replay of search + stencils" if graph else "eager calls",
                   "ms_per_step_eager": round(ms_eager, 4),
                   "fallbacks": int(sum(r["n_fallback"] + r["n_not_converged"] for r in reps)),
                   "rank_deficient": int(sum(r["n_rank_deficient"] for r in reps))},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
