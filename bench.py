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
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target duration of the oracle timing leg (every target when they are estimated to "
                         "take at most twice this)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scheme", type=int, default=0,
                    help="mixed scheme: 0 auto, 1 fused/rows residual, 2 fused/moment Gram, 3 pipeline, 4 wavefront per target")
    ap.add_argument("--chunk", type=int, default=0, help="pipeline chunk (targets; 0 = whole batch)")
    ap.add_argument("--layout", choices=["sorted", "index"], default="index",
                    help="stencil sources: the search's cell-ordered records (gmls_neighbors_sorted) or the "
                         "points in their own order")
    ap.add_argument("--no-autotune", action="store_true",
                    help="mixed pipeline: keep the default row shapes instead of autotuning them first")
    ap.add_argument("--tune-cache", default="",
                    help="autotune table (JSON): loaded if the file exists, else written after tuning")
    ap.add_argument("--copy-probe", action="store_true", help="run a 1 GiB device copy (counter scaling) and exit")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager calls instead of HIP graph replays of search + stencils")
    ap.add_argument("--no-fp64", action="store_true",
                    help="mixed workloads: skip the FP64 leg (timed and checked after the mixed one by default)")
    ap.add_argument("--cpu-seconds-1", type=float, default=6.0,
                    help="target duration of the one-core oracle timing")
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


def oracle_sample_size(n, m, dt, cpu_seconds):
    """Targets for the oracle's timing leg, from a calibration run of m
    targets that took dt seconds: every target when they are estimated to
    take at most twice cpu_seconds (so that the all-target parity does not
    hinge on the host's speed), else enough for about cpu_seconds."""
    if dt * n / m <= 2 * cpu_seconds:
        return n
    return int(min(n, max(m, m * cpu_seconds / max(dt, 1e-3))))


def host_info():
    """Host cores available to this job and the CPU model.  The oracle's
    timing uses every core of the job's CPU share: the affinity mask, capped
    by OMP_NUM_THREADS where the launcher sets it (one GPU's share of the
    host)."""
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    omp = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(avail, int(omp)) if omp.isdigit() and int(omp) > 0 else avail
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": nproc, "affinity": avail, "omp_num_threads": omp or None, "threads": threads,
            "cpu_model": model}


def executed_flops_workload(nnz, n_tgt, dim, bases):
    """The count of the arithmetic the mixed and FP64-moment kernels do for
    the Gram: the weighted moments of degree <= 2m, 2*NM flops per
    neighbour row (NM monomials), in place of the conventional N*Q*(Q+1);
    the other terms as in alg_flops_workload."""
    qs_max = max(b["Qs"] for b in bases)
    order = max(b["order"] + (1 if b["name"] == "staggered" else 0) for b in bases)
    nm = _binom(2 * order + dim, dim)
    return alg_flops_workload(nnz, n_tgt, dim, bases) - nnz * qs_max * (qs_max + 1) + nnz * 2 * nm


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.stokes:
        stokes_main(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
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

    precs = {"mixed": G.PREC_MIXED, "fp64": G.PREC_FP64}
    if args.prec == "auto":
        prec_name = "mixed" if "mixed" in wl["modes"] else "fp64"
    else:
        prec_name = args.prec
    legs = [prec_name]
    if prec_name == "mixed" and "fp64" in wl["modes"] and not args.no_fp64:
        legs.append("fp64")

    def stencils(c, prec, bs, src, eps_, rp_, col_, weights=None, status=None, aux=None, report=False):
        """One basis of the configuration through its entry point; `aux`
        receives the h-weights (constrained) or target weights (staggered)."""
        if bs["name"] == "staggered":
            return G.gmls_stencils_staggered(c, src, xt, bs["order"], bs["mask"], p, eps_, rp_, col_, prec=prec,
                                             weights=weights, t_weights=aux, status=status, report=report)
        if bs["name"] == "neumann":
            return G.gmls_stencils_constrained(c, src, xt, bs["order"], bs["mask"], p, eps_, rp_, col_, nrm,
                                               prec=prec, weights=weights, h_weights=aux, status=status,
                                               report=report)
        w_, st_, r_ = G.gmls_stencils(c, src, xt, bs["order"], bs["b"], bs["mask"], p, eps_, rp_, col_, prec=prec,
                                      weights=weights, status=status, report=report)
        return w_, None, st_, r_

    # a scalar and a divergence-free basis of one order on the same neighbour
    # lists go through one gmls_stencils_multi call (the library shares their
    # Gram where the scheme allows)
    shared = len(bases) == 2 and sorted(b["name"] for b in bases) == ["divfree", "scalar"] and \
        bases[0]["order"] == bases[1]["order"]

    def all_stencils(c, prec, src, eps_, rp_, col_, bufs, report=False):
        if shared:
            outs = [(bufs[i]["w"], bufs[i]["st"]) for i in range(len(bases))]
            return [G.gmls_stencils_multi(c, src, xt, bases[0]["order"], p, eps_, rp_, col_,
                                          [(bs["b"], bs["mask"]) for bs in bases], prec=prec, outputs=outs,
                                          report=report)[1]]
        return [stencils(c, prec, bs, src, eps_, rp_, col_, weights=bufs[i]["w"], status=bufs[i]["st"],
                         aux=bufs[i]["aux"], report=report)[3] for i, bs in enumerate(bases)]

    # source layout of the stencil calls: the search's cell-ordered records
    # and the rows as positions in them (gmls_neighbors_sorted, source stride
    # 4), or the points in their own order
    sorted_layout = args.layout == "sorted"

    def search(c, col=None, pcol=None, rec=None):
        """(row_ptr, col, eps, stencil sources, stencil rows)"""
        if sorted_layout:
            rp_, col_, eps_, rec_, pcol_ = G.gmls_neighbors_sorted(c, x, xt, col=col, col_sorted=pcol, records=rec,
                                                                   **spec)
            return rp_, col_, eps_, rec_, pcol_
        rp_, col_, eps_ = G.gmls_neighbors(c, x, xt, col=col, **spec)
        return rp_, col_, eps_, x, col_

    if sorted_layout:
        ctx.set_option(G.OPT_SOURCE_STRIDE, 4)
    rp0, col0, eps0, src0, scol0 = search(ctx)
    nnz = col0.numel()
    col_buf = torch.empty(int(nnz * 1.05) + 1024, dtype=torch.int32, device=dev)
    pcol_buf = torch.empty_like(col_buf) if sorted_layout else None
    rec_buf = torch.empty((n, 4), dtype=torch.float64, device=dev) if sorted_layout else None

    def new_bufs():
        return [dict(w=torch.empty(bs["F"] * bs["C"] * nnz, dtype=torch.float64, device=dev),
                     st=torch.empty(n_t, dtype=torch.uint8, device=dev),
                     aux=torch.empty((n_t, bs["F"]), dtype=torch.float64, device=dev)) for bs in bases]

    # ---- autotune the mixed pipeline's row shapes (before any timing) ----
    # ---- autotune the per-bin kernel shapes (before any timing): the mixed
    # scheme's kernels and the FP64 QR kernel, per basis and, for a scalar and
    # a divergence-free basis on one call, the shared kernels ----
    tune_summary = "off"
    tune_path = None
    if not args.no_autotune:
        if args.tune_cache and os.path.exists(args.tune_cache):
            G.gmls_autotune_load(ctx, args.tune_cache)
            tune_summary = {"loaded": args.tune_cache}
            tune_path = args.tune_cache
        else:
            tune_summary = {}
            t0 = time.time()
            jobs = []
            for bs in bases:
                if bs["name"] == "neumann":
                    continue
                # staggered stencils run the scalar pipeline of order + 1
                order_t, b_t = (bs["order"] + 1, G.BASIS_SCALAR) if bs["name"] == "staggered" \
                    else (bs["order"], bs["b"])
                jobs.append((bs["name"], order_t, b_t, bs["mask"]))
                if bs["name"] == "staggered":  # its FP64 QR kernel has a key of its own
                    jobs.append(("staggered-qr", bs["order"], G.TUNE_STAGGERED, bs["mask"]))
            if shared:
                ms_ = [bs["mask"] for bs in bases if bs["name"] == "scalar"][0]
                mv_ = [bs["mask"] for bs in bases if bs["name"] == "divfree"][0]
                jobs.append(("shared", bases[0]["order"], G.TUNE_SHARED, ms_ | (mv_ << 4)))
            for name_t, order_t, b_t, mask_t in jobs:
                try:
                    res = G.gmls_autotune(ctx, src0, xt, order_t, b_t, mask_t, p, eps0, rp0, scol0, reps=3)
                except G.GmlsError as e:
                    if e.status != G.GMLS_ERR_UNSUPPORTED:  # no tunable kernel compiled for the shape
                        raise
                    continue
                tune_summary[name_t] = {k_: {b: "x".join(str(u) for u in v["chosen"]) for b, v in d.items()}
                                        for k_, d in res.items()}
            print(f"# autotune: {tune_summary} ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
            if tune_summary:
                if args.tune_cache:
                    tune_path = args.tune_cache
                else:
                    fd, tune_path = tempfile.mkstemp(suffix=".json")
                    os.close(fd)
                G.gmls_autotune_save(ctx, tune_path)
            else:
                tune_summary = "nothing tunable in this configuration"

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run_leg(leg):
        """Eager steps (per-phase HIP event times, reports), then the timed
        unit: HIP graph replays of search + stencils.  Returns the figures and
        the outputs of the last replay."""
        prec = precs[leg]
        bufs = new_bufs()

        def step(report=False):
            ev0.record()
            rp_, col_, eps_, src_, scol_ = search(ctx, col_buf, pcol_buf, rec_buf)
            ev1.record()
            reps_ = all_stencils(ctx, prec, src_, eps_, rp_, scol_, bufs, report=report)
            return rp_, col_, eps_, reps_

        for i in range(args.warmup):
            step()
            print(f"# {leg}: warmup step {i} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        stencil_ms, search_ms = [], []
        t_start = time.perf_counter()
        for i in range(args.steps):
            out_ = step(report=True)
            stencil_ms.append(sum(r["t_stencil_ms"] + r["t_fallback_ms"] for r in out_[3]))
            search_ms.append(ev0.elapsed_time(ev1))
        torch.cuda.synchronize()
        ms_eager = 1e3 * (time.perf_counter() - t_start) / args.steps
        rp_t, col_t, eps_t, reps_ = out_
        print(f"# {leg} eager: {args.steps} steps: {ms_eager:.3f} ms/step; stencil kernels "
              f"{np.mean(stencil_ms):.3f} ms; search {np.mean(search_ms):.3f} ms; reports {reps_}",
              file=sys.stderr, flush=True)
        res = {"prec": leg, "ms_eager": ms_eager, "stencil_ms": float(np.mean(stencil_ms)),
               "search_ms": float(np.mean(search_ms)), "reports": reps_, "ms_per_step": ms_eager,
               "graph": False}
        out = {"rp": rp_t, "col": col_t, "eps": eps_t, "bufs": bufs}
        if not args.no_graph:
            gs = torch.cuda.Stream()
            gctx = G.Context(0, stream=gs)
            gctx.set_option(G.OPT_MIXED_SCHEME, args.scheme)
            if sorted_layout:
                gctx.set_option(G.OPT_SOURCE_STRIDE, 4)
            if tune_path:
                G.gmls_autotune_load(gctx, tune_path)  # the same shapes as the eager steps
            gbufs = new_bufs()
            gcol = torch.empty(nnz + 1024, dtype=torch.int32, device=dev)
            gpcol = torch.empty_like(gcol) if sorted_layout else None
            grec = torch.empty((n, 4), dtype=torch.float64, device=dev) if sorted_layout else None
            with torch.cuda.stream(gs):
                # one normal call of each kind sizes the context's workspace
                rpw, colw, epsw, srcw, scolw = search(gctx)
                all_stencils(gctx, prec, srcw, epsw, rpw, scolw, gbufs)
                gctx.set_option(G.OPT_CAPTURE_SAFE, 1)
                gout = {}

                def gstep():
                    rp_, col_, eps_, src_, scol_ = search(gctx, gcol, gpcol, grec)
                    all_stencils(gctx, prec, src_, eps_, rp_, scol_[:nnz], gbufs)
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
            res["ms_per_step"] = 1e3 * (time.perf_counter() - t_start) / args.steps
            res["graph"] = True
            gctx.check()
            print(f"# {leg} graph: {args.steps} replays: {res['ms_per_step']:.3f} ms/step", file=sys.stderr,
                  flush=True)
            # the parity gate checks the replayed outputs
            out = {"rp": gout["rp"], "col": gcol[:nnz], "eps": gout["eps"], "bufs": gbufs}
        return res, out

    results, outputs = {}, {}
    for leg in legs:
        results[leg], outputs[leg] = run_leg(leg)
    if tune_path and not args.tune_cache:
        os.remove(tune_path)

    # ---- the CPU-baseline leg: the only part of this file that uses the
    # oracle.  It times the oracle on the host cores (all of the job's share,
    # then one core), and checks the timed runs' outputs against the oracle's:
    # every target the timed oracle run covered, plus a random sample ----
    import oracle

    tol_of = {"mixed": 1e-8, "fp64": 1e-10}

    def oracle_stencils(sub_pts, o_rp, o_col, o_eps, nthreads=0):
        outs = []
        for bs in bases:
            if bs["name"] == "staggered":
                from oracle import staggered as OS
                ow, oaux, _ = OS.stencils_staggered(pts, sub_pts, bs["order"], bs["mask"], p, o_eps, o_rp, o_col)
                ost = np.zeros(len(sub_pts), dtype=np.uint8)
            elif bs["name"] == "neumann":
                from oracle import constrained as OC
                ow, oaux, _ = OC.stencils_constrained(pts, sub_pts, bs["order"], bs["mask"], p, o_eps, o_rp, o_col,
                                                      nrm_h[:len(sub_pts)] if sub_pts is tpts else nrm_h[o_sel])
                ost = np.zeros(len(sub_pts), dtype=np.uint8)
            else:
                ow, ost, _, _ = oracle.stencils(pts, sub_pts, bs["order"], bs["name"], bs["mask"], p, o_eps, o_rp,
                                                o_col, nthreads=nthreads)
                oaux = None
            outs.append((ow, ost, oaux))
        return outs

    def oracle_search(sub_pts, nthreads=0, use_grid=None):
        if knn:
            return oracle.knn(pts, sub_pts, k, mult, use_grid=use_grid, nthreads=nthreads)
        return oracle.radius(pts, sub_pts, r0, k_min, use_grid=use_grid, nthreads=nthreads)

    def compare(leg, m, o_rp, o_col, o_eps, o_out, sel=None):
        """GPU outputs of `leg` for targets sel (default: 0..m-1) against the
        oracle's: search bit for bit (radius rows as sets), statuses, and the
        weights per (target, functional row) relative error.  Radius rows are
        matched by sorting each GPU row by source index on the GPU (torch,
        as test plumbing); the weights follow the same permutation."""
        o = outputs[leg]
        if sel is None:
            rph = o["rp"][: m + 1].cpu().numpy()
            g_idx = torch.arange(int(rph[-1]), device=dev)
            cols = o["col"][: int(rph[-1])]
            wsel = None
        else:
            rp_all = o["rp"].cpu().numpy()
            lens = np.diff(rp_all)[sel]
            rph = np.zeros(len(sel) + 1, dtype=np.int64)
            rph[1:] = np.cumsum(lens)
            g_idx = torch.from_numpy(np.concatenate([np.arange(rp_all[t], rp_all[t + 1]) for t in sel])).to(dev)
            cols = o["col"][g_idx]
            wsel = rp_all[sel]
        search_ok = np.array_equal(rph, o_rp)
        nn = int(rph[-1])
        cnt = torch.from_numpy(np.diff(rph)).to(dev)
        rows = torch.repeat_interleave(torch.arange(len(rph) - 1, device=dev), cnt)
        if search_ok:
            if knn:
                perm = torch.arange(nn, device=dev)
                search_ok = np.array_equal(cols.cpu().numpy(), o_col)
            else:
                keys = (rows << 32) | cols.to(torch.int64)
                skeys, perm = torch.sort(keys)
                okeys = (torch.from_numpy(np.repeat(np.arange(len(rph) - 1), np.diff(o_rp))).to(dev) << 32) | \
                    torch.from_numpy(o_col.astype(np.int64)).to(dev)
                search_ok = bool(torch.equal(skeys, okeys))
            eps_g = o["eps"].cpu().numpy()[sel] if sel is not None else o["eps"][:m].cpu().numpy()
            search_ok = search_ok and np.array_equal(eps_g, o_eps)
        if not search_ok:
            return {"search_ok": False, "status_ok": False, "max": float("inf"), "p99": float("inf"),
                    "p50": float("inf"), "targets": len(rph) - 1}
        rp_d = torch.from_numpy(rph[:-1]).to(dev)
        jd = torch.arange(nn, device=dev) - rp_d[rows]       # position in the oracle's row
        js = perm - rp_d[rows]                                # the GPU's position of that entry
        nrow = cnt[rows]
        errs_all, status_ok = [], True
        for i, bs in enumerate(bases):
            F, C = bs["F"], bs["C"]
            ow, ost, oaux = o_out[i]
            gst = o["bufs"][i]["st"].cpu().numpy()
            gst = gst[sel] if sel is not None else gst[:m]
            status_ok = status_ok and np.array_equal(gst == 1, ost == 1)
            gw = o["bufs"][i]["w"]
            if wsel is not None:
                gbase = torch.from_numpy(F * C * wsel).to(dev)[rows]
            else:
                gbase = F * C * rp_d[rows]
            obase = F * C * rp_d[rows]
            wo = torch.from_numpy(ow).to(dev)
            d2 = torch.zeros(len(rph) - 1, F, dtype=torch.float64, device=dev)
            r2 = torch.zeros_like(d2)
            for f in range(F):
                for c in range(C):
                    a = gw[gbase + (f * nrow + js) * C + c]
                    b = wo[obase + (f * nrow + jd) * C + c]
                    d2[:, f].index_add_(0, rows, (a - b) ** 2)
                    r2[:, f].index_add_(0, rows, b * b)
            if bs["name"] == "divfree" and bs["mask"] & G.F_DIV:
                r2[:, F - 1] = r2[:, 0]  # identically zero row: the same target's scale
            if oaux is not None:  # target weights / h-weights, relative to the row norms
                ga = o["bufs"][i]["aux"][:m] if sel is None else o["bufs"][i]["aux"][torch.from_numpy(sel).to(dev)]
                oa = torch.from_numpy(np.asarray(oaux).reshape(len(rph) - 1, F)).to(dev)
                d2 = d2 + (ga - oa) ** 2
                r2 = r2 + oa * oa
            e = torch.sqrt(d2 / r2)
            live = torch.from_numpy(ost != 1).to(dev)
            errs_all.append(e[live].reshape(-1))
        errs = torch.cat(errs_all).cpu().numpy() if errs_all else np.zeros(1)
        return {"search_ok": True, "status_ok": bool(status_ok), "max": float(errs.max()),
                "p99": float(np.percentile(errs, 99)), "p50": float(np.percentile(errs, 50)),
                "targets": len(rph) - 1, "tol": tol_of[leg],
                "gate": bool(status_ok and errs.max() <= tol_of[leg])}

    info = host_info()
    threads = info["threads"]
    full_ok = all(bs["name"] in ("scalar", "divfree") for bs in bases) and n_t == n
    cpu = None
    parity = {}
    o_sel = None
    # a random sample over the whole cloud (every workload)
    g = W.rng(424242)
    o_sel = np.sort(g.choice(n_t, size=min(args.sample, n_t), replace=False))
    s_rp, s_col, s_eps = oracle_search(tpts[o_sel])
    s_out = oracle_stencils(tpts[o_sel], s_rp, s_col, s_eps)
    for leg in legs:
        parity[leg] = {"random_sample": compare(leg, 0, s_rp, s_col, s_eps, s_out, sel=o_sel)}
        print(f"# {leg} parity on {len(o_sel)} random targets: {parity[leg]['random_sample']}", file=sys.stderr,
              flush=True)
    if full_ok and not args.no_cpu_baseline:
        def oracle_run(m_, nthreads):
            sub = tpts[:m_]
            a_rp, a_col, a_eps = oracle_search(sub, nthreads=nthreads, use_grid=True)
            outs_ = [oracle.stencils(pts, sub, bs["order"], bs["name"], bs["mask"], p, a_eps, a_rp, a_col,
                                     nthreads=nthreads)[:2] + (None,) for bs in bases]
            return a_rp, a_col, a_eps, outs_

        # calibrate on 1/64 of the targets, then size the sample
        m = max(1000, n // 64)
        t1 = time.perf_counter()
        oracle_run(m, threads)
        dt = time.perf_counter() - t1
        m2 = oracle_sample_size(n, m, dt, args.cpu_seconds)
        t1 = time.perf_counter()
        a_rp, a_col, a_eps, a_out = oracle_run(m2, threads)
        dt2 = time.perf_counter() - t1
        what = "all" if m2 == n else f"the first {m2} of the"
        # one core: a sample sized from the all-core rate for ~cpu_seconds_1
        m1 = int(min(m2, max(200, (m2 / dt2) / threads * args.cpu_seconds_1)))
        t1 = time.perf_counter()
        oracle_run(m1, 1)
        dt1 = time.perf_counter() - t1
        cpu = {"value": round(m2 / dt2, 1), "unit": "stencils/s", "cores": threads, "kind": "oracle",
               "sample": f"{what} {n} targets of the same point cloud: bucket-grid neighbour search + "
                         f"Householder-QR stencils in FP64, {dt2:.1f} s wall on {threads} threads",
               "value_1core": round(m1 / dt1, 1),
               "sample_1core": f"the first {m1} targets, {dt1:.1f} s wall on 1 thread",
               "host": info}
        print(f"# oracle: {cpu}", file=sys.stderr, flush=True)
        for leg in legs:
            parity[leg]["oracle_run"] = compare(leg, m2, a_rp, a_col, a_eps, a_out)
            print(f"# {leg} parity on the first {m2} targets: {parity[leg]['oracle_run']}", file=sys.stderr,
                  flush=True)
        del a_rp, a_col, a_eps, a_out

    def summary(leg):
        pr = parity[leg]
        parts = [v for v in pr.values()]
        full = pr.get("oracle_run")
        return {"gate": bool(all(v["search_ok"] and v["status_ok"] and v["max"] <= tol_of[leg] for v in parts)),
                "max_rel_err": max(v["max"] for v in parts),
                "p99_rel_err": (full or pr["random_sample"])["p99"],
                "p50_rel_err": (full or pr["random_sample"])["p50"],
                "targets_compared": (full["targets"] if full else 0) + pr["random_sample"]["targets"],
                "all_targets": bool(full and full["targets"] == n_t)}

    head = results[legs[0]]
    sum_head = summary(legs[0])
    # ---- roofline of the stencil phase (its kernels timed by HIP events on
    # the library's stream, inside the timed steps).  No MFMA and no packed
    # FP32 instruction executes (packed FP32 is disabled at build time), so
    # FP32 and FP64 vector arithmetic run at the same rate: the peak of the
    # arithmetic that executes is the FP64 vector peak in both precisions ----
    flops = alg_flops_workload(nnz, n_t, dim, bases)
    flops_exec = executed_flops_workload(nnz, n_t, dim, bases)
    t_sten = head["stencil_ms"] * 1e-3
    achieved_tf = flops / t_sten / 1e12
    peak_tf = PEAK["fp64_TFs"]
    traffic = measured_traffic(legs[0]) if name == DEFAULT_WORKLOAD and n == wl["n"] else None
    alg_bytes = alg_bytes_workload(nnz, n_t, dim, bases)
    roofline = {"bound": "alu", "achieved": round(achieved_tf, 3), "peak": peak_tf, "unit": "TFLOP/s",
                "frac": round(achieved_tf / peak_tf, 4), "traffic": traffic,
                "kernel": "stencil phase: moments, solve and weights kernels of every row-count bin + FP64 "
                          "fallback (one launch sequence per basis per step)",
                "peak_basis": "FP64 vector (78.6 TF): no MFMA and no packed FP32 executes, so FP32 runs at the "
                              "FP64 rate",
                "alg_flops_per_step": flops, "alg_bytes_per_step": alg_bytes,
                "executed_flops_per_step": flops_exec,
                "achieved_executed": round(flops_exec / t_sten / 1e12, 3),
                "frac_executed": round(flops_exec / t_sten / 1e12 / peak_tf, 4),
                "alg_hbm_GBs": round(alg_bytes / t_sten / 1e9, 1),
                "alg_hbm_frac": round(alg_bytes / t_sten / 1e9 / PEAK["hbm_GBs"], 4),
                "kernel_ms": round(t_sten * 1e3, 4),
                "search_ms": round(head["search_ms"], 4)}
    if traffic:
        roofline["traffic_GBs"] = round(traffic / t_sten / 1e9, 1)
        roofline["traffic_hbm_frac"] = round(traffic / t_sten / 1e9 / PEAK["hbm_GBs"], 4)
        roofline["traffic_over_alg_bytes"] = round(traffic / alg_bytes, 2)

    def leg_fields(leg):
        r = results[leg]
        sm = summary(leg)
        reps_ = r["reports"]
        return {"ms_per_step": round(r["ms_per_step"], 4), "value": round(n_t / (r["ms_per_step"] * 1e-3), 1),
                "timed_unit": "HIP graph replay of search + stencils" if r["graph"] else "eager calls",
                "ms_per_step_eager": round(r["ms_eager"], 4), "stencil_ms": round(r["stencil_ms"], 4),
                "search_ms": round(r["search_ms"], 4),
                "stencils_only_per_s": round(n_t / (r["stencil_ms"] * 1e-3), 1),
                "parity_gate": sm["gate"], "parity_max_rel_err": sm["max_rel_err"],
                "parity_p99_rel_err": sm["p99_rel_err"], "parity_p50_rel_err": sm["p50_rel_err"],
                "parity_sample": sm["targets_compared"], "parity_all_targets": sm["all_targets"],
                "fallbacks": int(sum(x_["n_fallback"] + x_["n_not_converged"] for x_ in reps_)),
                "rank_deficient": int(sum(x_["n_rank_deficient"] for x_ in reps_)),
                "cond": {"min": min(x_["cond_min"] for x_ in reps_), "med": reps_[0]["cond_med"],
                         "max": max(x_["cond_max"] for x_ in reps_)}}

    hf = leg_fields(legs[0])
    value = n_t / (head["ms_per_step"] * 1e-3)
    # FP32 executes only in the Cholesky factor of the pipeline's scalar
    # solve (scalar bases of at most 20 functions; scheme 4, forced, is
    # FP64 throughout): elsewhere the mixed path's arithmetic is FP64
    fp32_used = legs[0] == "mixed" and args.scheme != 4 and any(
        bs["name"] in ("scalar", "staggered") and bs["Q"] <= 20 for bs in bases)
    line = {
        "metric": "GMLS stencils/sec (3D, order 3, uneven nbrs); mixed vs FP64 at <=1e-8 rel err",
        "value": round(value, 1),
        "unit": "stencils/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if fp32_used else "f64",
        "data": "synthetic",
        "config": {"workload": f"{name}: {DESCRIBE[name]}",
                   "n_points": n, "n_targets": n_t, "nnz": int(nnz), "precision": legs[0],
                   "search": wl["search"][0] + (f" k={k}" if knn else f" r={r0:.6f} k_min={k_min}"),
                   "source_layout": ("cell-ordered records (gmls_neighbors_sorted, source stride 4)"
                                     if sorted_layout else "points in their own order"),
                   "mixed_scheme": ["auto", "fused, rows residual", "fused, moment Gram",
                                    "pipeline", "wavefront per target"][args.scheme],
                   "autotune": tune_summary,
                   "bases_call": "gmls_stencils_multi (one call for both bases)" if shared else "gmls_stencils per basis",
                   "timed_unit": hf["timed_unit"],
                   "ms_per_step_eager": hf["ms_per_step_eager"],
                   "stencils_only_per_s": hf["stencils_only_per_s"],
                   "parity_gate": hf["parity_gate"], "parity_max_rel_err": hf["parity_max_rel_err"],
                   "parity_p99_rel_err": hf["parity_p99_rel_err"], "parity_p50_rel_err": hf["parity_p50_rel_err"],
                   "parity_sample": hf["parity_sample"], "parity_all_targets": hf["parity_all_targets"],
                   "fallbacks": hf["fallbacks"], "rank_deficient": hf["rank_deficient"], "cond": hf["cond"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if "fp64" in legs and legs[0] != "fp64":
        ff = leg_fields("fp64")
        ff["mixed_speedup"] = round(results["fp64"]["ms_per_step"] / head["ms_per_step"], 3)
        ff["dtype"] = "f64"
        line["fp64"] = ff
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
