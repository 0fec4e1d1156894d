"""Host-side parts of bench.py that need no GPU: the one-GPU refusal of the
command-line contract, and the algorithmic counts its roofline object
credits (the conventional per-stencil flop count N*Q(Q+1) + Q^3/3 + 2FQ^2 +
2NQF and the bytes 4N + 64 + 8FN per target for a scalar basis)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_scalar_flop_and_byte_counts_per_stencil():
    import bench
    # 3 targets of 10, 20 and 30 neighbours, scalar order 3 in 3-D (Q = 20), one functional
    nnz, n_tgt, Q, F = 60, 3, 20, 1
    basis = {"name": "scalar", "Qs": Q, "Q": Q, "F": F, "C": 1}
    flops = bench.alg_flops_workload(nnz, n_tgt, 3, [basis])
    per_target = [n * Q * (Q + 1) + Q ** 3 / 3.0 + 2 * F * Q * Q + 2 * n * Q * F for n in (10, 20, 30)]
    assert abs(flops - sum(per_target)) < 1e-6 * flops
    assert bench.alg_bytes_workload(nnz, n_tgt, 3, [basis]) == sum(4 * n + 64 + 8 * F * n for n in (10, 20, 30))


def test_shared_gram_is_counted_once_for_two_bases():
    import bench
    nnz, n_tgt = 100, 4
    s = {"name": "scalar", "Qs": 10, "Q": 10, "F": 3, "C": 1}
    v = {"name": "divfree", "Qs": 10, "Q": 17, "F": 2, "C": 3}
    both = bench.alg_flops_workload(nnz, n_tgt, 3, [s, v])
    # the N*Qs*(Qs+1) Gram term appears once; each basis adds its own solve and weights
    gram = nnz * 10 * 11
    only_s = bench.alg_flops_workload(nnz, n_tgt, 3, [s]) - gram
    only_v = bench.alg_flops_workload(nnz, n_tgt, 3, [v]) - gram
    assert abs(both - (gram + only_s + only_v)) < 1e-9 * both


def test_oracle_sample_size():
    """The oracle leg takes every target when they fit twice the timing
    budget, and a sample sized for the budget otherwise."""
    import bench
    n, m = 2_000_000, 31_250
    assert bench.oracle_sample_size(n, m, 0.10, 15.0) == n      # 6.4 s for all
    assert bench.oracle_sample_size(n, m, 0.24, 15.0) == n      # 15.4 s for all: within 2 x 15 s
    k = bench.oracle_sample_size(n, m, 1.0, 15.0)               # 64 s for all
    assert k == int(m * 15.0 / 1.0) and m <= k < n
    assert bench.oracle_sample_size(n, m, 100.0, 15.0) == m     # never below the calibration run
