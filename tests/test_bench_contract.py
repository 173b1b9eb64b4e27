"""CPU checks of the benchmark's command-line contract and of its byte
accounting (no GPU is touched)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""


def test_counted_bytes_of_the_default_workload():
    # 128^3 ILU(0): 6,242,304 off-diagonals in each factor, unit L, one RHS
    n, nnz = 128 ** 3, 6242304
    assert bench.counted_bytes(n, nnz, nnz, 1) == 250478592
    # per launch: L without a diagonal, U with it; their sum is the step
    total = bench.per_launch_bytes(n, nnz, 1, diag=False) + bench.per_launch_bytes(n, nnz, 1, diag=True)
    assert total == 250478592


def test_traffic_line_matches_the_current_kernel_sources():
    # the committed counter summary is valid only for the sources it was taken on
    t = bench.measured_traffic("k_dataflow", "poisson128_ilu0_f64_dataflow")
    assert t is None or 1.0 <= t / 125239296 <= 2.0
