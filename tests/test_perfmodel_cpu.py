"""The nominal work model the benchmark reports against, and the benchmark's
one-GPU contract.

The expected figures were computed by hand from the byte and flop counts
per step (12 B per nonzero and 24 B per row for a directional sweep, and so
on, as listed in perfmodel's docstring), not by calling the model.
"""
import os
import subprocess
import sys

import pytest

from paper_2304_08232_amd import perfmodel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("dims,dtype,gbytes,gflops", [
    ((128, 128, 128), "fp64", 5.047, 0.810),
    ((128, 128, 128), "fp32", 3.677, 0.810),
    ((192, 192, 192), "fp64", 17.12, 2.750),
    ((192, 192, 192), "fp32", 12.47, 2.750),
])
def test_iteration_totals(dims, dtype, gbytes, gflops):
    B, F = perfmodel.iteration([dims], 4, dtype)
    assert abs(B / 1e9 - gbytes) <= 0.0015 * gbytes
    assert abs(F / 1e9 - gflops) <= 0.0015 * gflops


def test_small_problem_and_standalone_kernels():
    B, F = perfmodel.iteration([(16, 16, 16)], 4, "fp64")
    assert abs(F / 1e6 - 1.4) < 0.05 and abs(B / 1e6 - 8.8) < 0.05
    n, nnz = 128 ** 3, 55742968
    assert perfmodel.level_sizes((128, 128, 128), 4)[0] == (n, nnz)
    # one directional sweep = eight colour passes: 719.2 MB, 119.9 MFLOP
    assert abs(8 * perfmodel.sweep_pass_bytes((128, 128, 128)) / 1e6 - 719.2) < 0.1
    assert abs((2 * nnz + 4 * n) / 1e6 - 119.9) < 0.1
    # the standalone SpMV: 702.5 MB, 111.5 MFLOP
    assert abs((12 * nnz + 16 * n) / 1e6 - 702.5) < 0.1
    assert abs(perfmodel.spmv_bytes((128, 128, 128)) / 1e6 - 702.5) < 0.1
    # a symmetric sweep is two directional sweeps: 1438.4 MB
    assert abs(perfmodel.sym_sweep_bytes((128, 128, 128)) / 1e6 - 1438.4) < 0.1


def test_batched_sum_and_rhs_scaling():
    one = perfmodel.iteration([(32, 32, 32)], 4, "fp64")
    two = perfmodel.iteration([(32, 32, 32), (32, 32, 32)], 4, "fp64")
    assert two[0] == pytest.approx(2 * one[0]) and two[1] == pytest.approx(2 * one[1])
    # sixteen right-hand sides read the matrix once per pass
    b16, f16 = perfmodel.iteration([(32, 32, 32)], 4, "fp64", nrhs=16)
    assert f16 == pytest.approx(16 * one[1])
    assert b16 < 16 * one[0]


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
