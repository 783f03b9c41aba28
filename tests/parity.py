"""Comparison rule for CG residual histories (GPU vs oracle).

Kernels are compared bit for bit; a CG history is not, because the GPU sums
dot products in a fixed tree and the oracle left to right.  The two
recurrences then separate by rounding noise whose size relative to the
residual grows as the residual shrinks.  Rule, per iteration k:
  h_ora >= 1e-6           |h_gpu - h_ora| <= 1e-12 * h_ora   (the target bar)
  1e-13 <= h_ora < 1e-6   |h_gpu - h_ora| <= 1e-6  * h_ora
  h_ora < 1e-13           h_gpu < 1e-12 (both are in the rounding regime)
"""
import numpy as np


def history_violations(h_gpu, h_ora):
    h_gpu, h_ora = np.asarray(h_gpu, dtype=np.float64), np.asarray(h_ora, dtype=np.float64)
    if h_gpu.shape != h_ora.shape:
        return np.array([-1])
    d = np.abs(h_gpu - h_ora)
    strict = h_ora >= 1e-6
    mid = (h_ora < 1e-6) & (h_ora >= 1e-13)
    tail = h_ora < 1e-13
    bad = (strict & (d > 1e-12 * h_ora)) | (mid & (d > 1e-6 * h_ora)) | (tail & ~(h_gpu < 1e-12))
    bad |= ~np.isfinite(h_gpu)
    return np.nonzero(bad)[0]


def assert_history_close(h_gpu, h_ora):
    bad = history_violations(h_gpu, h_ora)
    assert bad.size == 0, (f"history mismatch at iterations {bad[:6] + 1}: gpu {np.asarray(h_gpu)[bad[:3]]} "
                           f"oracle {np.asarray(h_ora)[bad[:3]]}")
