"""Comparison rule for CG residual histories (GPU vs oracle).

Kernels are compared bit for bit; a CG history is not, because the GPU sums
each inner product in a fixed tree and the oracle sequentially in extended
precision.  The two recurrences then separate by rounding noise.  One rule
holds at every iteration k:

    |h_gpu[k] - h_ora[k]| <= REL * h_ora[k] + TAU

REL = 1e-12 is the target bar.  TAU is the noise floor in units of the
initial residual (h is relative to ||r_0||): where the residual has fallen
to the rounding level of the recurrence, the two histories differ by an
amount that no longer shrinks with h.  Over every history the GPU tests
compare (4343 entries), the largest gap where h < 1e-6 was 4.4e-20, and
8.7e-22 where h < 1e-13; TAU is ten times the former.  The per-band maxima
and the smallest TAU each session's histories need are printed at its end.
"""
import numpy as np

REL = 1e-12
TAU = 5e-19

# largest observed gaps per band of h_ora, for the session summary
BANDS = (("h >= 1e-6", 1e-6, np.inf), ("1e-13 <= h < 1e-6", 1e-13, 1e-6), ("h < 1e-13", 0.0, 1e-13))
observed = {name: {"abs": 0.0, "rel": 0.0, "count": 0} for name, _, _ in BANDS}
needed_tau = [0.0]  # max over all compared entries of |dh| - REL*h


def _record(d, h_ora):
    for name, lo, hi in BANDS:
        m = (h_ora >= lo) & (h_ora < hi)
        if m.any():
            o = observed[name]
            o["abs"] = max(o["abs"], float(d[m].max()))
            with np.errstate(divide="ignore", invalid="ignore"):
                rel = np.where(h_ora[m] > 0, d[m] / h_ora[m], np.inf)
            o["rel"] = max(o["rel"], float(rel.max()))
            o["count"] += int(m.sum())


def history_violations(h_gpu, h_ora):
    h_gpu, h_ora = np.asarray(h_gpu, dtype=np.float64), np.asarray(h_ora, dtype=np.float64)
    if h_gpu.shape != h_ora.shape:
        return np.array([-1])
    d = np.abs(h_gpu - h_ora)
    _record(d, h_ora)
    if d.size:
        needed_tau[0] = max(needed_tau[0], float(np.max(d - REL * h_ora)))
    bad = ~(d <= REL * h_ora + TAU) | ~np.isfinite(h_gpu)
    return np.nonzero(bad)[0]


def assert_history_close(h_gpu, h_ora):
    bad = history_violations(h_gpu, h_ora)
    assert bad.size == 0, (f"history mismatch at iterations {bad[:6] + 1}: gpu {np.asarray(h_gpu)[bad[:3]]} "
                           f"oracle {np.asarray(h_ora)[bad[:3]]}")


def summary():
    lines = [f"CG history gaps, GPU vs oracle (rule |dh| <= {REL:g}*h + {TAU:g}):"]
    for name, _, _ in BANDS:
        o = observed[name]
        if o["count"]:
            lines.append(f"  {name:20s} entries {o['count']:6d}  max |dh| {o['abs']:.3e}  max |dh|/h {o['rel']:.3e}")
    if len(lines) == 1:
        return []
    lines.append(f"  smallest TAU these histories need: {max(needed_tau[0], 0.0):.3e}")
    return lines
