"""Writes the stored expected values of the full-size parity tests.

Calls only the CPU oracle (and the seeded input module for sample indices).
Usage: python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import Oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def pcg_128cubed():
    t = time.time()
    o = Oracle(128, 128, 128, levels=4, colour_order=0)
    b = o.spmv(np.ones(o.n()))
    x, hist, it, st = o.pcg(b, max_iters=50, tol=0.0, precond=1)
    assert st == 0 and it == 50
    idx = np.random.default_rng(0).choice(o.n(), size=64, replace=False)
    out = {
        "what": "FP64 MG-PCG, 128x128x128, 4 levels, colour order 0, b = A*1, x0 = 0, 50 iterations",
        "history": [float(v) for v in hist],
        "sample_index": [int(i) for i in idx],
        "sample_x": [float(x[i]) for i in idx],
        "max_abs_err": float(np.abs(x - 1.0).max()),
        "oracle_seconds": round(time.time() - t, 1),
    }
    with open(os.path.join(HERE, "pcg_128cubed_fp64.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    pcg_128cubed()
