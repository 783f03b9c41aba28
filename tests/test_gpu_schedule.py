"""Execution schedules and the autotuner.

A schedule changes how the kernels are launched (graph or eager, coarse
levels per pass / single-workgroup tail / persistent, 64- or 256-thread
workgroups per level, the sequential smoother's run limit), never what they
compute: solves must be bit-identical under every schedule, except for the
level-0 workgroup choice on problems whose <r,z> is fused into the level-0
post-smoother, which regroups that sum (compared to the oracle instead).
"""
import json
import os

import numpy as np
import pytest

from oracle import Oracle
from paper_2304_08232_amd import inputs
from parity import assert_history_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_08232_amd import mgpcg
    mgpcg.lib()
    return mgpcg


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def solve(p, b, iters=12):
    x, h, its, st = p.solve(b, max_iters=iters)
    torch.cuda.synchronize()
    return x.clone(), h.copy()


def candidates(levels, fuse_l0):
    out = []
    for graph in (1, 0):
        for cm, ct in ((0, 1), (0, 0), (1, 1)):
            for wide in range(1 << levels):
                if fuse_l0 and wide & 1:
                    continue
                out.append(dict(graph=graph, coarse_mode=cm, coarse_tail=ct, wide_levels=wide, lex_run_rows=256))
    return out


@pytest.mark.parametrize("case", ["single", "batched", "multi_rhs", "fp32"])
def test_every_schedule_bit_identical(mg, case):
    if case == "single":
        p, n = mg.Problem((32, 32, 32), levels=4), 32 ** 3
    elif case == "batched":
        dims = [(16, 16, 16), (24, 16, 32), (8, 16, 8)]
        p, n = mg.Problem(dims, levels=4), sum(a * b * c for a, b, c in dims)
    elif case == "multi_rhs":
        p, n = mg.Problem((16, 16, 16), nrhs=4), 4 * 16 ** 3
    else:
        p, n = mg.Problem((32, 32, 32), mg_dtype="fp32"), 32 ** 3
    print(f"schedules {case}", flush=True)
    b = dev(inputs.uniform(7, n))
    default = p.schedule
    x0, h0 = solve(p, b)
    # one grid in FP64: <r,z> rides on the level-0 post-smoother, whose
    # workgroup width regroups its partials
    fuse_l0 = case in ("single", "multi_rhs") and not default["wide_levels"] & 1
    for c in candidates(4, fuse_l0):
        p.set_schedule(**c)
        assert p.schedule == c
        x, h = solve(p, b)
        assert torch.equal(x, x0) and np.array_equal(h, h0), c
    p.check()


def test_every_schedule_order1_matches_oracle(mg):
    # Colour order 1 cannot fuse the transfers into the passes, so its levels
    # run the unfused restriction and refinement kernels, and a level whose
    # wide_levels bit is set runs the 256-thread, non-temporal builds with the
    # order-1 zero-start masks (by default only levels above 128 MiB, i.e. at
    # 128^3 and up).  Every schedule is compared with the oracle: the V-cycle
    # bit for bit, the CG history by the history rule (changing bit 0 regroups
    # the fused <r,z> partials, so solves are not bit-identical across it).
    dims = (32, 32, 32)
    o = Oracle(*dims, colour_order=1)
    p = mg.Problem(dims, levels=4, colour_order=1)
    print("schedules order 1", flush=True)
    r = inputs.uniform(12, o.n())
    z_ref = o.vcycle(r)
    b = inputs.uniform(7, o.n())
    xo, ho, ito, _ = o.pcg(b, max_iters=12)
    base = {}
    for c in candidates(4, False):
        p.set_schedule(**c)
        assert p.schedule == c
        np.testing.assert_array_equal(p.vcycle(dev(r)).cpu().numpy(), z_ref, err_msg=str(c))
        x, h = solve(p, dev(b))
        assert_history_close(h[0], ho)
        # within one setting of bit 0 every other choice is bit-identical
        key = c["wide_levels"] & 1
        if key in base:
            assert torch.equal(x, base[key][0]) and np.array_equal(h, base[key][1]), c
        else:
            base[key] = (x, h)
    p.check()


def test_level0_width_on_fused_problem_matches_oracle(mg):
    dims = (32, 32, 32)
    o = Oracle(*dims)
    p = mg.Problem(dims)
    b = inputs.uniform(8, o.n())
    xo, ho, ito, _ = o.pcg(b, max_iters=200, tol=1e-9)
    for wide0 in (0, 1):
        s = p.schedule
        p.set_schedule(wide_levels=(s["wide_levels"] & ~1) | wide0)
        x, h, its, st = p.solve(dev(b), max_iters=200, tol=1e-9)
        assert st == mg.OK and its[0] == ito
        assert_history_close(h[0, :ito], ho)


@pytest.mark.parametrize("rr", [0, 64, 512])
def test_sequential_run_limit_bit_identical(mg, rr):
    dims = (16, 8, 24)
    o = Oracle(*dims)
    p = mg.Problem(dims, smoother="sequential")
    r = inputs.uniform(9, o.n())
    p.set_schedule(lex_run_rows=rr)
    np.testing.assert_array_equal(p.vcycle(dev(r)).cpu().numpy(), o.vcycle_lex(r))


def test_invalid_schedules(mg):
    p = mg.Problem((16, 16, 16), levels=3)
    good = p.schedule
    for bad in (dict(graph=2), dict(coarse_mode=-1), dict(coarse_tail=5), dict(wide_levels=8),
                dict(lex_run_rows=513)):
        with pytest.raises(mg.MGPCGError):
            p.set_schedule(**bad)
        assert p.schedule == good
    with pytest.raises(mg.MGPCGError):
        p.autotune(iters=0)


def test_autotune_applies_caches_and_keeps_results(mg, tmp_path):
    dims = (32, 32, 32)
    p = mg.Problem(dims)
    b = dev(inputs.uniform(10, 32 ** 3))
    x0, h0 = solve(p, b)
    cache = str(tmp_path / "tune.jsonl")
    chosen = p.autotune(b, iters=5, reps=2, cache_path=cache)
    assert p.schedule == chosen
    x1, h1 = solve(p, b)
    assert torch.equal(x1, x0) and np.array_equal(h1, h0)  # level 0 is left alone here
    lines = open(cache).read().splitlines()
    assert len(lines) == 1
    entry = json.loads(lines[0])
    assert "dims=32x32x32" in entry["key"] and entry["graph"] == chosen["graph"]
    # a cache entry is applied without timing: plant a different schedule
    planted = dict(chosen, graph=1 - chosen["graph"], coarse_tail=1 - chosen["coarse_tail"])
    entry.update(planted)
    with open(cache, "a") as f:
        f.write(json.dumps(entry) + "\n")
    q = mg.Problem(dims)
    assert q.autotune(b, iters=5, reps=2, cache_path=cache) == planted
    assert q.schedule == planted
    # another problem shape gets its own entry
    r = mg.Problem((16, 16, 16))
    r.autotune(None, iters=5, reps=1, cache_path=cache)
    assert len(open(cache).read().splitlines()) == 3
    # an entry this build rejects (coarse_mode 7) is ignored: the tuning runs
    # and appends a valid entry, and the results stay bit-identical
    bad = dict(entry, coarse_mode=7)
    with open(cache, "a") as f:
        f.write(json.dumps(bad) + "\n")
    u = mg.Problem(dims)
    tuned = u.autotune(b, iters=5, reps=2, cache_path=cache)
    assert tuned["coarse_mode"] in (0, 1) and u.schedule == tuned
    assert len(open(cache).read().splitlines()) == 5
    x2, h2 = solve(u, b)
    assert torch.equal(x2, x0) and np.array_equal(h2, h0)


def test_autotune_batched_and_sequential(mg):
    dims = [(16, 16, 16), (24, 16, 32), (8, 16, 8)]
    p = mg.Problem(dims, levels=4)
    sizes = [a * b * c for a, b, c in dims]
    b = dev(inputs.batch_rhs(9, sizes))
    x0, h0 = solve(p, b)
    p.autotune(b, iters=4, reps=1)
    x1, h1 = solve(p, b)
    assert torch.equal(x1, x0) and np.array_equal(h1, h0)
    q = mg.Problem((16, 16, 16), smoother="sequential")
    bq = dev(inputs.uniform(11, 16 ** 3))
    y0, g0 = solve(q, bq)
    s = q.autotune(bq, iters=3, reps=1)
    assert s["lex_run_rows"] in (0, 64, 128, 256, 512)
    y1, g1 = solve(q, bq)
    assert torch.equal(y1, y0) and np.array_equal(g1, g0)
