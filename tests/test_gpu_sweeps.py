"""GPU parity with several symmetric sweeps per smoothing step.

Each smoothing step of the V-cycle (the pre- and post-smoothing of Listing 1,
and the coarsest level's) runs `sweeps` symmetric sweeps.  The library fuses the
restriction into the last pre-smoothing sweep, the refinement into the first
post-smoothing sweep and the <r,z> partials into the last one; the oracle
runs the steps one after another.  V-cycles compare bit for bit, PCG
histories with the rule in parity.py.
"""
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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("sweeps", [2, 3])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("dims", [(16, 16, 16), (24, 16, 32)])
def test_vcycle_bitwise(mg, dims, dtype, order, sweeps):
    print(f"sweeps={sweeps} {dims} {dtype} order {order}", flush=True)
    o = Oracle(*dims, levels=4, colour_order=order, sweeps=sweeps)
    p = mg.Problem(dims, levels=4, colour_order=order, mg_dtype=dtype, sweeps=sweeps)
    for seed in (1, 2):
        r = inputs.uniform(seed, o.n())
        ref = o.vcycle(r) if dtype == "fp64" else o.vcycle32(r)
        np.testing.assert_array_equal(host(p.vcycle(dev(r))), ref)


@pytest.mark.parametrize("sweeps", [2, 3])
def test_sequential_vcycle_bitwise(mg, sweeps):
    dims = (16, 8, 24)
    o = Oracle(*dims, levels=4, sweeps=sweeps)
    p = mg.Problem(dims, levels=4, smoother="sequential", sweeps=sweeps)
    r = inputs.uniform(3, o.n())
    np.testing.assert_array_equal(host(p.vcycle(dev(r))), o.vcycle_lex(r))


def test_sequential_batched_two_sweeps(mg):
    dims = [(16, 16, 16), (24, 16, 32), (8, 16, 8)]
    sizes = [a * b * c for a, b, c in dims]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    r = inputs.batch_rhs(83, sizes)
    p = mg.Problem(dims, levels=4, smoother="sequential", sweeps=2)
    z = host(p.vcycle(dev(r)))
    for g, d in enumerate(dims):
        o = Oracle(*d, sweeps=2)
        np.testing.assert_array_equal(z[offs[g]:offs[g + 1]], o.vcycle_lex(r[offs[g]:offs[g + 1]]))


def test_one_sweep_is_the_default(mg):
    dims = (16, 16, 16)
    r = dev(inputs.uniform(4, 16 ** 3))
    a = host(mg.Problem(dims).vcycle(r))
    b = host(mg.Problem(dims, sweeps=1).vcycle(r))
    c = host(mg.Problem(dims, sweeps=0).vcycle(r))
    assert np.array_equal(a, b) and np.array_equal(a, c)


@pytest.mark.parametrize("smoother,precond", [("coloured", 1), ("sequential", 3)])
def test_pcg_matches_oracle(mg, smoother, precond):
    dims = (24, 16, 32)
    o = Oracle(*dims, sweeps=2)
    p = mg.Problem(dims, smoother=smoother, sweeps=2)
    b = inputs.uniform(5, o.n())
    xo, ho, ito, sto = o.pcg(b, max_iters=200, tol=1e-9, precond=precond)
    x, h, its, st = p.solve(dev(b), max_iters=200, tol=1e-9)
    assert st == mg.OK and sto == 0 and its[0] == ito
    assert_history_close(h[0, :ito], ho)
    xg = host(x)
    assert np.linalg.norm(xg - xo) <= 1e-11 * np.linalg.norm(xo)


def test_batched_and_multi_rhs(mg):
    dims = [(16, 16, 16), (24, 16, 32), (8, 16, 8)]
    p = mg.Problem(dims, levels=4, sweeps=2)
    oras = [Oracle(*d, sweeps=2) for d in dims]
    sizes = [o.n() for o in oras]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    b = inputs.batch_rhs(9, sizes)
    z = host(p.vcycle(dev(b)))
    for g, o in enumerate(oras):
        np.testing.assert_array_equal(z[offs[g]:offs[g + 1]], o.vcycle(b[offs[g]:offs[g + 1]]))
    o = Oracle(16, 16, 16, sweeps=3)
    n = o.n()
    p = mg.Problem((16, 16, 16), nrhs=4, sweeps=3)
    B = inputs.multi_rhs(41, 4, n)
    Z = host(p.vcycle(dev(B)))
    for v in range(4):
        np.testing.assert_array_equal(Z[v * n:(v + 1) * n], o.vcycle(B[v * n:(v + 1) * n]))


def test_coarse_mode_falls_back(mg):
    # the persistent coarse kernel runs one sweep per step; with more the
    # library keeps one kernel per pass and the results stay the same
    dims = (32, 32, 32)
    o = Oracle(*dims, sweeps=2)
    p = mg.Problem(dims, sweeps=2)
    p.set_coarse_mode(1)
    r = inputs.uniform(6, o.n())
    np.testing.assert_array_equal(host(p.vcycle(dev(r))), o.vcycle(r))
    b = dev(r)
    x1, h1, _, _ = p.solve(b, max_iters=8)
    p.set_coarse_mode(0)
    x2, h2, _, _ = p.solve(b, max_iters=8)
    assert torch.equal(x1, x2) and np.array_equal(h1, h2)


def test_rejected_counts(mg):
    for bad in (-1, 17):
        with pytest.raises(mg.MGPCGError):
            mg.Problem((16, 16, 16), sweeps=bad)


def _departure(op, x, y):
    """|x'(Oy) - y'(Ox)| / ((|x||Oy| + |y||Ox|) eps), the HPCG-style symmetry
    measure: a few units for an operator symmetric up to rounding."""
    ox, oy = host(op(dev(x))), host(op(dev(y)))
    num = abs(float(np.dot(x, oy)) - float(np.dot(y, ox)))
    return num / ((np.linalg.norm(x) * np.linalg.norm(oy) + np.linalg.norm(y) * np.linalg.norm(ox))
                  * np.finfo(np.float64).eps)


@pytest.mark.parametrize("kw", [{}, {"colour_order": 1}, {"sweeps": 2}, {"smoother": "sequential"},
                                {"smoother": "sequential", "sweeps": 2}])
def test_symmetry_departures(mg, kw):
    # a replacement smoother must keep the preconditioner symmetric
    # (Sec. III-A); a forward-only coloured smoother shows ~3e12 here
    dims = (32, 32, 32)
    x, y = inputs.uniform(91, 32 ** 3), inputs.uniform(92, 32 ** 3)
    p = mg.Problem(dims, **kw)
    assert _departure(p.spmv, x, y) < 10
    assert _departure(p.vcycle, x, y) < 10
