"""GPU parity of the sequential smoother against the oracle.

The library runs the sequential symmetric Gauss-Seidel of Eq. (1) wavefront
by wavefront (t = ix + 2 iy + 4 iz); the oracle runs it row by row.  Both
evaluate each update as the same IEEE sequence (off-diagonal sum in ascending
column order, then one subtraction and one division), so sweeps and V-cycles
compare bit for bit.  PCG histories use the rule in parity.py, as for the
coloured smoother.

MGPCG_LEX_RUN_ROWS sets the largest wavefront a single-workgroup run takes:
"0" gives every wavefront a launch of its own, "64" mixes both launch kinds,
"512" puts whole small levels into single-workgroup runs.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2304_08232_amd import inputs
from parity import assert_history_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RUN_ROWS = ["0", "64", "512"]


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


@pytest.mark.parametrize("run_rows", RUN_ROWS)
@pytest.mark.parametrize("dims", [(16, 16, 16), (24, 16, 32), (8, 8, 56), (24, 40, 24)])
def test_sweep_bitwise_each_level(mg, dims, run_rows, monkeypatch):
    # (24, 40, 24) has odd extents at level 3
    monkeypatch.setenv("MGPCG_LEX_RUN_ROWS", run_rows)
    print(f"sequential sweep {dims} run_rows={run_rows}", flush=True)
    o = Oracle(*dims, levels=4)
    p = mg.Problem(dims, levels=4, smoother="sequential")
    for l in range(4):
        n = o.n(l)
        r = inputs.uniform(400 + l, n)
        z0 = inputs.uniform(500 + l, n)
        np.testing.assert_array_equal(host(p.gs_sweep(dev(r), dev(z0), level=l)), o.sgs_lex(r, z0, level=l))
        # from zero, and on the internal layout as well
        zi = host(p.to_natural(p.gs_sweep(p.to_internal(dev(r), l), torch.zeros(n, dtype=torch.float64,
                                                                                 device="cuda"),
                                          level=l, layout=mg.INTERNAL), l))
        np.testing.assert_array_equal(zi, o.sgs_lex(r, np.zeros(n), level=l))


@pytest.mark.parametrize("run_rows", RUN_ROWS)
@pytest.mark.parametrize("dims", [(1, 1, 1), (7, 5, 3), (1, 3, 2), (33, 1, 2), (2, 9, 1)])
def test_sweep_small_and_flat_grids(mg, dims, run_rows, monkeypatch):
    # flat grids leave some wavefront numbers without points
    monkeypatch.setenv("MGPCG_LEX_RUN_ROWS", run_rows)
    print(f"sequential sweep {dims} run_rows={run_rows}", flush=True)
    o = Oracle(*dims, levels=1)
    p = mg.Problem(dims, levels=1, smoother="sequential")
    n = o.n()
    r, z0 = inputs.uniform(31, n), inputs.uniform(32, n)
    np.testing.assert_array_equal(host(p.gs_sweep(dev(r), dev(z0))), o.sgs_lex(r, z0))
    np.testing.assert_array_equal(host(p.vcycle(dev(r))), o.vcycle_lex(r))


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("run_rows", RUN_ROWS)
@pytest.mark.parametrize("dims", [(16, 16, 16), (24, 16, 32)])
def test_vcycle_bitwise(mg, dims, run_rows, order, monkeypatch):
    monkeypatch.setenv("MGPCG_LEX_RUN_ROWS", run_rows)
    print(f"sequential V-cycle {dims} run_rows={run_rows} order={order}", flush=True)
    o = Oracle(*dims, levels=4, colour_order=order)
    p = mg.Problem(dims, levels=4, smoother="sequential", colour_order=order)
    for seed in (1, 2):
        r = inputs.uniform(seed, o.n())
        np.testing.assert_array_equal(host(p.vcycle(dev(r))), o.vcycle_lex(r))


def test_vcycle_with_theta_and_set_theta(mg):
    dims = (16, 8, 24)
    n = dims[0] * dims[1] * dims[2]
    th1 = inputs.uniform(61, n, -4.0, 4.0)
    th2 = inputs.uniform(62, n, -4.0, 4.0)
    p = mg.Problem(dims, levels=4, smoother="sequential", theta=dev(th1))
    r = inputs.uniform(63, n)

    def close(got, ref):
        # softplus is evaluated by the device's exp/log1p and the host's libm:
        # a diagonal can differ in the last bit, so this comparison is not
        # bitwise; a stale operator would be off by ~1e-2
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())

    v1 = Oracle(*dims, levels=4, theta=th1).vcycle_lex(r)
    close(host(p.vcycle(dev(r))), v1)
    # the wavefront-major values follow a new coefficient field
    p.set_theta(dev(th2))
    v2 = Oracle(*dims, levels=4, theta=th2).vcycle_lex(r)
    assert np.abs(v2 - v1).max() > 1e-4 * np.abs(v2).max()
    close(host(p.vcycle(dev(r))), v2)


def test_pcg_matches_oracle(mg):
    dims = (24, 16, 32)
    o = Oracle(*dims)
    p = mg.Problem(dims, smoother="sequential")
    b = inputs.uniform(5, o.n())
    xo, ho, ito, sto = o.pcg(b, max_iters=200, tol=1e-9, precond=3)
    x, h, its, st = p.solve(dev(b), max_iters=200, tol=1e-9)
    assert st == mg.OK and sto == 0 and its[0] == ito
    assert_history_close(h[0, :ito], ho)
    xg = host(x)
    assert np.linalg.norm(xg - xo) <= 1e-11 * np.linalg.norm(xo)


def test_graph_and_eager_identical(mg):
    dims = (16, 16, 16)
    p = mg.Problem(dims, smoother="sequential")
    b = dev(inputs.uniform(6, p.n()))
    x1, h1, _, _ = p.solve(b, max_iters=12)
    p.set_graph_mode(0)
    x2, h2, _, _ = p.solve(b, max_iters=12)
    p.set_graph_mode(1)
    x3, h3, _, _ = p.solve(b, max_iters=12)
    assert torch.equal(x1, x2) and torch.equal(x1, x3)
    assert np.array_equal(h1, h2) and np.array_equal(h1, h3)


def test_batched_grids(mg):
    dims = [(16, 16, 16), (24, 16, 32), (8, 16, 8)]
    p = mg.Problem(dims, levels=4, smoother="sequential")
    oras = [Oracle(*d) for d in dims]
    sizes = [o.n() for o in oras]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    b = inputs.batch_rhs(9, sizes)
    z = host(p.vcycle(dev(b)))
    for g, o in enumerate(oras):
        np.testing.assert_array_equal(z[offs[g]:offs[g + 1]], o.vcycle_lex(b[offs[g]:offs[g + 1]]))
    x, h, its, st = p.solve(dev(b), max_iters=200, tol=1e-9)
    assert st == mg.OK
    xg = host(x)
    for g, o in enumerate(oras):
        xo, ho, ito, _ = o.pcg(b[offs[g]:offs[g + 1]], max_iters=200, tol=1e-9, precond=3)
        assert its[g] == ito
        assert_history_close(h[g, :ito], ho)
        np.testing.assert_allclose(xg[offs[g]:offs[g + 1]], xo, rtol=0, atol=1e-11 * np.abs(xo).max())


def test_rejected_configurations(mg):
    with pytest.raises(mg.MGPCGError):
        mg.Problem((16, 16, 16), smoother="sequential", mg_dtype="fp32")
    with pytest.raises(mg.MGPCGError):
        mg.Problem((16, 16, 16), smoother="sequential", nrhs=2)


def test_128cubed_sweep_vcycle_and_first_iterations(mg):
    o = Oracle(128, 128, 128)
    p = mg.Problem((128, 128, 128), levels=4, smoother="sequential")
    print("sequential smoother 128^3", flush=True)
    r = inputs.uniform(2, o.n())
    z0 = inputs.uniform(3, o.n())
    np.testing.assert_array_equal(host(p.gs_sweep(dev(r), dev(z0))), o.sgs_lex(r, z0))
    np.testing.assert_array_equal(host(p.vcycle(dev(r))), o.vcycle_lex(r))
    b = o.spmv(np.ones(o.n()))
    xo, ho, ito, _ = o.pcg(b, max_iters=4, precond=3)
    x, h, its, st = p.solve(dev(b), max_iters=4)
    assert st == mg.OK and its[0] == ito == 4
    assert_history_close(h[0], ho)
