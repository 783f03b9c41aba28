"""GPU parity: every hot-path step through the C ABI against the CPU oracle.

Per-kernel results (SpMV, coloured sweep, restriction, prolongation, the
whole V-cycle) are compared bit for bit: the library disables FP contraction
and sums each row in the oracle's order, so the same IEEE operations happen
on both sides.  CG adds reductions whose summation order differs (tree on the
GPU, sequential in the oracle), so residual histories are compared with the
rule in parity.py: 1e-12 relative plus a noise floor, in units of the
initial residual, that matters only where the residual is made of rounding
noise.
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

HERE = os.path.dirname(os.path.abspath(__file__))


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


def hist_ok(h_gpu, h_ora):
    assert_history_close(h_gpu, h_ora)


DIMS = [(16, 16, 16), (24, 16, 32), (32, 8, 16)]


@pytest.mark.parametrize("dims", DIMS)
def test_sizes_match(mg, dims):
    o = Oracle(*dims, levels=4)
    p = mg.Problem(dims, levels=4)
    for l in range(4):
        assert p.n(l) == o.n(l)
        assert p.nnz(l) == o.nnz(l)


@pytest.mark.parametrize("dims", DIMS)
def test_layout_round_trip(mg, dims):
    p = mg.Problem(dims, levels=4)
    for l in range(4):
        v = dev(inputs.uniform(20 + l, p.n(l)))
        w = p.to_natural(p.to_internal(v, l), l)
        assert torch.equal(v, w)
        assert not torch.equal(v, p.to_internal(v, l)) or p.n(l) <= 8


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("order", [0, 1])
def test_kernels_bitwise_each_level(mg, dims, order):
    o = Oracle(*dims, levels=4, colour_order=order)
    p = mg.Problem(dims, levels=4, colour_order=order)
    for l in range(4):
        n = o.n(l)
        x = inputs.uniform(100 + l, n)
        z0 = inputs.uniform(200 + l, n)
        # SpMV
        np.testing.assert_array_equal(host(p.spmv(dev(x), level=l)), o.spmv(x, level=l))
        # one symmetric coloured sweep from a nonzero z
        np.testing.assert_array_equal(host(p.gs_sweep(dev(x), dev(z0), level=l)), o.sgs(x, z0, level=l))
        # each colour pass on its own (Listing 3), same colour numbering
        for k in range(o.ncolours(l)):
            np.testing.assert_array_equal(host(p.colour_pass(dev(x), dev(z0), k, level=l)),
                                          o.colour_pass(k, x, z0, level=l))
        if l + 1 < 4:
            np.testing.assert_array_equal(host(p.restrict(dev(x), dev(z0), level=l)),
                                          o.restrict(x, z0, level=l))
            zc = inputs.uniform(300 + l, o.n(l + 1))
            np.testing.assert_array_equal(host(p.prolong_add(dev(zc), dev(z0), level=l)),
                                          o.prolong_add(zc, z0, level=l))


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("order", [0, 1])
def test_vcycle_bitwise(mg, dims, order):
    o = Oracle(*dims, levels=4, colour_order=order)
    p = mg.Problem(dims, levels=4, colour_order=order)
    for seed in (1, 2):
        r = inputs.uniform(seed, o.n())
        np.testing.assert_array_equal(host(p.vcycle(dev(r))), o.vcycle(r))


@pytest.mark.parametrize("dims,levels", [((1, 1, 1), 1), ((5, 1, 1), 1), ((1, 7, 1), 1), ((3, 1, 5), 1),
                                         ((2, 9, 1), 1), ((8, 8, 8), 4), ((16, 16, 8), 4)])
@pytest.mark.parametrize("order", [0, 1])
def test_degenerate_grids(mg, dims, levels, order):
    # one point, flat grids (fewer colours: the parity bits of extent-1
    # dimensions are dropped), and hierarchies whose coarsest level is
    # 1x1x1 (8^3) or flat 2x2x1 (16x16x8)
    o = Oracle(*dims, levels=levels, colour_order=order)
    p = mg.Problem(dims, levels=levels, colour_order=order)
    for l in range(levels):
        n = o.n(l)
        x, z0 = inputs.uniform(90 + l, n), inputs.uniform(95 + l, n)
        np.testing.assert_array_equal(host(p.spmv(dev(x), level=l)), o.spmv(x, level=l))
        np.testing.assert_array_equal(host(p.gs_sweep(dev(x), dev(z0), level=l)), o.sgs(x, z0, level=l))
        for k in range(o.ncolours(l)):
            np.testing.assert_array_equal(host(p.colour_pass(dev(x), dev(z0), k, level=l)),
                                          o.colour_pass(k, x, z0, level=l))
    r = inputs.uniform(99, o.n())
    np.testing.assert_array_equal(host(p.vcycle(dev(r))), o.vcycle(r))
    xo, ho, ito, sto = o.pcg(r, max_iters=30, tol=1e-10)
    x, h, its, st = p.solve(dev(r), max_iters=30, tol=1e-10)
    assert st == sto and its[0] == ito
    assert_history_close(h[0, :ito], ho)


def test_rhs_ones(mg):
    o = Oracle(16, 16, 16)
    p = mg.Problem((16, 16, 16))
    b = host(p.make_rhs_ones())
    np.testing.assert_array_equal(b, o.spmv(np.ones(o.n())))
    bi = p.make_rhs_ones(layout=mg.INTERNAL)
    np.testing.assert_array_equal(host(p.to_natural(bi)), b)


@pytest.mark.parametrize("order", [0, 1])
def test_pcg_16cubed_history(mg, order):
    o = Oracle(16, 16, 16, colour_order=order)
    p = mg.Problem((16, 16, 16), colour_order=order)
    b = o.spmv(np.ones(o.n()))
    xo, ho, ito, sto = o.pcg(b, max_iters=50)
    x, h, its, st = p.solve(dev(b), max_iters=50)
    assert st == mg.OK and its[0] == 50 and ito == 50
    hist_ok(h[0], ho)
    xg = host(x)
    assert np.linalg.norm(xg - xo) <= 1e-12 * np.linalg.norm(xo)
    assert np.abs(xg - 1.0).max() < 1e-12


def test_pcg_tolerance_stop_and_status(mg):
    o = Oracle(24, 16, 32)
    p = mg.Problem((24, 16, 32))
    b = inputs.uniform(5, o.n())
    xo, ho, ito, sto = o.pcg(b, max_iters=200, tol=1e-9)
    x, h, its, st = p.solve(dev(b), max_iters=200, tol=1e-9)
    assert st == mg.OK and sto == 0
    assert its[0] == ito
    hist_ok(h[0, :ito], ho)
    assert np.all(h[0, ito:] == 0)
    assert np.linalg.norm(host(x) - xo) <= 1e-12 * np.linalg.norm(xo)
    # not converged within max_iters
    x, h, its, st = p.solve(dev(b), max_iters=3, tol=1e-12)
    assert st == mg.NOT_CONVERGED and its[0] == 3
    # zero right-hand side: zero iterations
    x, h, its, st = p.solve(dev(np.zeros(o.n())), max_iters=10, tol=1e-9)
    assert st == mg.OK and its[0] == 0 and float(host(x).max()) == 0.0
    # breakdown: NaN in b
    bn = b.copy()
    bn[7] = np.nan
    x, h, its, st = p.solve(dev(bn), max_iters=10, tol=0.0)
    assert st == mg.ERR_BREAKDOWN and its[0] == 0


@pytest.mark.parametrize("dims,nrhs", [((24, 16, 32), 1), ((64, 64, 64), 1), ((16, 16, 16), 4)])
def test_iterations_after_convergence_change_nothing(mg, dims, nrhs):
    # A tolerance-driven solve reads the count of finished systems only once
    # a later iteration is queued, so iterations run after the last system
    # converged; with one grid the colour passes store regardless of the
    # flag, and the CG updates and finalizes must leave x, r, p and the
    # scalars of a converged system alone.  The solve must therefore give,
    # bit for bit, the x and history of a fixed-count solve of exactly the
    # iterations it reports.
    n = dims[0] * dims[1] * dims[2]
    p = mg.Problem(dims, nrhs=nrhs)
    b = dev(inputs.uniform(15, n * nrhs))
    for graph in (1, 0):
        p.set_graph_mode(graph)
        x, h, its, st = p.solve(b, max_iters=300, tol=1e-9)
        assert st == mg.OK and len(set(int(k) for k in its)) >= 1
        k = int(max(its))
        xf, hf, itsf, stf = p.solve(b, max_iters=k, tol=0.0)
        if nrhs == 1:
            assert int(itsf[0]) == k
            assert torch.equal(x, xf), f"graph {graph}: x moved after convergence"
            assert np.array_equal(h[0, :k], hf[0, :k])
        else:
            # right-hand sides that converged earlier stop early in the
            # tolerance solve and run on in the fixed-count one: compare the
            # last-converging ones, and the others' histories up to their stop
            last = [v for v in range(nrhs) if int(its[v]) == k]
            # natural layout holds the right-hand sides one after another
            X, XF = host(x).reshape(nrhs, -1), host(xf).reshape(nrhs, -1)
            for v in last:
                assert np.array_equal(X[v], XF[v]), f"graph {graph}, rhs {v}"
            for v in range(nrhs):
                kv = int(its[v])
                assert np.array_equal(h[v, :kv], hf[v, :kv]), f"graph {graph}, rhs {v}"
                assert np.all(h[v, kv:] == 0)


def test_pcg_nonzero_x0(mg):
    o = Oracle(16, 16, 16)
    p = mg.Problem((16, 16, 16))
    b = inputs.uniform(6, o.n())
    x0 = inputs.uniform(7, o.n())
    xo, ho, _, _ = o.pcg(b, x0=x0, max_iters=20)
    x, h, its, st = p.solve(dev(b), x0=dev(x0), max_iters=20)
    hist_ok(h[0], ho)
    assert np.linalg.norm(host(x) - xo) <= 1e-12 * np.linalg.norm(xo)


@pytest.mark.parametrize("nrhs", [1, 4, 16])
def test_graph_and_eager_identical_and_deterministic(mg, nrhs):
    # (4 and 16 right-hand sides: the box-tiled product and the folded
    # partials in the same comparison)
    p = mg.Problem((16, 16, 16), nrhs=nrhs)
    b = p.make_rhs_ones() if nrhs == 1 else dev(inputs.multi_rhs(51, nrhs, 16 ** 3))
    outs = []
    for mode in (1, 1, 0, 1):
        p.set_graph_mode(mode)
        x, h, its, st = p.solve(b, max_iters=30)
        outs.append((host(x), h.copy()))
        # eager work and a sync between graph replays
        torch.cuda.synchronize()
        _ = p.spmv(x)
    for xg, hg in outs[1:]:
        np.testing.assert_array_equal(xg, outs[0][0])
        np.testing.assert_array_equal(hg, outs[0][1])


def test_async_solve_and_result(mg):
    p = mg.Problem((16, 16, 16))
    b = p.make_rhs_ones(layout=mg.INTERNAL)
    x = p.zeros()
    assert p.solve_async(b, x, max_iters=25, layout=mg.INTERNAL) == mg.OK
    h = np.zeros(25)
    its = np.zeros(1, np.int32)
    assert mg.mgpcg_solve_result(p.h, 25, h, its) == mg.OK
    x2, h2, its2, _ = p.solve(p.to_natural(b), max_iters=25)
    np.testing.assert_array_equal(h, h2[0])
    np.testing.assert_array_equal(host(p.to_natural(x)), host(x2))


def test_error_paths(mg):
    p = mg.Problem((16, 16, 16))
    v = p.zeros()
    with pytest.raises(mg.MGPCGError) as e:
        p.spmv(v, level=4)
    assert e.value.status == -1
    with pytest.raises(mg.MGPCGError):
        p.restrict(v, v, level=3)
    with pytest.raises(mg.MGPCGError):
        mg.mgpcg_spmv(p.h, 0, v, v, layout=7)
    with pytest.raises(mg.MGPCGError):
        mg.mgpcg_pcg_solve(p.h, v, v, -1)
    for bad in (-1, 8):
        with pytest.raises(mg.MGPCGError) as e:
            mg.mgpcg_colour_pass(p.h, 0, bad, v, p.zeros())
        assert e.value.status == -1
    with pytest.raises(mg.MGPCGError) as e:
        mg.Problem((12, 16, 16))
    assert e.value.status == -2


# ---------------------------------------------------------------- FP32 V-cycle

@pytest.mark.parametrize("order", [0, 1])
def test_fp32_vcycle_bitwise(mg, order):
    dims = (24, 16, 32)
    o = Oracle(*dims, colour_order=order)
    p = mg.Problem(dims, mg_dtype="fp32", colour_order=order)
    r = inputs.uniform(8, o.n())
    np.testing.assert_array_equal(host(p.vcycle(dev(r))), o.vcycle32(r))
    for l in range(4):
        n = o.n(l)
        rr = inputs.uniform(30 + l, n).astype(np.float32)
        zz = inputs.uniform(40 + l, n).astype(np.float32)
        got = host(p.gs_sweep(dev(rr.astype(np.float64)), dev(zz.astype(np.float64)), level=l))
        np.testing.assert_array_equal(got, o.sgs32(rr, zz, level=l).astype(np.float64))


def test_fp32_pcg_matches_oracle(mg):
    dims = (32, 32, 32)
    o = Oracle(*dims)
    p = mg.Problem(dims, mg_dtype="fp32")
    b = o.spmv(np.ones(o.n())) + inputs.perturbation(3, o.n())
    xo, ho, ito, _ = o.pcg(b, max_iters=200, tol=1e-9, precond=2)
    x, h, its, st = p.solve(dev(b), max_iters=200, tol=1e-9)
    assert st == mg.OK and its[0] == ito
    # The V-cycle itself is bitwise equal (test above), but r is rounded to
    # FP32 at its entry: a last-bit FP64 difference in r (dot-product order)
    # can move an FP32 rounding decision by one FP32 ulp (6e-8), so FP32-MG
    # histories agree at FP32 level, not FP64 level.
    rel = np.abs(h[0, :ito] - ho) / ho
    print("fp32-mg history max relative difference", rel.max())
    assert rel.max() <= 1e-5
    x64, _, it64, _ = o.pcg(b, max_iters=200, tol=1e-9, precond=1)
    # same answer as the FP64-preconditioned solve to the solver tolerance
    assert np.linalg.norm(host(x) - x64) <= 1e-8 * np.linalg.norm(x64)


# -------------------------------------------------------- batched / multi-RHS

@pytest.mark.parametrize("order", [0, 1])
def test_batched_grids(mg, order):
    dims = [(16, 16, 16), (24, 16, 32), (8, 16, 8)]
    p = mg.Problem(dims, levels=4, colour_order=order)
    oras = [Oracle(*d, colour_order=order) for d in dims]
    sizes = [o.n() for o in oras]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    b = inputs.batch_rhs(9, sizes)
    # V-cycle of all grids at once equals each grid's own
    z = host(p.vcycle(dev(b)))
    for g, o in enumerate(oras):
        np.testing.assert_array_equal(z[offs[g]:offs[g + 1]], o.vcycle(b[offs[g]:offs[g + 1]]))
    # coarse levels too
    for l in range(1, 4):
        nl = [o.n(l) for o in oras]
        ol = np.concatenate([[0], np.cumsum(nl)])
        r = inputs.batch_rhs(10 + l, nl)
        zz = inputs.batch_rhs(20 + l, nl)
        got = host(p.gs_sweep(dev(r), dev(zz), level=l))
        for g, o in enumerate(oras):
            np.testing.assert_array_equal(got[ol[g]:ol[g + 1]], o.sgs(r[ol[g]:ol[g + 1]], zz[ol[g]:ol[g + 1]], level=l))
    x, h, its, st = p.solve(dev(b), max_iters=200, tol=1e-9)
    assert st == mg.OK
    xg = host(x)
    for g, o in enumerate(oras):
        xo, ho, ito, _ = o.pcg(b[offs[g]:offs[g + 1]], max_iters=200, tol=1e-9)
        assert its[g] == ito
        hist_ok(h[g, :ito], ho)
        assert np.all(h[g, ito:] == 0)
        np.testing.assert_allclose(xg[offs[g]:offs[g + 1]], xo, rtol=0, atol=1e-12 * np.abs(xo).max())


@pytest.mark.parametrize("order", [0, 1])
def test_fp32_vcycle_batched_and_multi_rhs(mg, order):
    # the FP32 V-cycle on several grids and on 4 and 16 right-hand sides,
    # bit for bit with the oracle's FP32 V-cycle of each grid / rhs
    dims = [(16, 16, 16), (24, 16, 32), (8, 16, 8)]
    sizes = [a * b * c for a, b, c in dims]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    r = inputs.batch_rhs(81, sizes)
    p = mg.Problem(dims, levels=4, mg_dtype="fp32", colour_order=order)
    z = host(p.vcycle(dev(r)))
    for g, d in enumerate(dims):
        o = Oracle(*d, colour_order=order)
        np.testing.assert_array_equal(z[offs[g]:offs[g + 1]], o.vcycle32(r[offs[g]:offs[g + 1]]))
    o = Oracle(16, 16, 16, colour_order=order)
    n = o.n()
    for nrhs in (4, 16):
        B = inputs.multi_rhs(82, nrhs, n)
        pm = mg.Problem((16, 16, 16), nrhs=nrhs, mg_dtype="fp32", colour_order=order)
        Z = host(pm.vcycle(dev(B)))
        for v in range(nrhs):
            np.testing.assert_array_equal(Z[v * n:(v + 1) * n], o.vcycle32(B[v * n:(v + 1) * n]))


@pytest.mark.parametrize("levels,dims", [
    (4, [(16, 16, 16), (24, 16, 32), (8, 16, 8)]),
    # ragged one-level grids: the SpMV table of a grid is padded with empty
    # entries up to a whole number of workgroups
    (1, [(5, 3, 7), (6, 4, 2), (3, 3, 3)]),
])
@pytest.mark.parametrize("nrhs", [4, 16])
def test_batched_multi_rhs(mg, levels, dims, nrhs):
    # several grids with several right-hand sides each: vectors are packed grid
    # after grid, and right-hand side after right-hand side within a grid
    sizes = [a * b * c for a, b, c in dims]
    blocks = [(g, v, inputs.uniform(300 + 20 * g + v, n)) for g, n in enumerate(sizes) for v in range(nrhs)]
    B = np.concatenate([blk for _, _, blk in blocks])
    print(f"batched {dims} levels {levels} x {nrhs} rhs", flush=True)
    p = mg.Problem(dims, levels=levels, nrhs=nrhs)
    Z = host(p.vcycle(dev(B)))
    Y = host(p.spmv(dev(B)))
    x, h, its, st = p.solve(dev(B), max_iters=200, tol=1e-9)
    assert st == mg.OK
    X = host(x)
    oras = [Oracle(*d, levels=levels) for d in dims]
    off = 0
    for g, v, bv in blocks:
        o, n = oras[g], sizes[g]
        np.testing.assert_array_equal(Z[off:off + n], o.vcycle(bv))
        np.testing.assert_array_equal(Y[off:off + n], o.spmv(bv))
        xo, ho, ito, _ = o.pcg(bv, max_iters=200, tol=1e-9)
        sys = g * nrhs + v
        assert its[sys] == ito
        hist_ok(h[sys, :ito], ho)
        np.testing.assert_allclose(X[off:off + n], xo, rtol=0, atol=1e-12 * np.abs(xo).max())
        off += n


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("order", [0, 1])
def test_batched_multi_rhs_vcycle_variants(mg, dtype, order):
    # several grids with 8 right-hand sides each (values staged in LDS), under
    # both colour orders and both V-cycle precisions: every (grid, rhs) block
    # of the V-cycle equals the oracle's, bit for bit
    dims = [(16, 16, 16), (24, 16, 32), (8, 16, 8)]
    nrhs = 8
    sizes = [a * b * c for a, b, c in dims]
    blocks = [(g, v, inputs.uniform(400 + 20 * g + v, n)) for g, n in enumerate(sizes) for v in range(nrhs)]
    B = np.concatenate([blk for _, _, blk in blocks])
    print(f"batched x {nrhs} rhs, {dtype}, order {order}", flush=True)
    p = mg.Problem(dims, levels=4, nrhs=nrhs, mg_dtype=dtype, colour_order=order)
    Z = host(p.vcycle(dev(B)))
    oras = [Oracle(*d, levels=4, colour_order=order) for d in dims]
    off = 0
    for g, v, bv in blocks:
        o, n = oras[g], sizes[g]
        want = o.vcycle32(bv) if dtype == "fp32" else o.vcycle(bv)
        np.testing.assert_array_equal(Z[off:off + n], want)
        off += n


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("nrhs", [2, 4, 8, 16])
def test_multi_rhs(mg, nrhs, order):
    dims = (16, 16, 16)
    o = Oracle(*dims, colour_order=order)
    n = o.n()
    p = mg.Problem(dims, nrhs=nrhs, colour_order=order)
    B = inputs.multi_rhs(41, nrhs, n)
    Z = host(p.vcycle(dev(B)))
    Y = host(p.spmv(dev(B)))
    for v in range(nrhs):
        np.testing.assert_array_equal(Z[v * n:(v + 1) * n], o.vcycle(B[v * n:(v + 1) * n]))
        np.testing.assert_array_equal(Y[v * n:(v + 1) * n], o.spmv(B[v * n:(v + 1) * n]))
    x, h, its, st = p.solve(dev(B), max_iters=100, tol=1e-9)
    assert st == mg.OK
    X = host(x)
    for v in range(nrhs):
        xo, ho, ito, _ = o.pcg(B[v * n:(v + 1) * n], max_iters=100, tol=1e-9)
        assert its[v] == ito
        hist_ok(h[v, :ito], ho)
        np.testing.assert_allclose(X[v * n:(v + 1) * n], xo, rtol=0, atol=1e-12 * np.abs(xo).max())


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("nrhs", [4, 16])
def test_multi_rhs_paired_lanes_both_widths(mg, nrhs, order):
    # From 4 right-hand sides on, a colour-pass lane updates two of them
    # (16-byte accesses) and a workgroup holds twice the rows.  On 32 x 64 x 64
    # every level has several workgroups per colour; the V-cycle must stay
    # bit-exact against the oracle with 64- and 256-thread passes on levels 0
    # and 1, and the solve must match the oracle's history on every
    # right-hand side.
    dims = (32, 64, 64)
    o = Oracle(*dims, colour_order=order)
    n = o.n()
    B = inputs.multi_rhs(43, nrhs, n)
    print(f"paired lanes nrhs={nrhs} order={order}", flush=True)
    p = mg.Problem(dims, levels=4, nrhs=nrhs, colour_order=order)
    zref = {v: o.vcycle(B[v * n:(v + 1) * n]) for v in (0, nrhs - 1)}
    for wide in (0, 1, 3):
        p.set_schedule(wide_levels=wide)
        Z = host(p.vcycle(dev(B)))
        for v, zr in zref.items():
            np.testing.assert_array_equal(Z[v * n:(v + 1) * n], zr, err_msg=f"wide {wide} rhs {v}")
    x, h, its, st = p.solve(dev(B), max_iters=8)
    for v in (0, nrhs - 1):
        xo, ho, ito, _ = o.pcg(B[v * n:(v + 1) * n], max_iters=8)
        hist_ok(h[v, :ito], ho)
    Y = host(p.spmv(dev(B)))
    for v in (0, nrhs - 1):
        np.testing.assert_array_equal(Y[v * n:(v + 1) * n], o.spmv(B[v * n:(v + 1) * n]), err_msg=f"rhs {v}")
    p.check()


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("nrhs", [4, 8, 16])
@pytest.mark.parametrize("dims,levels", [((16, 2, 2), 2), ((48, 6, 10), 2), ((32, 12, 4), 3), ((64, 4, 6), 2),
                                         ((20, 8, 8), 3)])
def test_multi_rhs_box_product(mg, dims, levels, nrhs, order):
    # One grid with R >= 4 and even extents, nx a multiple of the box length
    # (8, 16, 32 fine points at 16, 8, 4 right-hand sides): the CG product
    # stages p on boxes of 2x2 half-lines plus a one-point halo in LDS.  The
    # product must equal the oracle's bit for bit on every right-hand side
    # (boxes at every face and edge, thin extents of 2), and a short solve
    # must follow the oracle's history.  Shapes whose nx is not a multiple
    # ((16, 2, 2) and (48, 6, 10) at 4 rhs, (20, 8, 8) always) take the
    # table-driven product, for contrast.
    o = Oracle(*dims, levels=levels, colour_order=order)
    n = o.n()
    B = inputs.multi_rhs(47, nrhs, n)
    print(f"box product {dims} nrhs={nrhs} order={order}", flush=True)
    p = mg.Problem(dims, levels=levels, nrhs=nrhs, colour_order=order)
    Y = host(p.spmv(dev(B)))
    for v in range(nrhs):
        np.testing.assert_array_equal(Y[v * n:(v + 1) * n], o.spmv(B[v * n:(v + 1) * n]), err_msg=f"rhs {v}")
    x, h, its, st = p.solve(dev(B), max_iters=6)
    for v in (0, nrhs // 2, nrhs - 1):
        xo, ho, ito, _ = o.pcg(B[v * n:(v + 1) * n], max_iters=6)
        hist_ok(h[v, :ito], ho)
    p.check()


# ---------------------------------------------------------------- full size

@pytest.fixture(scope="module")
def p128(mg):
    return mg.Problem((128, 128, 128), levels=4)


def test_128cubed_kernels_bitwise(mg, p128):
    o = Oracle(128, 128, 128)
    x = inputs.uniform(2, o.n())
    np.testing.assert_array_equal(host(p128.spmv(dev(x))), o.spmv(x))
    np.testing.assert_array_equal(host(p128.vcycle(dev(x))), o.vcycle(x))
    z0 = inputs.uniform(3, o.n())
    np.testing.assert_array_equal(host(p128.gs_sweep(dev(x), dev(z0))), o.sgs(x, z0))


def test_128cubed_pcg_history_golden(mg, p128):
    gold = json.load(open(os.path.join(HERE, "golden", "pcg_128cubed_fp64.json")))
    b = p128.make_rhs_ones()
    x, h, its, st = p128.solve(b, max_iters=50)
    assert st == mg.OK and its[0] == 50
    ho = np.array(gold["history"])
    assert ho.min() >= 1e-6  # far above the noise floor: the rule is 1e-12 relative here
    np.testing.assert_allclose(h[0], ho, rtol=1e-12, atol=0)
    xg = host(x)
    idx = np.array(gold["sample_index"])
    np.testing.assert_allclose(xg[idx], np.array(gold["sample_x"]), rtol=1e-12, atol=0)
    assert abs(np.abs(xg - 1.0).max() - gold["max_abs_err"]) <= 1e-12


def test_128cubed_order1_streamed_levels(mg):
    # colour order 1 at full size: level 0 (453 MB of FP64 operator) runs the
    # 256-thread non-temporal builds with the order-1 zero-start masks and the
    # unfused restriction and refinement; the coarse levels do real work
    dims = (128, 128, 128)
    print("128^3 order 1", flush=True)
    o = Oracle(*dims, colour_order=1)
    p = mg.Problem(dims, levels=4, colour_order=1)
    assert p.schedule["wide_levels"] & 1
    r = inputs.uniform(80, o.n())
    np.testing.assert_array_equal(host(p.vcycle(dev(r))), o.vcycle(r))
    for l in range(4):
        n = o.n(l)
        x, z0 = inputs.uniform(81 + l, n), inputs.uniform(85 + l, n)
        np.testing.assert_array_equal(host(p.gs_sweep(dev(x), dev(z0), level=l)), o.sgs(x, z0, level=l))
        if l < 3:
            np.testing.assert_array_equal(host(p.restrict(dev(x), dev(z0), level=l)), o.restrict(x, z0, level=l))
    b = o.spmv(np.ones(o.n()))
    xo, ho, ito, _ = o.pcg(b, max_iters=20)
    x, h, its, st = p.solve(dev(b), max_iters=20)
    assert st == mg.OK and its[0] == 20
    hist_ok(h[0], ho)
    np.testing.assert_allclose(host(x), xo, rtol=0, atol=1e-12 * np.abs(xo).max())


# ------------------------------------------- coarse levels: persistent kernel

@pytest.mark.parametrize("dims", [(16, 16, 16), (24, 16, 32)])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("order", [0, 1])
def test_coarse_persistent_equals_per_pass(mg, dims, dtype, order):
    # Under colour order 0 the restricted residual is ~0 (the coarse levels only
    # add rounding), so order 1 is the case in which a coarse-level mistake
    # would show; both are compared bit for bit with the oracle.
    o = Oracle(*dims, colour_order=order)
    p = mg.Problem(dims, mg_dtype=dtype, colour_order=order)
    r = dev(inputs.uniform(60, o.n()))
    outs = []
    for mode in (0, 1, 0, 1):
        p.set_coarse_mode(mode)
        z = p.vcycle(r)
        assert p.check() == mg.OK
        outs.append(host(z))
    for z in outs[1:]:
        np.testing.assert_array_equal(z, outs[0])
    ref = o.vcycle(host(r)) if dtype == "fp64" else o.vcycle32(host(r))
    np.testing.assert_array_equal(outs[1], ref)
    np.testing.assert_array_equal(outs[0], ref)
    b = p.make_rhs_ones()
    hs = []
    for mode in (1, 0):
        p.set_coarse_mode(mode)
        x, h, its, st = p.solve(b, max_iters=30)
        assert st == mg.OK and p.check() == mg.OK
        hs.append((host(x), h.copy()))
    np.testing.assert_array_equal(hs[0][0], hs[1][0])
    np.testing.assert_array_equal(hs[0][1], hs[1][1])


@pytest.mark.parametrize("order", [0, 1])
def test_coarse_persistent_batched_and_multi_rhs(mg, order, monkeypatch):
    dims = [(16, 16, 16), (24, 16, 32), (8, 16, 8)]
    # the persistent kernel takes several grids with int32 columns only
    monkeypatch.setenv("MGPCG_DELTA_COLS", "0")
    p = mg.Problem(dims, colour_order=order)
    sizes = [a * b * c for a, b, c in dims]
    r = dev(inputs.batch_rhs(61, sizes))
    p.set_coarse_mode(0)
    z0 = host(p.vcycle(r))
    p.set_coarse_mode(1)
    z1 = host(p.vcycle(r))
    assert p.check() == mg.OK
    np.testing.assert_array_equal(z0, z1)
    oras = [Oracle(*d, colour_order=order) for d in dims]
    rr = host(r)
    off = 0
    for o in oras:
        np.testing.assert_array_equal(z1[off:off + o.n()], o.vcycle(rr[off:off + o.n()]))
        off += o.n()
    # 16 right-hand sides: the persistent mode is not used (falls back)
    pm = mg.Problem((16, 16, 16), nrhs=16, colour_order=order)
    B = dev(inputs.multi_rhs(62, 16, 4096))
    pm.set_coarse_mode(0)
    z0 = host(pm.vcycle(B))
    pm.set_coarse_mode(1)
    z1 = host(pm.vcycle(B))
    assert pm.check() == mg.OK
    np.testing.assert_array_equal(z0, z1)


# ---------------- column formats (int32 / int8 deltas / implied by the bases)
# MGPCG_DELTA_COLS caps the format; 24x16x32 has an odd extent on its
# coarsest level (3x2x4), whose deltas are then nonzero, so "2" mixes the
# implied format (finer levels) with int8 deltas (coarsest level)

@pytest.mark.parametrize("dims", [(16, 16, 16), (24, 16, 32)])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_delta_coded_columns_identical(mg, dims, dtype, monkeypatch):
    r = dev(inputs.uniform(70, int(np.prod(dims))))
    outs = []
    for flag in ("0", "1", "2"):
        monkeypatch.setenv("MGPCG_DELTA_COLS", flag)
        p = mg.Problem(dims, mg_dtype=dtype)
        z = host(p.vcycle(r))
        y = host(p.spmv(r))
        x, h, its, st = p.solve(r, max_iters=20)
        outs.append((z, y, host(x), h.copy()))
        p.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            np.testing.assert_array_equal(a, b)


# ------------------------------- single-workgroup tail of the smallest levels

@pytest.mark.parametrize("dims", [(16, 16, 16), (32, 32, 32)])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("order", [0, 1])
def test_tail_equals_per_pass(mg, dims, dtype, order, monkeypatch):
    o = Oracle(*dims, colour_order=order)
    r = inputs.uniform(71, o.n())
    ref = o.vcycle(r) if dtype == "fp64" else o.vcycle32(r)
    outs = []
    for nbytes in ("0", "65536"):
        monkeypatch.setenv("MGPCG_TAIL_BYTES", nbytes)
        p = mg.Problem(dims, mg_dtype=dtype, colour_order=order)
        z = host(p.vcycle(dev(r)))
        np.testing.assert_array_equal(z, ref)
        x, h, its, st = p.solve(dev(r), max_iters=25)
        assert st == mg.OK and p.check() == mg.OK
        outs.append((host(x), h.copy()))
        p.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
