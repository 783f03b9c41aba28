"""Pins of the CPU oracle against what the problem and the mathematics fix.

None of these compares the oracle with itself: closed forms, invariants,
special cases that reduce to textbook algorithms, and brute force from the
dense references in bruteforce.py.
"""
import numpy as np
import pytest

import bruteforce as bf
from oracle import Oracle

SMALL_DIMS = [(2, 2, 2), (3, 3, 3), (4, 4, 4), (6, 5, 4), (7, 4, 5), (5, 3, 2)]


# ---------------------------------------------------------------- matrix (Sec. II-A/B)

@pytest.mark.parametrize("dims", SMALL_DIMS + [(16, 16, 16), (24, 32, 48)])
def test_nnz_closed_form(dims):
    nx, ny, nz = dims
    o = Oracle(nx, ny, nz, levels=1)
    assert o.nnz() == (3 * nx - 2) * (3 * ny - 2) * (3 * nz - 2)


def test_nnz_per_level_16cubed():
    o = Oracle(16, 16, 16, levels=4)
    assert [o.n(l) for l in range(4)] == [4096, 512, 64, 8]
    assert [o.nnz(l) for l in range(4)] == [97336, 10648, 1000, 64]


@pytest.mark.parametrize("dims", SMALL_DIMS)
def test_matrix_equals_chebyshev_stencil(dims):
    o = Oracle(*dims, levels=1)
    assert np.array_equal(o.dense(), bf.dense_stencil(*dims))


@pytest.mark.parametrize("dims", [(6, 5, 4), (8, 8, 8)])
def test_matrix_symmetric_rowsums_rhs(dims):
    o = Oracle(*dims, levels=1)
    rp, col, val = o.crs()
    A = o.dense()
    assert np.array_equal(A, A.T)
    # columns ascending within every row (CRS order used for the sums)
    for i in range(o.n()):
        assert np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0)
    # b = A*1 gives b_i = 27 - nnz_i exactly; interior rows sum to zero
    b = o.spmv(np.ones(o.n()))
    nnz_row = np.diff(rp)
    assert np.array_equal(b, 27.0 - nnz_row)
    assert np.all(b[nnz_row == 27] == 0.0)


@pytest.mark.parametrize("dims", [(4, 4, 4), (6, 6, 6), (6, 5, 4)])
def test_matrix_spd(dims):
    A = Oracle(*dims, levels=1).dense()
    np.linalg.cholesky(A)  # raises if not positive definite
    assert np.linalg.eigvalsh(A).min() > 0


def test_theta_diagonal():
    rng = np.random.default_rng(0)
    th = rng.normal(0, 0.5, 4 * 4 * 4)
    o = Oracle(4, 4, 4, levels=3, theta=th)
    np.testing.assert_allclose(o.dense(0), bf.dense_stencil(4, 4, 4, th), rtol=1e-15, atol=0)
    # coarse level: theta injected at (2jx, 2jy, 2jz)
    R = bf.injection_matrix(4, 4, 4)
    np.testing.assert_allclose(o.dense(1), bf.dense_stencil(2, 2, 2, R @ th), rtol=1e-15, atol=0)
    # large |theta| stays finite and correct
    th2 = np.array([800.0, -800.0, 0.0, 30.0, -30.0, 1e-3, 5.0, -5.0])
    o2 = Oracle(2, 2, 2, levels=1, theta=th2)
    d = np.diag(o2.dense())
    np.testing.assert_allclose(d, 26.0 + np.array([800.0, 0.0, np.log(2.0), 30.0 + np.log1p(np.exp(-30.0)),
                                                   np.exp(-30.0), np.log1p(np.exp(1e-3)),
                                                   5.0 + np.log1p(np.exp(-5.0)), np.log1p(np.exp(-5.0))]),
                               rtol=1e-15)


def test_invalid_problems_rejected():
    with pytest.raises(ValueError):
        Oracle(6, 6, 6, levels=3)  # 6 not divisible by 4
    with pytest.raises(ValueError):
        Oracle(0, 4, 4, levels=1)


# ------------------------------------------------------------ colouring (Sec. III-A)

def greedy_bruteforce(A):
    n = A.shape[0]
    col = -np.ones(n, int)
    for i in range(n):
        used = {col[j] for j in np.nonzero(A[i])[0] if j < i}
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


@pytest.mark.parametrize("dims", SMALL_DIMS + [(8, 6, 4)])
def test_greedy_equals_parity_code(dims):
    o = Oracle(*dims, levels=1)
    c = o.colours()
    assert np.array_equal(c, greedy_bruteforce(bf.dense_stencil(*dims)))
    assert np.array_equal(c, bf.parity_colour(*dims))
    assert o.ncolours() == 8


@pytest.mark.parametrize("dims", [(4, 4, 4), (16, 16, 16), (6, 5, 4)])
def test_colouring_proper_and_balanced(dims):
    o = Oracle(*dims, levels=1)
    rp, col, _ = o.crs()
    c = o.colours()
    rows = np.repeat(np.arange(o.n()), np.diff(rp))
    off = rows != col
    assert not np.any(c[rows[off]] == c[col[off]])
    if all(d % 2 == 0 for d in dims):
        assert np.all(np.bincount(c, minlength=8) == o.n() // 8)


def test_colour_order_reversed():
    o0 = Oracle(4, 4, 4, levels=1, colour_order=0)
    o1 = Oracle(4, 4, 4, levels=1, colour_order=1)
    assert np.array_equal(o1.colours(), 7 - o0.colours())


@pytest.mark.parametrize("dims,nc", [((4, 4, 1), 4), ((4, 1, 1), 2), ((1, 1, 1), 1), ((1, 3, 4), 4)])
def test_colouring_flat_grids(dims, nc):
    o = Oracle(*dims, levels=1)
    c = o.colours()
    assert o.ncolours() == nc
    assert np.array_equal(c, greedy_bruteforce(bf.dense_stencil(*dims)))


# ------------------------------------------------------- smoother (Eq. (1), Listings 2-3)

@pytest.mark.parametrize("dims", [(4, 4, 4), (6, 5, 4), (3, 3, 3)])
@pytest.mark.parametrize("order", [0, 1])
def test_coloured_sweep_equals_sequential_gs(dims, order):
    rng = np.random.default_rng(1)
    o = Oracle(*dims, levels=1, colour_order=order)
    A = o.dense()
    n = o.n()
    r = rng.uniform(-1, 1, n)
    z0 = rng.uniform(-1, 1, n)
    c = o.colours()
    # forward pass only: colour passes 0..7 == sequential GS over rows sorted by colour
    zf = z0.copy()
    for k in range(o.ncolours()):
        zf = o.colour_pass(k, r, zf)
    zbf = bf.gs_sequential(A, r, z0, bf.colour_sorted_order(c))
    np.testing.assert_allclose(zf, zbf, rtol=1e-13, atol=1e-15)
    # full symmetric sweep
    np.testing.assert_allclose(o.sgs(r, z0), bf.sgs_sequential(A, r, z0, c), rtol=1e-13, atol=1e-15)


def test_forward_sweep_on_2cubed_is_lexicographic_gs():
    # on 2x2x2 the colour number equals the row index, so the coloured forward
    # pass is textbook lexicographic Gauss-Seidel
    rng = np.random.default_rng(2)
    o = Oracle(2, 2, 2, levels=1)
    A = o.dense()
    r, z0 = rng.uniform(-1, 1, 8), rng.uniform(-1, 1, 8)
    z = z0.copy()
    for k in range(8):
        z = o.colour_pass(k, r, z)
    L = np.tril(A)
    U = A - L
    np.testing.assert_allclose(z, np.linalg.solve(L, r - U @ z0), rtol=1e-14)


def test_sweep_fixed_point():
    rng = np.random.default_rng(3)
    o = Oracle(6, 5, 4, levels=1)
    A = o.dense()
    zs = rng.uniform(-1, 1, o.n())
    r = A @ zs
    np.testing.assert_allclose(o.sgs(r, zs), zs, rtol=0, atol=1e-14)


# ----------------------------------------------------------- transfers (Sec. II-F, III-B)

def test_injection_map_and_adjointness():
    rng = np.random.default_rng(4)
    o = Oracle(8, 6, 4, levels=2)
    R = bf.injection_matrix(8, 6, 4)
    f2c = o.f2c(0)
    assert np.array_equal(R[np.arange(R.shape[0]), f2c], np.ones(R.shape[0]))
    np.testing.assert_array_equal(R @ R.T, np.eye(R.shape[0]))
    # restriction of (r - A z) by the oracle equals R (r - A z)
    A = o.dense()
    r, z = rng.uniform(-1, 1, o.n()), rng.uniform(-1, 1, o.n())
    np.testing.assert_allclose(o.restrict(r, z), R @ (r - A @ z), rtol=1e-15, atol=1e-15)
    # refinement is the transpose: <R u, v> = <u, R^T v> exactly (pure copies)
    u, v = rng.uniform(-1, 1, o.n()), rng.uniform(-1, 1, o.n(1))
    pz = o.prolong_add(v, np.zeros(o.n()))
    assert np.array_equal(pz, R.T @ v)
    assert Oracle.dot(R @ u, v) == Oracle.dot(u[f2c], v)


# ------------------------------------------------------------ V-cycle (Listing 1)

def _dense_hierarchy(o):
    As = [o.dense(l) for l in range(o.levels)]
    cs = [o.colours(l) for l in range(o.levels)]
    Rs = [bf.injection_matrix(*o.level_dims(l)) for l in range(o.levels - 1)]
    return As, cs, Rs


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("dims,levels", [((4, 4, 4), 3), ((8, 8, 4), 3), ((8, 8, 8), 4)])
def test_vcycle_equals_dense_bruteforce(dims, levels, order):
    rng = np.random.default_rng(5)
    o = Oracle(*dims, levels=levels, colour_order=order)
    As, cs, Rs = _dense_hierarchy(o)
    for _ in range(3):
        r = rng.uniform(-1, 1, o.n())
        np.testing.assert_allclose(o.vcycle(r), bf.vcycle_dense(As, cs, Rs, r), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("order", [0, 1])
def test_vcycle_linear_symmetric_positive(order):
    rng = np.random.default_rng(6)
    o = Oracle(16, 16, 16, levels=4, colour_order=order)
    u, v = rng.uniform(-1, 1, o.n()), rng.uniform(-1, 1, o.n())
    Mu, Mv = o.vcycle(u), o.vcycle(v)
    np.testing.assert_allclose(o.vcycle(2.0 * u + 3.0 * v), 2.0 * Mu + 3.0 * Mv, rtol=1e-12, atol=1e-14)
    # the symmetry test a replacement smoother must pass (Sec. III-A)
    a, b = u @ Mv, v @ Mu
    assert abs(a - b) <= 1e-14 * abs(a)
    assert u @ Mu > 0 and v @ Mv > 0


def test_restricted_residual_vanishes_under_literal_order():
    # Greedy colour 0 is the set of all-even points, i.e. exactly the
    # injection points, and the backward pass ends on it, so every injected
    # equation is solved exactly by the pre-smoother: r_c = 0 up to rounding.
    rng = np.random.default_rng(7)
    o0 = Oracle(16, 16, 16, levels=4, colour_order=0)
    o1 = Oracle(16, 16, 16, levels=4, colour_order=1)
    for lvl in range(3):
        n = o0.n(lvl)
        r = rng.uniform(-1, 1, n)
        z0 = o0.sgs(r, np.zeros(n), level=lvl)
        rc0 = o0.restrict(r, z0, level=lvl)
        assert np.linalg.norm(rc0) <= 1e-14 * np.linalg.norm(r)
        z1 = o1.sgs(r, np.zeros(n), level=lvl)
        rc1 = o1.restrict(r, z1, level=lvl)
        assert np.linalg.norm(rc1) >= 1e-3 * np.linalg.norm(r[o1.f2c(lvl)])


# ------------------------------------ sequential smoother (Sec. II-E, Eq. (1))

LEX_DIMS = [(2, 2, 2), (5, 3, 2), (6, 5, 4), (7, 1, 3), (1, 1, 1)]


@pytest.mark.parametrize("dims", LEX_DIMS)
def test_lex_sweep_equals_sequential_gs(dims):
    rng = np.random.default_rng(21)
    n = dims[0] * dims[1] * dims[2]
    theta = rng.normal(0, 2, n)
    o = Oracle(*dims, levels=1, theta=theta)
    A = bf.dense_stencil(*dims, theta=theta)
    r, z0 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    order = np.arange(n)
    ref = bf.gs_sequential(A, r, bf.gs_sequential(A, r, z0, order), order[::-1])
    np.testing.assert_allclose(o.sgs_lex(r, z0), ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("dims", [(5, 3, 2), (6, 5, 4)])
def test_lex_sweep_from_zero_is_the_sgs_splitting(dims):
    # from z = 0 the two sweeps apply M^{-1} with M = (D + L) D^{-1} (D + U),
    # L and U the strict triangles of A in natural order
    rng = np.random.default_rng(22)
    o = Oracle(*dims, levels=1)
    A = o.dense()
    D = np.diag(np.diag(A))
    M = (D + np.tril(A, -1)) @ np.linalg.inv(D) @ (D + np.triu(A, 1))
    r = rng.uniform(-1, 1, o.n())
    np.testing.assert_allclose(o.sgs_lex(r, np.zeros(o.n())), np.linalg.solve(M, r), rtol=1e-12, atol=1e-14)


def test_lex_sweep_fixed_point_and_energy_decrease():
    rng = np.random.default_rng(23)
    o = Oracle(6, 5, 4, levels=1)
    A = o.dense()
    zs = rng.uniform(-1, 1, o.n())
    r = A @ zs
    np.testing.assert_allclose(o.sgs_lex(r, zs), zs, rtol=0, atol=1e-14)
    # Gauss-Seidel on an SPD matrix strictly reduces the error in the A-norm
    z = rng.uniform(-1, 1, o.n())
    for _ in range(3):
        e0 = z - zs
        z = o.sgs_lex(r, z)
        e1 = z - zs
        assert e1 @ A @ e1 < e0 @ A @ e0


@pytest.mark.parametrize("dims,levels", [((4, 4, 4), 3), ((8, 8, 4), 3), ((8, 8, 8), 4)])
def test_lex_vcycle_equals_dense_bruteforce(dims, levels):
    # one colour holding every row in natural order is exactly the sequential
    # smoother in the brute-force V-cycle
    rng = np.random.default_rng(24)
    o = Oracle(*dims, levels=levels)
    As, _, Rs = _dense_hierarchy(o)
    cs = [np.zeros(o.n(l), dtype=np.int64) for l in range(levels)]
    for _ in range(3):
        r = rng.uniform(-1, 1, o.n())
        np.testing.assert_allclose(o.vcycle_lex(r), bf.vcycle_dense(As, cs, Rs, r), rtol=1e-12, atol=1e-14)


def test_lex_vcycle_linear_symmetric_positive():
    rng = np.random.default_rng(25)
    o = Oracle(16, 16, 16, levels=4)
    u, v = rng.uniform(-1, 1, o.n()), rng.uniform(-1, 1, o.n())
    Mu, Mv = o.vcycle_lex(u), o.vcycle_lex(v)
    np.testing.assert_allclose(o.vcycle_lex(2.0 * u + 3.0 * v), 2.0 * Mu + 3.0 * Mv, rtol=1e-12, atol=1e-14)
    a, b = u @ Mv, v @ Mu
    assert abs(a - b) <= 1e-14 * abs(a)
    assert u @ Mu > 0 and v @ Mv > 0


def test_lex_pcg_krylov_optimal_and_fewer_iterations():
    rng = np.random.default_rng(26)
    o = Oracle(4, 4, 4, levels=3)
    A = o.dense()
    n = o.n()
    Minv = np.stack([o.vcycle_lex(e) for e in np.eye(n)], axis=1)
    b, x0 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    for k in range(1, 5):
        xk, _, it, st = o.pcg(b, x0=x0, max_iters=k, precond=3)
        assert it == k and st == 0
        np.testing.assert_allclose(xk, bf.krylov_optimal(A, Minv, b, x0, k), rtol=1e-9, atol=1e-11)
    # Sec. III-A: the coloured smoother needs more iterations than the
    # sequential one it replaces
    o = Oracle(32, 32, 32, levels=4)
    b = rng.uniform(0, 1, o.n())
    _, _, it_lex, st_lex = o.pcg(b, max_iters=100, tol=1e-9, precond=3)
    _, _, it_col, st_col = o.pcg(b, max_iters=100, tol=1e-9, precond=1)
    assert st_lex == 0 and st_col == 0 and it_lex < it_col


# ------------------------------------ several smoother sweeps (Listing 1, Sec. V)

@pytest.mark.parametrize("nu", [2, 3])
@pytest.mark.parametrize("order,lex", [(0, False), (1, False), (0, True)])
def test_sweeps_vcycle_equals_dense_bruteforce(nu, order, lex):
    rng = np.random.default_rng(27)
    o = Oracle(8, 8, 4, levels=3, colour_order=order, sweeps=nu)
    As, cs, Rs = _dense_hierarchy(o)
    if lex:
        cs = [np.zeros(o.n(l), dtype=np.int64) for l in range(o.levels)]
    r = rng.uniform(-1, 1, o.n())
    got = o.vcycle_lex(r) if lex else o.vcycle(r)
    np.testing.assert_allclose(got, bf.vcycle_dense(As, cs, Rs, r, nu=nu), rtol=1e-12, atol=1e-14)


def test_sweeps_one_level_is_the_truncated_neumann_series():
    # one level: nu sweeps from z = 0 give sum_{k<nu} (I - B A)^k B r, with B
    # the one-sweep operator (its columns are sweeps of unit vectors)
    rng = np.random.default_rng(28)
    o1 = Oracle(6, 5, 4, levels=1)
    A = o1.dense()
    n = o1.n()
    B = np.stack([o1.vcycle(e) for e in np.eye(n)], axis=1)
    r = rng.uniform(-1, 1, n)
    E = np.eye(n) - B @ A
    for nu in (2, 4):
        ref = sum(np.linalg.matrix_power(E, k) @ B @ r for k in range(nu))
        np.testing.assert_allclose(Oracle(6, 5, 4, levels=1, sweeps=nu).vcycle(r), ref, rtol=1e-11, atol=1e-13)
    # many sweeps converge to the solution
    np.testing.assert_allclose(Oracle(6, 5, 4, levels=1, sweeps=60).vcycle(r), np.linalg.solve(A, r),
                               rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("lex", [False, True])
def test_sweeps_vcycle_symmetric_and_fewer_iterations(lex):
    rng = np.random.default_rng(29)
    o = Oracle(16, 16, 16, levels=4, sweeps=2)
    vc = o.vcycle_lex if lex else o.vcycle
    u, v = rng.uniform(-1, 1, o.n()), rng.uniform(-1, 1, o.n())
    a, b = u @ vc(v), v @ vc(u)
    assert abs(a - b) <= 1e-14 * abs(a) and u @ vc(u) > 0
    # Sec. V: several smoother runs may improve convergence
    b = rng.uniform(0, 1, 32 ** 3)
    its = []
    for nu in (1, 2, 3):
        _, _, it, st = Oracle(32, 32, 32, levels=4, sweeps=nu).pcg(b, max_iters=100, tol=1e-9,
                                                                    precond=3 if lex else 1)
        assert st == 0
        its.append(it)
    assert its[0] > its[1] >= its[2]


def test_sweeps_fp32_close_to_fp64_and_invalid():
    rng = np.random.default_rng(30)
    o = Oracle(16, 16, 16, levels=4, sweeps=2)
    r = rng.uniform(-1, 1, o.n())
    z64 = o.vcycle(r)
    assert np.linalg.norm(o.vcycle32(r) - z64) <= 1e-5 * np.linalg.norm(z64)
    with pytest.raises(ValueError):
        Oracle(4, 4, 4, levels=2, sweeps=0)


# ----------------------------------------------------------------- PCG (Sec. II-C)

@pytest.mark.parametrize("precond", [0, 1])
@pytest.mark.parametrize("order", [0, 1])
def test_pcg_iterates_are_krylov_optimal(precond, order):
    rng = np.random.default_rng(8)
    o = Oracle(4, 4, 4, levels=3, colour_order=order)
    A = o.dense()
    n = o.n()
    Minv = np.eye(n) if precond == 0 else np.stack([o.vcycle(e) for e in np.eye(n)], axis=1)
    b = rng.uniform(-1, 1, n)
    x0 = rng.uniform(-1, 1, n)
    for k in range(1, 6):
        xk, hist, it, st = o.pcg(b, x0=x0, max_iters=k, precond=precond)
        assert it == k and st == 0
        xopt = bf.krylov_optimal(A, Minv, b, x0, k)
        np.testing.assert_allclose(xk, xopt, rtol=1e-9, atol=1e-11)
        # the recursive residual history equals the true residual here
        np.testing.assert_allclose(hist[-1], np.linalg.norm(b - A @ xk) / np.linalg.norm(b - A @ x0),
                                   rtol=1e-8, atol=1e-14)


def test_pcg_converges_to_ones_and_error_monotone():
    o = Oracle(8, 8, 8, levels=4)
    A = o.dense()
    b = o.spmv(np.ones(o.n()))
    prev = np.inf
    for k in range(1, 12):
        xk, _, _, _ = o.pcg(b, max_iters=k)
        e = xk - 1.0
        ea = np.sqrt(e @ A @ e)
        assert ea <= prev * (1 + 1e-12)
        prev = ea
    x, hist, it, st = o.pcg(b, max_iters=200, tol=1e-13)
    assert st == 0 and hist[-1] <= 1e-13
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-11)
    np.testing.assert_allclose(x, 1.0, rtol=0, atol=1e-11)


def test_pcg_status_codes():
    o = Oracle(4, 4, 4, levels=3)
    b = o.spmv(np.ones(o.n()))
    _, hist, it, st = o.pcg(b, max_iters=3, tol=1e-30)
    assert st == 1 and it == 3 and hist.size == 3
    bn = b.copy()
    bn[3] = np.nan
    _, _, it, st = o.pcg(bn, max_iters=5)
    assert st == -5 and it == 0
    _, hist, it, st = o.pcg(np.zeros(o.n()), max_iters=5)
    assert st == 0 and it == 0


# --------------------------------------------------------------- FP32 V-cycle

def test_fp32_vcycle_close_to_fp64():
    rng = np.random.default_rng(9)
    o = Oracle(16, 16, 16, levels=4, colour_order=1)
    r = rng.uniform(-1, 1, o.n())
    z64 = o.vcycle(r)
    z32 = o.vcycle32(r)
    err = np.abs(z32 - z64).max() / np.abs(z64).max()
    assert 1e-9 < err < 1e-5  # genuinely single precision, and close
    # the FP32 sweep equals the dense sequential GS carried out in float32
    o2 = Oracle(4, 4, 4, levels=1)
    A32 = o2.dense().astype(np.float32)
    rr = rng.uniform(-1, 1, 64).astype(np.float32)
    zz = o2.sgs32(rr, np.zeros(64, np.float32))
    ref = bf.sgs_sequential(A32.astype(np.float64), rr.astype(np.float64), np.zeros(64), o2.colours())
    np.testing.assert_allclose(zz, ref, rtol=1e-5, atol=1e-7)


# The V-cycle is held bit for bit by the GPU tests (FP64 and FP32), so its
# arithmetic is pinned bit for bit here: against a brute force that visits
# rows one at a time (sequential Gauss-Seidel in colour-stable order, which
# equals the coloured pass because no two rows of a colour are coupled),
# reads the rows of a dense matrix, and rounds every operation to the working
# precision (numpy scalars of that type).  The update is the coloured form of
# Sec. III-A, the whole-row sum with the diagonal term put back (reading D6).
# A mistake that widens a step of the FP32 path (a double accumulator, a
# double residual, FP64 operator values), or that uses another form of the
# update, moves last bits and fails these.

def _bf_rows(A, dt):
    """Nonzero columns (ascending) and values, rounded to dt, of each dense row."""
    Ad = A.astype(dt)
    rows = []
    for i in range(Ad.shape[0]):
        cols = np.nonzero(Ad[i])[0]
        rows.append((cols, Ad[i, cols]))
    return rows, np.diag(Ad).copy()


def _bf_row_dot(cols, vals, z):
    dt = z.dtype.type
    acc = dt(0.0)
    for j, a in zip(cols, vals):
        acc = dt(acc + dt(a * z[j]))
    return acc


def _bf_gs_visit(rows, d, r, z, order):
    dt = z.dtype.type
    z = z.copy()
    for i in order:
        cols, vals = rows[i]
        s = _bf_row_dot(cols, vals, z)
        z[i] = dt(dt(dt(r[i] - s) + dt(z[i] * d[i])) / d[i])
    return z


def _bf_sgs(rows, d, colour, r, z):
    fwd = bf.colour_sorted_order(colour)
    return _bf_gs_visit(rows, d, r, _bf_gs_visit(rows, d, r, z, fwd), fwd[::-1])


def _bf_vcycle(hier, r, l=0):
    rows, d, colour, inj = hier[l]
    z = _bf_sgs(rows, d, colour, r, np.zeros_like(r))
    if l == len(hier) - 1:
        return z
    f = np.array([_bf_row_dot(c, v, z) for c, v in rows], dtype=r.dtype)
    rc = (r - f)[inj]
    zc = _bf_vcycle(hier, rc, l + 1)
    z = z.copy()
    z[inj] = z[inj] + zc
    return _bf_sgs(rows, d, colour, r, z)


def _bf_hierarchy(o, dt):
    hier = []
    for l in range(o.levels):
        rows, d = _bf_rows(o.dense(l), dt)
        inj = bf.injection_matrix(*o.level_dims(l)).argmax(axis=1) if l + 1 < o.levels else None
        hier.append((rows, d, o.colours(l), inj))
    return hier


@pytest.mark.parametrize("dims,theta", [((4, 4, 4), False), ((6, 5, 4), False), ((4, 4, 4), True)])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_sweep_bitexact_scalar_bruteforce(dims, theta, order, dt):
    rng = np.random.default_rng(60)
    n = dims[0] * dims[1] * dims[2]
    th = rng.normal(0, 0.5, n) if theta else None
    o = Oracle(*dims, levels=1, colour_order=order, theta=th)
    rows, d = _bf_rows(o.dense(), dt)
    r = rng.uniform(-1, 1, n).astype(dt)
    z0 = rng.uniform(-1, 1, n).astype(dt)
    ref = _bf_sgs(rows, d, o.colours(), r, z0)
    assert ref.dtype == dt
    if dt == np.float32:
        np.testing.assert_array_equal(o.sgs32(r, z0), ref)
        # genuinely single precision: the FP64 sweep differs
        assert not np.array_equal(o.sgs(r.astype(np.float64), z0.astype(np.float64)), ref.astype(np.float64))
    else:
        np.testing.assert_array_equal(o.sgs(r, z0), ref)


@pytest.mark.parametrize("dims,levels", [((4, 4, 4), 3), ((8, 8, 8), 4), ((8, 4, 4), 3)])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_vcycle_bitexact_scalar_bruteforce(dims, levels, order, dt):
    rng = np.random.default_rng(61)
    o = Oracle(*dims, levels=levels, colour_order=order)
    hier = _bf_hierarchy(o, dt)
    for _ in range(2):
        r = rng.uniform(-1, 1, o.n())
        ref = _bf_vcycle(hier, r.astype(dt))  # FP32: r rounded to nearest at entry
        got = o.vcycle32(r) if dt == np.float32 else o.vcycle(r)
        np.testing.assert_array_equal(got, ref.astype(np.float64))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_vcycle_bitexact_with_theta(dt):
    rng = np.random.default_rng(62)
    th = rng.normal(0, 0.5, 64)
    o = Oracle(4, 4, 4, levels=3, theta=th)
    r = rng.uniform(-1, 1, 64)
    ref = _bf_vcycle(_bf_hierarchy(o, dt), r.astype(dt))
    got = o.vcycle32(r) if dt == np.float32 else o.vcycle(r)
    np.testing.assert_array_equal(got, ref.astype(np.float64))


def test_fp32_pcg_reaches_tolerance():
    o = Oracle(16, 16, 16, levels=4)
    b = o.spmv(np.ones(o.n()))
    _, h64, it64, _ = o.pcg(b, max_iters=100, tol=1e-9, precond=1)
    _, h32, it32, st = o.pcg(b, max_iters=100, tol=1e-9, precond=2)
    assert st == 0 and h32[-1] <= 1e-9
    assert abs(it32 - it64) <= 2


# ---------------------------------------------------- inner product (Sec. II-C)
#
# Reading taken for the inner products of CG: their value is the exact sum
# of the products, which the oracle approaches by accumulating in the x87
# extended format (64-bit significand) and rounding once.  These pin that
# claim against exact arithmetic, on inputs where a plain left-to-right
# double sum fails.

def test_dot_exact_on_integer_cancellation():
    # integers of at most 26 bits: every product is exact in double, and with
    # every partial sum below 2^63 (checked below with exact integers) every
    # partial sum is exact in a 64-bit significand, so the result must be the
    # exact sum rounded once.  Terms cancel in shuffled pairs, and the
    # partial sums reach far past 2^53, where double addition rounds.
    import math
    rng = np.random.default_rng(70)
    m = 3000
    a1 = rng.integers(1 << 22, 1 << 26, m) * rng.choice([-1, 1], m)
    b1 = rng.integers(1 << 22, 1 << 26, m)
    a = np.concatenate([a1, -a1])
    b = np.concatenate([b1, b1 + rng.integers(-3, 4, m)])
    perm = rng.permutation(2 * m)
    a, b = a[perm], b[perm]
    prods = [int(x) * int(y) for x, y in zip(a, b)]
    partial, exact = 0, 0
    for t in prods:
        exact += t
        partial = max(partial, abs(exact))
    assert partial < 2 ** 63 and partial > 2 ** 56
    af, bf_ = a.astype(np.float64), b.astype(np.float64)
    assert math.fsum(af * bf_) == float(exact)  # products exact, fsum correctly rounded
    assert Oracle.dot(af, bf_) == float(exact)
    naive = 0.0
    for x, y in zip(af, bf_):
        naive += x * y
    assert naive != float(exact)  # a plain double sum gets it wrong


def test_dot_two_million_terms_against_fsum():
    # the size of the 128^3 problem's vectors; the reference is the correctly
    # rounded exact dot product: each product split exactly into its rounded
    # value and its error (Dekker's product with Veltkamp splitting), then
    # summed by math.fsum
    import math
    rng = np.random.default_rng(71)
    n = 1 << 21
    a, b = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)

    def split(x):
        c = 134217729.0 * x  # 2^27 + 1
        hi = c - (c - x)
        return hi, x - hi

    p = a * b
    ah, al = split(a)
    bh, bl = split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    ref = math.fsum(np.concatenate([p, e]))
    got = Oracle.dot(a, b)
    naive = float(np.cumsum(p)[-1])  # left to right in double
    assert abs(got - ref) <= 2.0 ** -52 * abs(ref)
    assert abs(naive - ref) > 16 * 2.0 ** -52 * abs(ref)


# ------------------------------------------------------- differentiable solve

def test_theta_gradient_matches_dense_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(10)
    n = 64
    theta = rng.normal(0, 0.5, n)
    b = rng.uniform(-1, 1, n)
    xt = rng.uniform(-1, 1, n)
    o = Oracle(4, 4, 4, levels=3, theta=theta)
    x, _, _, st = o.pcg(b, max_iters=200, tol=1e-14)
    assert st == 0
    lam, _, _, st = o.pcg(x - xt, max_iters=200, tol=1e-14)
    g = Oracle.theta_grad(lam, x, theta)
    # dense reference: autograd through a direct solve
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    A0 = torch.tensor(bf.dense_stencil(4, 4, 4), dtype=torch.float64)
    A = A0 + torch.diag(torch.nn.functional.softplus(th))
    xs = torch.linalg.solve(A, torch.tensor(b, dtype=torch.float64))
    loss = 0.5 * ((xs - torch.tensor(xt, dtype=torch.float64)) ** 2).sum()
    loss.backward()
    np.testing.assert_allclose(g, th.grad.numpy(), rtol=1e-9, atol=1e-13)


def test_theta_gradient_matches_finite_differences():
    rng = np.random.default_rng(11)
    n = 8 * 8 * 8
    theta = rng.normal(0, 0.5, n)
    b = rng.uniform(-1, 1, n)
    xt = rng.uniform(-1, 1, n)

    def loss(th):
        o = Oracle(8, 8, 8, levels=4, theta=th)
        x, _, _, st = o.pcg(b, max_iters=300, tol=1e-14)
        assert st == 0
        return 0.5 * np.sum((x - xt) ** 2), x

    _, x = loss(theta)
    o = Oracle(8, 8, 8, levels=4, theta=theta)
    lam, _, _, _ = o.pcg(x - xt, max_iters=300, tol=1e-14)
    g = Oracle.theta_grad(lam, x, theta)
    # central differences with h = 1e-4: truncation O(h^2) and cancellation
    # eps*|L|/h (|L| ~ 1e2) are both below 1e-9 in absolute terms here
    h = 1e-4
    for i in [0, 7, 100, 273, 511]:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (loss(tp)[0] - loss(tm)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-9 + 1e-6 * abs(g[i])
