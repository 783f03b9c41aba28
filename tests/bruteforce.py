"""Tiny dense brute-force references used to pin the oracle (test-only).

Everything here is built a different way from the oracle: the matrix from the
Chebyshev distance between grid points, the smoother as sequential
Gauss-Seidel (Eq. (1) of the paper) over an explicit visiting order, the
transfers as dense 0/1 matrices, and the preconditioned CG iterate as the
A-norm-optimal point of the Krylov space.  Only for grids of a few hundred
points.
"""
import numpy as np


def coords(nx, ny, nz):
    """(n, 3) integer coordinates in natural order i = ix + nx*(iy + ny*iz)."""
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)


def softplus(t):
    return np.logaddexp(0.0, t)


def dense_stencil(nx, ny, nz, theta=None):
    """27-point operator: -1 between distinct points at Chebyshev distance 1,
    26 (+ softplus(theta)) on the diagonal."""
    c = coords(nx, ny, nz)
    dist = np.abs(c[:, None, :] - c[None, :, :]).max(axis=2)
    A = np.where(dist == 1, -1.0, 0.0)
    d = np.full(len(c), 26.0)
    if theta is not None:
        d = d + softplus(np.asarray(theta, dtype=np.float64))
    A[np.arange(len(c)), np.arange(len(c))] = d
    return A


def parity_colour(nx, ny, nz):
    c = coords(nx, ny, nz)
    return (c[:, 0] & 1) + 2 * (c[:, 1] & 1) + 4 * (c[:, 2] & 1)


def gs_sequential(A, r, z, order):
    """Eq. (1) applied row by row in the given visiting order."""
    z = z.copy()
    for i in order:
        s = A[i] @ z - A[i, i] * z[i]
        z[i] = (r[i] - s) / A[i, i]
    return z


def colour_sorted_order(colour):
    """Rows stably sorted by colour number."""
    return np.argsort(colour, kind="stable")


def sgs_sequential(A, r, z, colour):
    fwd = colour_sorted_order(colour)
    # backward: colours in reverse; within a colour the order does not matter
    # for a proper colouring, so the reversed stable order is used
    z = gs_sequential(A, r, z, fwd)
    return gs_sequential(A, r, z, fwd[::-1])


def injection_matrix(nx, ny, nz):
    """R (n_c x n_f): one 1 per row at the fine point (2jx, 2jy, 2jz)."""
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    cc = coords(cx, cy, cz)
    R = np.zeros((len(cc), nx * ny * nz))
    fine = 2 * cc[:, 0] + nx * (2 * cc[:, 1] + ny * 2 * cc[:, 2])
    R[np.arange(len(cc)), fine] = 1.0
    return R


def vcycle_dense(levels_A, levels_colour, levels_R, r, l=0, nu=1):
    """Brute-force V-cycle from dense pieces; nu symmetric sweeps per smoothing."""
    A = levels_A[l]
    z = np.zeros_like(r)
    for _ in range(nu):
        z = sgs_sequential(A, r, z, levels_colour[l])
    if l == len(levels_A) - 1:
        return z
    R = levels_R[l]
    rc = R @ (r - A @ z)
    zc = vcycle_dense(levels_A, levels_colour, levels_R, rc, l + 1, nu)
    z = z + R.T @ zc
    for _ in range(nu):
        z = sgs_sequential(A, r, z, levels_colour[l])
    return z


def krylov_optimal(A, Minv, b, x0, k):
    """argmin over x in x0 + K_k(Minv A, Minv r0) of ||x - A^{-1} b||_A."""
    r0 = b - A @ x0
    v = Minv @ r0
    basis = []
    for _ in range(k):
        basis.append(v)
        v = Minv @ (A @ v)
    V = np.linalg.qr(np.stack(basis, axis=1))[0]
    y = np.linalg.solve(V.T @ A @ V, V.T @ r0)
    return x0 + V @ y
