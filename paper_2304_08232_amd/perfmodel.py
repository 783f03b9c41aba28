"""Nominal work model of one MG-PCG iteration (bytes and flops).

The method as written: every pass streams its operands once.  Per pass over
all rows of a level: one directional coloured sweep moves 12 B per nonzero
(8 B value + 4 B int32 column) plus 24 B per row (r read, z read, z write);
a SpMV 12 B per nonzero + 16 B per row; restriction and prolongation 24 B per
coarse row each; zeroing z 8 B per row; a dot product 16 B per row (8 B for
a norm); an axpy 24 B per row.  FP32 V-cycles halve value and vector bytes
inside the V-cycle (8 B per nonzero, 12 B per sweep row).
Flops: sweep 2*nnz + 4*n, SpMV 2*nnz, dot and axpy 2*n each.
"""


def level_sizes(dims, levels):
    """[(n, nnz)] per level for one grid."""
    out = []
    for l in range(levels):
        nx, ny, nz = (d >> l for d in dims)
        out.append((nx * ny * nz, (3 * nx - 2) * (3 * ny - 2) * (3 * nz - 2)))
    return out


def iteration(dims_list, levels=4, mg_dtype="fp64", nrhs=1):
    """(bytes, flops) of one PCG iteration summed over grids; matrix bytes are
    counted once per pass regardless of the number of right-hand sides."""
    vb = 8 if mg_dtype == "fp64" else 4      # V-cycle vector element
    mb = 12 if mg_dtype == "fp64" else 8     # V-cycle bytes per nonzero
    B = F = 0.0
    R = nrhs
    for dims in dims_list:
        sz = level_sizes(dims, levels)
        for l, (n, nnz) in enumerate(sz):
            sweeps = 2 if l == levels - 1 else 4
            B += sweeps * (mb * nnz + 3 * vb * n * R)
            F += sweeps * (2 * nnz + 4 * n) * R
            B += vb * n * R                   # z = 0 at entry
            if l < levels - 1:
                nc = sz[l + 1][0]
                B += mb * nnz + 2 * vb * n * R   # residual SpMV
                F += 2 * nnz * R
                B += 2 * 3 * vb * nc * R         # restriction + prolongation
        n0, nnz0 = sz[0]
        B += 12 * nnz0 + 16 * n0 * R          # CG SpMV (FP64)
        F += 2 * nnz0 * R
        B += (16 + 16 + 8) * n0 * R           # <r,z>, <p,q>, ||r||
        F += 3 * 2 * n0 * R
        B += 3 * 24 * n0 * R                  # p, x, r updates
        F += 3 * 2 * n0 * R
        if mg_dtype == "fp32":
            B += (8 + 4) * n0 * R + (4 + 8) * n0 * R   # casts at V-cycle entry and exit
    return B, F


def sweep_pass_bytes(dims, mg_dtype="fp64"):
    """Average bytes of one colour pass of a directional sweep at level 0."""
    n, nnz = level_sizes(dims, 1)[0]
    mb, vb = (12, 8) if mg_dtype == "fp64" else (8, 4)
    return (mb * nnz + 3 * vb * n) / 8.0


def spmv_bytes(dims):
    """Bytes of one standalone FP64 SpMV y = A x at level 0."""
    n, nnz = level_sizes(dims, 1)[0]
    return 12 * nnz + 16 * n


def sym_sweep_bytes(dims):
    """Bytes of one standalone FP64 symmetric sweep (forward and backward
    directional sweeps) at level 0."""
    n, nnz = level_sizes(dims, 1)[0]
    return 2 * (12 * nnz + 24 * n)


HBM_PEAK_GBS = 8000.0
