/*
 * oracle.c -- plain sequential FP64 CPU reference for MG-preconditioned CG on
 * the 27-point stencil.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
 * benchmark's CPU-baseline leg.  The GPU library never uses it, and it uses
 * nothing of the GPU library.
 *
 * Each function names the passage of arXiv 2304.08232 it follows.  Where the
 * paper is silent the reading taken is stated next to the code.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/*
 * Two builds come from this one file.  Without OpenMP it is the canonical
 * sequential checker.  With -fopenmp (a timing mode only: the CPU baseline
 * the benchmark reports) the loops over independent rows -- the rows of one
 * colour, the rows of a product, the elements of a vector update -- are
 * split statically over the threads, and inner products are summed over
 * fixed per-thread chunks, so that a run is deterministic for a given
 * thread count.  Sequential parts (the V-cycle recursion, the sequential
 * smoother of Eq. (1)) stay sequential.
 */

/* ------------------------------------------------------------------ utils */

static void *xcalloc(size_t n, size_t sz) {
    void *p = calloc(n ? n : 1, sz);
    return p;
}

/* softplus(t) = log(1 + e^t), written so that it neither overflows for large t
 * nor loses the tail for very negative t. */
static double softplus(double t) {
    return (t > 0 ? t : 0.0) + log1p(exp(-fabs(t)));
}

/* logistic function, the derivative of softplus */
static double logistic(double t) {
    return 1.0 / (1.0 + exp(-t));
}

/* Inner product (Sec. II-C).  Its definition is the exact sum; a left to
 * right FP64 sum over millions of terms can be off by ~1e-13 relative, which
 * CG amplifies past a 1e-12 comparison bar, so the terms are accumulated in
 * the x87 extended format (64-bit significand) and rounded once at the end. */
double ora_dot(int64_t n, const double *a, const double *b) {
#ifdef _OPENMP
    /* timing mode: one contiguous chunk per thread, chunk sums added in
     * thread order */
    int nt = omp_get_max_threads();
    if (nt > 1 && n >= 4096) {
        long double part[256];
        if (nt > 256) nt = 256;
#pragma omp parallel num_threads(nt)
        {
            int t = omp_get_thread_num(), T = omp_get_num_threads();
            int64_t lo = n * t / T, hi = n * (t + 1) / T;
            long double s = 0.0L;
            for (int64_t i = lo; i < hi; ++i) s += (long double)a[i] * (long double)b[i];
            part[t] = s;
            if (t == 0)
                for (int u = T; u < nt; ++u) part[u] = 0.0L;
        }
        long double s = 0.0L;
        for (int t = 0; t < nt; ++t) s += part[t];
        return (double)s;
    }
#endif
    long double s = 0.0L;
    for (int64_t i = 0; i < n; ++i) s += (long double)a[i] * (long double)b[i];
    return (double)s;
}

/* threads the loops of this build run on (1 for the sequential checker) */
int ora_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------- problem generation */

/*
 * Sec. II-A/B: the HPCG problem is a heat-diffusion operator on an
 * nx*ny*nz grid; each point couples to itself and to every in-grid point of
 * its 3x3x3 neighbourhood (8 to 27 nonzeros per row).  Values: -1 off the
 * diagonal, 26 on it (the HPCG operator), plus softplus(theta_i) when a
 * coefficient field is given.  Columns are emitted with dz outermost, then dy,
 * then dx, which is ascending natural order.
 */
static int build_level(ora_level *L, int nx, int ny, int nz, const double *theta) {
    memset(L, 0, sizeof(*L));
    L->nx = nx; L->ny = ny; L->nz = nz;
    int64_t n = (int64_t)nx * ny * nz;
    L->n = n;
    /* count */
    L->rowptr = (int64_t *)xcalloc((size_t)n + 1, sizeof(int64_t));
    if (!L->rowptr) return -1;
    int64_t nnz = 0;
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                int64_t i = ix + (int64_t)nx * (iy + (int64_t)ny * iz);
                int cnt = 0;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int jx = ix + dx, jy = iy + dy, jz = iz + dz;
                            if (jx < 0 || jx >= nx || jy < 0 || jy >= ny || jz < 0 || jz >= nz) continue;
                            ++cnt;
                        }
                L->rowptr[i + 1] = cnt;
                nnz += cnt;
            }
    for (int64_t i = 0; i < n; ++i) L->rowptr[i + 1] += L->rowptr[i];
    L->nnz = nnz;
    L->col = (int32_t *)xcalloc((size_t)nnz, sizeof(int32_t));
    L->val = (double *)xcalloc((size_t)nnz, sizeof(double));
    L->val32 = (float *)xcalloc((size_t)nnz, sizeof(float));
    L->diag = (double *)xcalloc((size_t)n, sizeof(double));
    L->diag32 = (float *)xcalloc((size_t)n, sizeof(float));
    if (!L->col || !L->val || !L->val32 || !L->diag || !L->diag32) return -1;
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                int64_t i = ix + (int64_t)nx * (iy + (int64_t)ny * iz);
                int64_t e = L->rowptr[i];
                double d = 26.0;
                if (theta) d += softplus(theta[i]);
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int jx = ix + dx, jy = iy + dy, jz = iz + dz;
                            if (jx < 0 || jx >= nx || jy < 0 || jy >= ny || jz < 0 || jz >= nz) continue;
                            int64_t j = jx + (int64_t)nx * (jy + (int64_t)ny * jz);
                            L->col[e] = (int32_t)j;
                            L->val[e] = (j == i) ? d : -1.0;
                            ++e;
                        }
                L->diag[i] = d;
            }
    for (int64_t e = 0; e < nnz; ++e) L->val32[e] = (float)L->val[e];
    for (int64_t i = 0; i < n; ++i) L->diag32[i] = (float)L->diag[i];
    return 0;
}

/*
 * Sec. III-A: greedy colouring that tracks only direct (i,j) dependencies:
 * rows are visited in ascending order and each takes the smallest colour not
 * already held by one of its (previously coloured) neighbours.  The paper
 * gives neither the visiting order nor the numbering; ascending row order and
 * first-fit numbering are the readings taken here.  colour_order = 1 reverses
 * the numbering (c -> ncolours-1-c), which changes the order in which the
 * colour classes are swept.
 */
static int colour_level(ora_level *L, int colour_order) {
    int64_t n = L->n;
    L->colour = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    if (!L->colour) return -1;
    int ncol = 0;
    for (int64_t i = 0; i < n; ++i) {
        int used[28] = {0};
        for (int64_t e = L->rowptr[i]; e < L->rowptr[i + 1]; ++e) {
            int64_t j = L->col[e];
            if (j < i) used[L->colour[j]] = 1;
        }
        int c = 0;
        while (used[c]) ++c;
        L->colour[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    if (colour_order == 1)
        for (int64_t i = 0; i < n; ++i) L->colour[i] = ncol - 1 - L->colour[i];
    L->ncolours = ncol;
    L->cstart = (int64_t *)xcalloc((size_t)ncol + 1, sizeof(int64_t));
    L->clist = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
    if (!L->cstart || !L->clist) return -1;
    for (int64_t i = 0; i < n; ++i) L->cstart[L->colour[i] + 1]++;
    for (int c = 0; c < ncol; ++c) L->cstart[c + 1] += L->cstart[c];
    int64_t *fill = (int64_t *)xcalloc((size_t)ncol, sizeof(int64_t));
    if (!fill) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int c = L->colour[i];
        L->clist[L->cstart[c] + fill[c]++] = i;
    }
    free(fill);
    return 0;
}

/*
 * Sec. II-F: straight injection.  Coarse point (jx,jy,jz) takes the value of
 * the fine point at the lowest coordinates of its octet, (2jx,2jy,2jz).
 */
static int transfer_map(ora_level *F, const ora_level *C) {
    F->f2c = (int64_t *)xcalloc((size_t)C->n, sizeof(int64_t));
    if (!F->f2c) return -1;
    for (int jz = 0; jz < C->nz; ++jz)
        for (int jy = 0; jy < C->ny; ++jy)
            for (int jx = 0; jx < C->nx; ++jx) {
                int64_t j = jx + (int64_t)C->nx * (jy + (int64_t)C->ny * jz);
                F->f2c[j] = 2 * jx + (int64_t)F->nx * (2 * jy + (int64_t)F->ny * 2 * jz);
            }
    return 0;
}

static void free_level(ora_level *L) {
    free(L->rowptr); free(L->col); free(L->val); free(L->val32);
    free(L->diag); free(L->diag32); free(L->colour); free(L->cstart);
    free(L->clist); free(L->f2c);
    memset(L, 0, sizeof(*L));
}

void ora_destroy(ora_hier *h) {
    if (!h) return;
    for (int l = 0; l < h->levels; ++l) free_level(&h->lev[l]);
    free(h);
}

/*
 * Sec. II-D and II-F: the hierarchy halves every dimension per level; each
 * level carries its own operator (the same stencil rebuilt on the coarse grid:
 * the paper stores mg_level.A per level without saying how it is formed, and
 * rediscretisation is the reading taken here).  With a coefficient field the
 * coarse level takes theta at the injection point.
 */
ora_hier *ora_create(int nx, int ny, int nz, int levels, int colour_order,
                     const double *theta) {
    if (nx < 1 || ny < 1 || nz < 1 || levels < 1 || levels > ORA_MAX_LEVELS) return NULL;
    if (colour_order != 0 && colour_order != 1) return NULL;
    int div = 1 << (levels - 1);
    if (nx % div || ny % div || nz % div) return NULL;
    ora_hier *h = (ora_hier *)xcalloc(1, sizeof(ora_hier));
    if (!h) return NULL;
    h->levels = levels;
    h->colour_order = colour_order;
    h->sweeps = 1;
    double *th = NULL;
    if (theta) {
        int64_t n0 = (int64_t)nx * ny * nz;
        th = (double *)malloc((size_t)n0 * sizeof(double));
        if (!th) { free(h); return NULL; }
        memcpy(th, theta, (size_t)n0 * sizeof(double));
    }
    for (int l = 0; l < levels; ++l) {
        int lx = nx >> l, ly = ny >> l, lz = nz >> l;
        if (build_level(&h->lev[l], lx, ly, lz, th) || colour_level(&h->lev[l], colour_order)) {
            free(th);
            h->levels = l + 1;
            ora_destroy(h);
            return NULL;
        }
        if (l + 1 < levels) {
            /* coarse theta by injection */
            if (th) {
                int cx = lx >> 1, cy = ly >> 1, cz = lz >> 1;
                for (int jz = 0; jz < cz; ++jz)
                    for (int jy = 0; jy < cy; ++jy)
                        for (int jx = 0; jx < cx; ++jx)
                            th[jx + (int64_t)cx * (jy + (int64_t)cy * jz)] =
                                th[2 * jx + (int64_t)lx * (2 * jy + (int64_t)ly * 2 * jz)];
            }
        }
    }
    free(th);
    for (int l = 0; l + 1 < levels; ++l)
        if (transfer_map(&h->lev[l], &h->lev[l + 1])) { ora_destroy(h); return NULL; }
    return h;
}

int64_t ora_n(const ora_hier *h, int level) { return h->lev[level].n; }
int64_t ora_nnz(const ora_hier *h, int level) { return h->lev[level].nnz; }
int ora_ncolours(const ora_hier *h, int level) { return h->lev[level].ncolours; }

void ora_get_crs(const ora_hier *h, int level, int64_t *rowptr, int32_t *col, double *val) {
    const ora_level *L = &h->lev[level];
    memcpy(rowptr, L->rowptr, (size_t)(L->n + 1) * sizeof(int64_t));
    memcpy(col, L->col, (size_t)L->nnz * sizeof(int32_t));
    memcpy(val, L->val, (size_t)L->nnz * sizeof(double));
}

void ora_get_colours(const ora_hier *h, int level, int32_t *colour) {
    const ora_level *L = &h->lev[level];
    memcpy(colour, L->colour, (size_t)L->n * sizeof(int32_t));
}

void ora_get_f2c(const ora_hier *h, int level, int64_t *f2c) {
    const ora_level *L = &h->lev[level];
    const ora_level *C = &h->lev[level + 1];
    memcpy(f2c, L->f2c, (size_t)C->n * sizeof(int64_t));
}

/* ------------------------------------------------------------ FP64 kernels */

/* Sec. II-C: y = A x, each row summed in CRS order. */
void ora_spmv(const ora_hier *h, int level, const double *x, double *y) {
    const ora_level *L = &h->lev[level];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < L->n; ++i) {
        double s = 0.0;
        for (int64_t e = L->rowptr[i]; e < L->rowptr[i + 1]; ++e) s += L->val[e] * x[L->col[e]];
        y[i] = s;
    }
}

/* (A z)_i over the stored row in ascending column order, diagonal included */
static double row_product(const ora_level *L, int64_t i, const double *z) {
    double acc = 0.0;
    for (int64_t e = L->rowptr[i]; e < L->rowptr[i + 1]; ++e) acc += L->val[e] * z[L->col[e]];
    return acc;
}

/*
 * Sec. III-A with Eq. (1): the colour class k of the coloured Gauss-Seidel
 * smoother.  Each row i of the class solves its own equation of A z = r for
 * z_i, every other unknown held at its value from before the class is
 * visited.  Eq. (1) sums the off-diagonal terms; the coloured form of
 * Sec. III-A sums the whole stored row and puts the diagonal term back,
 *     z_i <- (r_i - (A z)_i + a_ii z_i) / a_ii,
 * equal to Eq. (1) in exact arithmetic, and the form whose rounding is
 * fixed here (left to right, one true division).  The new values of the
 * class are collected first and stored afterwards, so no row of the class
 * reads another row's new value (the class has no internal couplings when
 * the colouring is proper, which the tests pin separately).
 */
void ora_colour_pass(const ora_hier *h, int level, int k, const double *r, double *z) {
    const ora_level *L = &h->lev[level];
    int64_t first = L->cstart[k], count = L->cstart[k + 1] - first;
    double *znew = (double *)xcalloc((size_t)count, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        int64_t i = L->clist[first + t];
        double aii = L->diag[i];
        znew[t] = (r[i] - row_product(L, i, z) + z[i] * aii) / aii;
    }
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) z[L->clist[first + t]] = znew[t];
    free(znew);
}

/*
 * Sec. II-E / III-A: symmetric smoother = forward pass over colours
 * 0..c-1, then the backward pass over colours c-1..0 (the paper lists only
 * the forward pass; the backward pass with colours reversed is the reading
 * taken here, mirroring the index reversal of the sequential backward sweep).
 */
void ora_sgs(const ora_hier *h, int level, const double *r, double *z) {
    int c = h->lev[level].ncolours;
    for (int k = 0; k < c; ++k) ora_colour_pass(h, level, k, r, z);
    for (int k = c - 1; k >= 0; --k) ora_colour_pass(h, level, k, r, z);
}

/* Listing 1 (residual and restriction): f = A z, then rc = inject(r - f). */
void ora_restrict(const ora_hier *h, int level, const double *r, const double *z, double *rc) {
    const ora_level *L = &h->lev[level];
    const ora_level *C = &h->lev[level + 1];
    double *f = (double *)xcalloc((size_t)L->n, sizeof(double));
    ora_spmv(h, level, z, f);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < C->n; ++j) {
        int64_t i = L->f2c[j];
        rc[j] = r[i] - f[i];
    }
    free(f);
}

/* Sec. II-F: refinement puts the coarse values at the injection points and
 * zeros elsewhere; Listing 1 adds the result to z. */
void ora_prolong_add(const ora_hier *h, int level, const double *zc, double *z) {
    const ora_level *L = &h->lev[level];
    const ora_level *C = &h->lev[level + 1];
    for (int64_t j = 0; j < C->n; ++j) z[L->f2c[j]] += zc[j];
}

/*
 * Sec. II-D, Listing 1: z = MG(level, r) starting from z = 0.  One symmetric
 * smoothing pass before and after the coarse correction; on the coarsest
 * level only the pre-smoothing pass runs.
 */
/*
 * Sec. II-E, Eq. (1): the sequential symmetric Gauss-Seidel smoother that the
 * coloured one stands in for.  The forward sweep solves equation i for z_i
 * in increasing natural index, each update seeing every z_j already updated
 * in this sweep; the backward sweep does the same in decreasing index.  The
 * sum of Eq. (1) runs over the off-diagonal entries of row i in ascending
 * column order.
 */
static void gs_row(const ora_level *L, int64_t i, const double *r, double *z) {
    double acc = 0.0;
    for (int64_t e = L->rowptr[i]; e < L->rowptr[i + 1]; ++e)
        if (L->col[e] != i) acc += L->val[e] * z[L->col[e]];
    z[i] = (r[i] - acc) / L->diag[i];
}

void ora_sgs_lex(const ora_hier *h, int level, const double *r, double *z) {
    const ora_level *L = &h->lev[level];
    for (int64_t i = 0; i < L->n; ++i) gs_row(L, i, r, z);
    for (int64_t i = L->n - 1; i >= 0; --i) gs_row(L, i, r, z);
}

/*
 * The smoother of Listing 1 (pre- and post-smoothing): h->sweeps symmetric sweeps
 * in a row (Sec. V notes that several runs may help convergence; one is the
 * default), coloured or sequential.
 */
static void smooth(const ora_hier *h, int level, const double *r, double *z, int lex) {
    for (int k = 0; k < h->sweeps; ++k) {
        if (lex) ora_sgs_lex(h, level, r, z); else ora_sgs(h, level, r, z);
    }
}

int ora_set_sweeps(ora_hier *h, int sweeps) {
    if (sweeps < 1) return -1;
    h->sweeps = sweeps;
    return 0;
}

/* Listing 1 with the smoother chosen by `lex` (0: coloured, 1: sequential). */
static void vcycle_with(const ora_hier *h, int level, const double *r, double *z, int lex) {
    const ora_level *L = &h->lev[level];
    memset(z, 0, (size_t)L->n * sizeof(double));
    smooth(h, level, r, z, lex);
    if (level == h->levels - 1) return;
    const ora_level *C = &h->lev[level + 1];
    double *rc = (double *)xcalloc((size_t)C->n, sizeof(double));
    double *zc = (double *)xcalloc((size_t)C->n, sizeof(double));
    ora_restrict(h, level, r, z, rc);
    vcycle_with(h, level + 1, rc, zc, lex);
    ora_prolong_add(h, level, zc, z);
    smooth(h, level, r, z, lex);
    free(rc);
    free(zc);
}

void ora_vcycle(const ora_hier *h, int level, const double *r, double *z) {
    vcycle_with(h, level, r, z, 0);
}

void ora_vcycle_lex(const ora_hier *h, int level, const double *r, double *z) {
    vcycle_with(h, level, r, z, 1);
}

/* ------------------------------------------------------------ FP32 kernels */
/* The same steps as above in single precision, for the FP32 V-cycle. */

static void spmv32(const ora_level *L, const float *x, float *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < L->n; ++i) {
        float s = 0.0f;
        for (int64_t e = L->rowptr[i]; e < L->rowptr[i + 1]; ++e) s += L->val32[e] * x[L->col[e]];
        y[i] = s;
    }
}

static float row_product32(const ora_level *L, int64_t i, const float *z) {
    float acc = 0.0f;
    for (int64_t e = L->rowptr[i]; e < L->rowptr[i + 1]; ++e) acc += L->val32[e] * z[L->col[e]];
    return acc;
}

/* ora_colour_pass in single precision: FP32 values, sums and division */
static void colour_pass32(const ora_level *L, int k, const float *r, float *z) {
    int64_t first = L->cstart[k], count = L->cstart[k + 1] - first;
    float *znew = (float *)xcalloc((size_t)count, sizeof(float));
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        int64_t i = L->clist[first + t];
        float aii = L->diag32[i];
        znew[t] = (r[i] - row_product32(L, i, z) + z[i] * aii) / aii;
    }
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) z[L->clist[first + t]] = znew[t];
    free(znew);
}

void ora_sgs32(const ora_hier *h, int level, const float *r, float *z) {
    const ora_level *L = &h->lev[level];
    for (int k = 0; k < L->ncolours; ++k) colour_pass32(L, k, r, z);
    for (int k = L->ncolours - 1; k >= 0; --k) colour_pass32(L, k, r, z);
}

static void vcycle32_level(const ora_hier *h, int level, const float *r, float *z) {
    const ora_level *L = &h->lev[level];
    memset(z, 0, (size_t)L->n * sizeof(float));
    for (int k = 0; k < h->sweeps; ++k) ora_sgs32(h, level, r, z);
    if (level == h->levels - 1) return;
    const ora_level *C = &h->lev[level + 1];
    float *f = (float *)xcalloc((size_t)L->n, sizeof(float));
    float *rc = (float *)xcalloc((size_t)C->n, sizeof(float));
    float *zc = (float *)xcalloc((size_t)C->n, sizeof(float));
    spmv32(L, z, f);
    for (int64_t j = 0; j < C->n; ++j) rc[j] = r[L->f2c[j]] - f[L->f2c[j]];
    vcycle32_level(h, level + 1, rc, zc);
    for (int64_t j = 0; j < C->n; ++j) z[L->f2c[j]] += zc[j];
    for (int k = 0; k < h->sweeps; ++k) ora_sgs32(h, level, r, z);
    free(f);
    free(rc);
    free(zc);
}

void ora_vcycle32(const ora_hier *h, const double *r, double *z) {
    const ora_level *L = &h->lev[0];
    float *r32 = (float *)xcalloc((size_t)L->n, sizeof(float));
    float *z32 = (float *)xcalloc((size_t)L->n, sizeof(float));
    for (int64_t i = 0; i < L->n; ++i) r32[i] = (float)r[i];
    vcycle32_level(h, 0, r32, z32);
    for (int64_t i = 0; i < L->n; ++i) z[i] = (double)z32[i];
    free(r32);
    free(z32);
}

/* -------------------------------------------------------------------- PCG */

/*
 * Sec. II-C: preconditioned conjugate gradient.  The paper defers the exact
 * recurrences to its CG reference; the standard PCG with
 * beta = <r_k,z_k>/<r_{k-1},z_{k-1}> is the reading taken here.  The stopping
 * test uses the norm of the recursively updated residual relative to the
 * initial residual.
 */
int ora_pcg(const ora_hier *h, const double *b, double *x, int max_iters,
            double tol, int precond, double *history, int *iters) {
    const ora_level *L = &h->lev[0];
    int64_t n = L->n;
    double *r = (double *)xcalloc((size_t)n, sizeof(double));
    double *z = (double *)xcalloc((size_t)n, sizeof(double));
    double *p = (double *)xcalloc((size_t)n, sizeof(double));
    double *q = (double *)xcalloc((size_t)n, sizeof(double));
    int status = 0, k = 0;
    ora_spmv(h, 0, x, q);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    double nr0 = sqrt(ora_dot(n, r, r));
    double rho_old = 0.0;
    if (nr0 == 0.0) goto done;
    for (k = 1; k <= max_iters; ++k) {
        if (precond == 1) ora_vcycle(h, 0, r, z);
        else if (precond == 2) ora_vcycle32(h, r, z);
        else if (precond == 3) ora_vcycle_lex(h, 0, r, z);
        else memcpy(z, r, (size_t)n * sizeof(double));
        double rho = ora_dot(n, r, z);
        if (k == 1) {
            memcpy(p, z, (size_t)n * sizeof(double));
        } else {
            double beta = rho / rho_old;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
        rho_old = rho;
        ora_spmv(h, 0, p, q);
        double pq = ora_dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = -5; --k; break; }
        double alpha = rho / pq;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        double rel = sqrt(ora_dot(n, r, r)) / nr0;
        if (history) history[k - 1] = rel;
        if (tol > 0.0 && rel <= tol) break;
    }
    if (k > max_iters) {
        k = max_iters;
        if (tol > 0.0) status = 1;
    }
done:
    if (iters) *iters = k;
    free(r); free(z); free(p); free(q);
    return status;
}

/*
 * Differentiable solve: x = A(theta)^{-1} b with d_i = 26 + softplus(theta_i).
 * dA/dtheta_i has the single entry softplus'(theta_i) at (i,i), so with the
 * adjoint lambda = A^{-T} dL/dx (A is symmetric) the chain rule gives
 * dL/dtheta_i = -lambda_i * x_i * logistic(theta_i).
 */
void ora_theta_grad(int64_t n, const double *lambda, const double *x,
                    const double *theta, double *grad) {
    for (int64_t i = 0; i < n; ++i) grad[i] = -lambda[i] * x[i] * logistic(theta[i]);
}
