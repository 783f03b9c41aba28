/*
 * oracle.h -- CPU reference ("oracle") for multigrid-preconditioned conjugate
 * gradient on the 27-point HPCG stencil.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain, sequential FP64
 * statement of what the method computes.  It exists so that tests, the smoke
 * check and the benchmark's CPU-baseline leg can compare the GPU library
 * against it.  The GPU product path never links, loads or calls it, and it
 * shares no code, header, table or helper with the GPU path.
 *
 * Paper: "Effective implementation of the High Performance Conjugate Gradient
 * benchmark on GraphBLAS" (arXiv 2304.08232).
 *   - problem and inputs: Sec. II-A/B
 *   - preconditioned CG: Sec. II-C
 *   - multigrid V-cycle: Sec. II-D, Listing 1
 *   - Gauss-Seidel update: Sec. II-E, Eq. (1); coloured (RBGS) form:
 *     Sec. III-A, Listings 2 and 3
 *   - greedy colouring: Sec. III-A
 *   - restriction by straight injection and refinement: Sec. II-F, III-B
 *
 * Storage is compressed row storage (CRS, Sec. III-B) with columns in
 * ascending natural order.  Natural order is i = ix + nx*(iy + ny*iz).
 * All arrays are owned by the oracle; callers pass plain host buffers.
 */
#ifndef MGPCG_ORACLE_H
#define MGPCG_ORACLE_H
#include <stdint.h>

#define ORA_MAX_LEVELS 8

typedef struct {
    int nx, ny, nz;
    int64_t n;          /* rows */
    int64_t nnz;
    int64_t *rowptr;    /* n+1 */
    int32_t *col;       /* nnz, ascending per row */
    double *val;        /* nnz */
    double *diag;       /* n: the diagonal of A kept as a vector (Sec. III-A) */
    float *val32;       /* nnz: values rounded to FP32 (for the FP32 V-cycle) */
    float *diag32;      /* n */
    int ncolours;
    int32_t *colour;    /* n: colour number of each row */
    int64_t *cstart;    /* ncolours+1: offsets into clist */
    int64_t *clist;     /* n: rows grouped by colour, ascending within a colour */
    int64_t *f2c;       /* n_{l+1}: fine natural index of each coarse point (NULL on coarsest) */
} ora_level;

typedef struct {
    int levels;
    int colour_order;   /* 0: greedy numbering as found; 1: numbering reversed */
    int sweeps;         /* symmetric sweeps per smoothing step of the V-cycle (1) */
    ora_level lev[ORA_MAX_LEVELS];
} ora_hier;

/* Build the level hierarchy.  theta (may be NULL) has n_0 entries in natural
 * order; when given the diagonal is 26 + softplus(theta_i) and coarse levels
 * take theta at the injection point.  Returns NULL on invalid arguments. */
ora_hier *ora_create(int nx, int ny, int nz, int levels, int colour_order,
                     const double *theta);
void ora_destroy(ora_hier *h);
/* Symmetric sweeps per smoothing step of every V-cycle (default 1); returns
 * -1 and changes nothing if sweeps < 1. */
int ora_set_sweeps(ora_hier *h, int sweeps);

/* Introspection (for tests). */
int64_t ora_n(const ora_hier *h, int level);
int64_t ora_nnz(const ora_hier *h, int level);
int ora_ncolours(const ora_hier *h, int level);
void ora_get_crs(const ora_hier *h, int level, int64_t *rowptr, int32_t *col, double *val);
void ora_get_colours(const ora_hier *h, int level, int32_t *colour);
void ora_get_f2c(const ora_hier *h, int level, int64_t *f2c);

/* Building blocks, all in natural order, FP64. */
void ora_spmv(const ora_hier *h, int level, const double *x, double *y);
void ora_colour_pass(const ora_hier *h, int level, int k, const double *r, double *z);
void ora_sgs(const ora_hier *h, int level, const double *r, double *z);
void ora_restrict(const ora_hier *h, int level, const double *r, const double *z, double *rc);
void ora_prolong_add(const ora_hier *h, int level, const double *zc, double *z);
void ora_vcycle(const ora_hier *h, int level, const double *r, double *z);

/* Sequential symmetric Gauss-Seidel (Sec. II-E, Eq. (1)): rows in increasing,
 * then decreasing natural order; and the V-cycle that uses it as smoother. */
void ora_sgs_lex(const ora_hier *h, int level, const double *r, double *z);
void ora_vcycle_lex(const ora_hier *h, int level, const double *r, double *z);

/* FP32 V-cycle (project extension): r is rounded to FP32, the whole V-cycle
 * runs in FP32 with FP32 matrix values, z is widened back to FP64. */
void ora_vcycle32(const ora_hier *h, const double *r, double *z);
void ora_sgs32(const ora_hier *h, int level, const float *r, float *z);

/* Preconditioned CG (Sec. II-C).  precond: 0 none, 1 FP64 V-cycle,
 * 2 FP32 V-cycle, 3 FP64 V-cycle with the sequential smoother.  x holds x0
 * on entry and the iterate on exit.  history gets ||r_k||/||r_0|| for
 * k = 1..iters.  tol > 0 stops once history <= tol.
 * Returns 0 on success, 1 if max_iters was reached with tol > 0 unmet,
 * -5 on breakdown (<p,Ap> not finite or not positive). */
int ora_pcg(const ora_hier *h, const double *b, double *x, int max_iters,
            double tol, int precond, double *history, int *iters);

/* Gradient of a loss through x = A(theta)^{-1} b with respect to theta,
 * given the adjoint lambda = A^{-1} dL/dx:  dL/dtheta_i = -lambda_i x_i s(theta_i)
 * where s is the logistic function (derivative of softplus). */
void ora_theta_grad(int64_t n, const double *lambda, const double *x,
                    const double *theta, double *grad);

/* Threads the loops of this build use: 1 for the sequential checker, the
 * OpenMP thread count for the timing build (-fopenmp). */
int ora_threads(void);

/* Inner product used by CG: sequential, extended-precision accumulator. */
double ora_dot(int64_t n, const double *a, const double *b);

#endif
