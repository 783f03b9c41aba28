/*
 * mgpcg.h -- C ABI of the MI355X (gfx950) multigrid-preconditioned conjugate
 * gradient library for the 27-point HPCG stencil.
 *
 * Method: arXiv 2304.08232, "Effective implementation of the High Performance
 * Conjugate Gradient benchmark on GraphBLAS":
 *   - problem (27-point operator, b, x0)         Sec. II-A, II-B
 *   - preconditioned CG                           Sec. II-C
 *   - multigrid V-cycle                           Sec. II-D, Listing 1
 *   - Gauss-Seidel update                         Sec. II-E, Eq. (1)
 *   - coloured symmetric Gauss-Seidel (RBGS)      Sec. III-A, Listings 2-3
 *   - greedy colouring                            Sec. III-A
 *   - straight-injection restriction/refinement   Sec. II-F, Sec. III-B
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an mgpcg_status.  Nothing is thrown across the ABI.
 *   On a negative status, mgpcg_last_error() returns a message (thread-local).
 * - Argument checks happen before anything is launched; a call that fails them
 *   has no effect.
 * - Vector arguments are DEVICE pointers (e.g. torch.Tensor.data_ptr()) owned
 *   by the caller, which must keep them alive until the stream work is done.
 *   They hold FP64 values.  Matrices, colour tables, transfer maps and all
 *   workspaces are owned by the problem handle.
 * - Streams are HIP streams (NULL = the legacy default stream).  Calls are
 *   asynchronous on the stream unless stated otherwise.
 * - A handle's workspaces (permutation buffers, level vectors, CG vectors,
 *   reduction partials, captured graphs) are shared by all calls on it.  Calls
 *   on one handle must therefore be ordered: issue them on one stream, or
 *   synchronise between the streams used.  Do not call on one handle from
 *   several host threads at once.  Separate handles are independent.
 * - Environment overrides, read by mgpcg_create, for tuning and tests.  None
 *   changes the arithmetic:
 *     MGPCG_DELTA_COLS     cap on the column format: 0 int32 columns, 1 int8
 *                          deltas, 2 (default) implied columns where possible
 *     MGPCG_NT_BYTES       operators larger than this use 256-thread
 *                          workgroups and non-temporal loads (default 128 MiB)
 *     MGPCG_TAIL_BYTES     largest coarsest level (r and z bytes) run in one
 *                          workgroup (default and maximum 64 KiB)
 *     MGPCG_COARSE_BLOCKS  workgroups of the persistent coarse kernel
 *                          (1..number of CUs)
 *     MGPCG_LEX_RUN_ROWS   largest wavefront a single-workgroup run of the
 *                          sequential smoother takes (0..512, default 256)
 *   MGPCG_NT_BYTES also regroups the partial sums of <r,z> when that product
 *   is fused into the level-0 smoother (the same caveat as wide_levels in
 *   mgpcg_schedule).
 * - A problem holds G >= 1 independent grids ("batched problems") with R >= 1
 *   right-hand sides each, i.e. S = G*R systems.  Vectors at level l are packed
 *   grid after grid; within a grid, right-hand side after right-hand side;
 *   within a right-hand side, one value per grid point.
 * - Layout MGPCG_LAYOUT_NATURAL: grid point order i = ix + nx*(iy + ny*iz).
 *   MGPCG_LAYOUT_INTERNAL: the library's own colour-major, rhs-interleaved
 *   order (for benchmarks that want no permutation in the timed region; use
 *   mgpcg_to_internal / mgpcg_to_natural to convert).
 */
#ifndef MGPCG_H
#define MGPCG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgpcg_problem mgpcg_problem;

typedef enum {
    MGPCG_OK = 0,
    MGPCG_NOT_CONVERGED = 1,       /* tol > 0 and max_iters reached; results valid */
    MGPCG_ERR_INVALID_ARG = -1,    /* NULL pointer, bad enum, bad level, ... */
    MGPCG_ERR_DIMS = -2,           /* dims < 1, levels out of range, dims not divisible */
    MGPCG_ERR_OOM = -3,            /* device allocation failed */
    MGPCG_ERR_HIP = -4,            /* a HIP runtime call failed (text in last_error) */
    MGPCG_ERR_BREAKDOWN = -5,      /* <p,Ap> not finite or not positive */
    MGPCG_ERR_NO_DEVICE = -6       /* no usable GPU */
} mgpcg_status;

enum { MGPCG_FP64 = 0, MGPCG_FP32 = 1 };
enum { MGPCG_LAYOUT_NATURAL = 0, MGPCG_LAYOUT_INTERNAL = 1 };
enum { MGPCG_SMOOTHER_COLOURED = 0, MGPCG_SMOOTHER_SEQUENTIAL = 1 };
#define MGPCG_MAX_LEVELS 8
#define MGPCG_MAX_RHS 16
#define MGPCG_MAX_SWEEPS 16

typedef struct {
    int ngrids;          /* G >= 1 */
    const int *dims;     /* HOST array of 3*G ints: nx, ny, nz of each grid */
    int levels;          /* 1..MGPCG_MAX_LEVELS; every dim divisible by 2^(levels-1) */
    int nrhs;            /* R in {1, 2, 4, 8, 16} */
    int mg_dtype;        /* MGPCG_FP64, or MGPCG_FP32 for an FP32 V-cycle inside FP64 CG */
    int colour_order;    /* 0: greedy colour numbering as found (Sec. III-A);
                            1: numbering reversed, so colour classes are swept
                               in the opposite order */
    const double *theta; /* DEVICE pointer or NULL.  When set: one value per
                            level-0 grid point (packed over grids, natural
                            order); the diagonal becomes 26 + softplus(theta_i)
                            and coarse levels take theta at the injection point */
    int smoother;        /* MGPCG_SMOOTHER_COLOURED (default): the coloured
                            symmetric Gauss-Seidel of Sec. III-A;
                            MGPCG_SMOOTHER_SEQUENTIAL: the sequential symmetric
                            Gauss-Seidel it replaces (Sec. II-E, Eq. (1): rows
                            in increasing, then decreasing natural order),
                            executed wavefront by wavefront
                            (t = ix + 2 iy + 4 iz).  Requires mg_dtype
                            MGPCG_FP64 and nrhs 1. */
    int sweeps;          /* symmetric sweeps per smoothing step of the V-cycle
                            (the pre- and post-smoothing of Listing 1, and
                            the coarsest level's), 0..MGPCG_MAX_SWEEPS; 0
                            means 1, the default of the paper's experiments
                            (Sec. V). */
} mgpcg_config;

/* Sec. II-A/B, II-D, III-A: build the level hierarchy on the current device:
 * per level the 27-point operator (diagonal 26, off-diagonals -1 for every
 * in-grid neighbour), its greedy colouring, and the injection maps.  The
 * operator is stored as 27-slot ELL with FP64 (and/or FP32) values, rows
 * grouped by colour; each level keeps its column indices in the most compact
 * exact form: implied by per-colour offsets, int8 deltas against them, or
 * int32 indices.  Synchronises the stream before returning.  *out receives
 * the handle (NULL on failure). */
mgpcg_status mgpcg_create(const mgpcg_config *cfg, hipStream_t stream, mgpcg_problem **out);

/* Releases every device buffer of the handle.  NULL is accepted. */
mgpcg_status mgpcg_destroy(mgpcg_problem *p);

/* Sizes at one level, summed over grids: rows n, structural nonzeros nnz
 * (closed form (3nx-2)(3ny-2)(3nz-2) per grid), and ELL slots (27 per row). */
mgpcg_status mgpcg_info(const mgpcg_problem *p, int level, int64_t *n, int64_t *nnz,
                        int64_t *ell_slots);

/* Replaces the coefficient field: theta as in mgpcg_config (DEVICE, level-0
 * points).  Rewrites the diagonal on every level. */
mgpcg_status mgpcg_set_theta(mgpcg_problem *p, const double *theta, hipStream_t stream);

/* Permutes an FP64 vector of level `level` (all grids, all rhs) between the
 * natural and the internal layout.  src and dst must not overlap. */
mgpcg_status mgpcg_to_internal(const mgpcg_problem *p, int level, const double *src, double *dst,
                               hipStream_t stream);
mgpcg_status mgpcg_to_natural(const mgpcg_problem *p, int level, const double *src, double *dst,
                              hipStream_t stream);

/* Sec. II-C: y = A_l x at level `level`.  Level 0 uses the FP64 operator; a
 * coarser level uses the V-cycle precision (FP32 problems round x to FP32 and
 * widen y back).  x and y must not overlap. */
mgpcg_status mgpcg_spmv(const mgpcg_problem *p, int level, const double *x, double *y, int layout,
                        hipStream_t stream);

/* b = A_0 * 1 (so that the exact solution is all ones).  FP64. */
mgpcg_status mgpcg_make_rhs_ones(const mgpcg_problem *p, double *b, int layout, hipStream_t stream);

/* Sec. III-A, Listings 2-3 (forward pass) and Sec. II-E (symmetric form):
 * one symmetric sweep of the problem's smoother at `level`, in place on z
 * (one sweep, whatever the config's `sweeps`).  Coloured: colours 0..c-1,
 * then c-1..0; for each row i of the colour being swept
 * z_i <- (r_i - sum_j a_ij z_j + z_i a_ii) / a_ii with the sum over the whole
 * row.  Sequential (Eq. (1)): rows in increasing, then decreasing natural
 * order, z_i <- (r_i - sum_{j != i} a_ij z_j) / a_ii with every z_j as last
 * updated.  Runs in the V-cycle precision.  r and z must not overlap. */
mgpcg_status mgpcg_gs_sweep(const mgpcg_problem *p, int level, const double *r, double *z, int layout,
                            hipStream_t stream);

/* Sec. III-A, Listings 2-3: one colour pass of the coloured Gauss-Seidel
 * smoother at `level`, in place on z: for every row i of colour `colour`,
 * z_i <- (r_i - sum_j a_ij z_j + z_i a_ii) / a_ii, the sum over the whole row
 * with z as it stands (rows of one colour are not coupled, so the order
 * within the colour does not matter).  Colours are numbered as the greedy
 * colouring finds them (reversed under colour_order 1); a 3-D grid with every
 * extent >= 2 has 8.  Runs in the V-cycle precision.  r and z must not
 * overlap.  MGPCG_ERR_INVALID_ARG if colour is not a colour of the level. */
mgpcg_status mgpcg_colour_pass(const mgpcg_problem *p, int level, int colour, const double *r, double *z,
                               int layout, hipStream_t stream);

/* Sec. II-D Listing 1 and Sec. II-F: rc = inject(r - A_l z), the residual at
 * the injection points (2jx, 2jy, 2jz) of level `level` written to level+1.
 * V-cycle precision.  Requires level+1 < levels. */
mgpcg_status mgpcg_restrict(const mgpcg_problem *p, int level, const double *r, const double *z,
                            double *rc, int layout, hipStream_t stream);

/* Sec. II-F, Listing 1: z += refine(zc), i.e. zc added at the injection
 * points of level `level`.  V-cycle precision. */
mgpcg_status mgpcg_prolong_add(const mgpcg_problem *p, int level, const double *zc, double *z,
                               int layout, hipStream_t stream);

/* Sec. II-D, Listing 1: z = M^{-1} r, one V-cycle from z = 0: smoothing,
 * restriction, recursion, refinement, smoothing; the coarsest level only
 * smooths.  Each smoothing step is `sweeps` symmetric sweeps of the
 * problem's smoother.  r and z are level-0 vectors. */
mgpcg_status mgpcg_mg_vcycle(const mgpcg_problem *p, const double *r, double *z, int layout,
                             hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the V-cycle
 * of mgpcg_mg_vcycle, same arguments and the same results bit for bit, with
 * no device allocation and no hipMalloc/hipFree in the call.  (mgpcg_mg_vcycle
 * allocates per-level staging buffers on its first call.)  The natural-layout
 * staging of r and z goes through a fixed 32 MiB array that the library holds
 * on every device it runs on until the process ends: in natural layout at
 * most 2^21 level-0 values (n*R) are accepted, larger problems return
 * MGPCG_ERR_INVALID_ARG before anything is launched (MGPCG_LAYOUT_INTERNAL has
 * no limit; it stages nothing).  Every call on one device shares that array,
 * and the handle's own level vectors as mgpcg_mg_vcycle does: calls that
 * overlap on one device (other streams, other handles) race and must be
 * ordered by the caller. */
mgpcg_status mgpcg_mg_vcycle_noalloc(const mgpcg_problem *p, const double *r, double *z, int layout,
                                     hipStream_t stream);

/* Sec. II-C: preconditioned CG for all S systems at once, starting from x
 * (x holds x0 on entry and the iterate on exit).  Per system: r = b - A x,
 * then per iteration z = M r, rho = <r,z>, p = z + (rho/rho_old) p (p = z at
 * the first), q = A p, alpha = rho/<p,q>, x += alpha p, r -= alpha q, and the
 * relative residual ||r||/||r_0|| is recorded.  rel_tol > 0 stops a system at
 * the first iteration whose relative residual is <= rel_tol; rel_tol = 0 runs
 * exactly max_iters iterations.  A system whose b - A x0 is zero does 0
 * iterations.
 *
 * history_host: NULL or S*max_iters doubles (system-major); entries past a
 * system's iteration count are set to 0.  iters_host: NULL or S ints.
 * When both are NULL and rel_tol == 0 the call is asynchronous (only argument
 * errors are reported; fetch results with mgpcg_solve_result).  Otherwise it
 * synchronises the stream and returns MGPCG_OK, MGPCG_NOT_CONVERGED (some
 * system missed rel_tol) or MGPCG_ERR_BREAKDOWN (some system stopped on a
 * breakdown; its x is the last good iterate). */
mgpcg_status mgpcg_pcg_solve(mgpcg_problem *p, const double *b, double *x, int max_iters,
                             double rel_tol, double *history_host, int *iters_host, int layout,
                             hipStream_t stream);

/* Results of the most recent mgpcg_pcg_solve (synchronises the stream).
 * Same meaning of history_host / iters_host / the returned status as above;
 * max_iters must equal the value that solve used. */
mgpcg_status mgpcg_solve_result(mgpcg_problem *p, int max_iters, double *history_host,
                                int *iters_host, hipStream_t stream);

/* Differentiable solve: with x = A(theta)^{-1} b and the adjoint
 * lambda = A^{-1} dL/dx (A is symmetric), writes
 * grad_i = -lambda_i * x_i * logistic(theta_i), the gradient of L with respect
 * to theta when a_ii = 26 + softplus(theta_i).  Element-wise over the n level-0
 * points of every grid (R must be 1); any common layout. */
mgpcg_status mgpcg_theta_grad(const mgpcg_problem *p, const double *lambda, const double *x,
                              const double *theta, double *grad, hipStream_t stream);

/* Execution mode of mgpcg_pcg_solve: on = 1 (default) captures one CG
 * iteration into a HIP graph on first use and replays it; on = 0 launches the
 * iteration's kernels one by one.  Results are identical either way. */
mgpcg_status mgpcg_set_graph_mode(mgpcg_problem *p, int on);

/* Execution of the coarse levels of the V-cycle: mode 0 (default) launches
 * one kernel per colour pass; mode 1 runs levels 1..L-1 of each V-cycle in
 * one persistent launch whose workgroups separate the phases with a grid
 * barrier (used when nrhs is 1, sweeps is 1, the smoother is the coloured
 * one, every coarse grid has the standard 8-colour numbering and the coarse
 * levels share one column format, int32 when the problem has several grids;
 * otherwise mode 0 runs).  Results are identical either way. */
mgpcg_status mgpcg_set_coarse_mode(mgpcg_problem *p, int mode);

/* Execution schedule of a problem: how its kernels are launched, never what
 * they compute.  A solve gives bit-identical results under every schedule,
 * except that changing bit 0 of wide_levels on a problem that fuses <r,z>
 * into the level-0 post-smoother (one grid, one right-hand side, FP64
 * V-cycle, coloured smoother) regroups that sum's partials, which moves its
 * rounding. */
typedef struct {
    int graph;         /* as mgpcg_set_graph_mode: 1 replay a captured
                          iteration, 0 launch its kernels one by one */
    int coarse_mode;   /* as mgpcg_set_coarse_mode */
    int coarse_tail;   /* 1: the coarsest level of the coloured V-cycle runs in
                          one single-workgroup kernel when it fits (nrhs 1,
                          sweeps 1, r and z of the level within 64 KiB, at
                          most 512 rows per colour); 0: one kernel per pass */
    unsigned wide_levels; /* bit l: level l's colour passes use 256-thread
                          workgroups and stream the operator with
                          non-temporal loads; clear: 64-thread workgroups and
                          cached loads.  Bits at and above `levels` must be
                          0.  Default: set for levels whose operator exceeds
                          128 MiB */
    int lex_run_rows;  /* sequential smoother: the largest wavefront, in
                          rows, that a single-workgroup run sweeps (0..512;
                          0: one launch per wavefront); default 256 */
} mgpcg_schedule;

/* Reads the current schedule into *out (HOST). */
mgpcg_status mgpcg_get_schedule(const mgpcg_problem *p, mgpcg_schedule *out);

/* Applies *sched (HOST).  Invalid fields return MGPCG_ERR_INVALID_ARG and
 * change nothing.  Discards the captured iteration graph; may synchronise the
 * stream. */
mgpcg_status mgpcg_set_schedule(mgpcg_problem *p, const mgpcg_schedule *sched, hipStream_t stream);

/* Autotuner for the schedule of this problem.  Times candidate schedules by
 * coordinate descent from the current one (graph mode; coarse mode and tail;
 * each level's workgroup choice, leaving bit 0 alone where changing it would
 * move rounding; the sequential smoother's run limit), each as `reps` timed
 * runs of `iters` PCG iterations from x = 0 after one warm-up run, keeps the
 * fastest (best of its runs) and applies it.  b: DEVICE right-hand side in
 * natural layout, or NULL for b = A*1.  cache_path (HOST string, may be
 * NULL): a text file with one JSON object per line; if it holds an entry for
 * this problem (grids, levels, right-hand sides, precision, colour order,
 * smoother, sweeps) on this kind of device, the last such entry is applied
 * without timing; an entry with fields mgpcg_set_schedule would reject is
 * ignored.  Otherwise the chosen schedule is appended.  *chosen (HOST, may be NULL)
 * receives the applied schedule.  iters in 1..1000, reps in 1..100.
 * Allocates two vectors of the level-0 size for the duration of the call and
 * synchronises the stream.  The timed runs are solves on this problem: a
 * later mgpcg_solve_result reports the last of them, not an earlier solve. */
mgpcg_status mgpcg_autotune(mgpcg_problem *p, const double *b, int iters, int reps, const char *cache_path,
                            mgpcg_schedule *chosen, hipStream_t stream);

/* Synchronises the stream and reports a device-side failure of earlier
 * asynchronous work on this problem (MGPCG_ERR_HIP, e.g. a coarse-level grid
 * barrier that timed out), else MGPCG_OK. */
mgpcg_status mgpcg_check(mgpcg_problem *p, hipStream_t stream);

/* Message describing the last non-OK status returned on this thread. */
const char *mgpcg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MGPCG_H */
