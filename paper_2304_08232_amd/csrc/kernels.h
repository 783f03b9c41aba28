// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once
#include "mgpcg_internal.h"

namespace mg {

// Problem setup: fill the ELL operator of one level (values, columns).
hipError_t launch_build_ell(const mgpcg_problem *P, int level, const double *theta, hipStream_t s);

// natural <-> internal permutation of an FP64 level vector (R rhs)
hipError_t launch_permute(const mgpcg_problem *P, int level, const double *src, double *dst,
                          bool to_internal, hipStream_t s);

template <typename T>
hipError_t launch_spmv(const mgpcg_problem *P, int level, const T *val, const T *x, T *y, hipStream_t s);

// zero-start skip mask compiled into the kernels for colour k (standard colouring)
uint32_t standard_zs_mask(int k, int order);

// one colour pass of the coloured Gauss-Seidel smoother; mode: plain,
// zero start, or with the restriction / refinement of the level fused in
// (`coarse` is then the coarse-level rc or zc)
enum { kPassPlain = 0, kPassZeroStart = 1, kPassRestrict = 2, kPassProlong = 3, kPassTwice = 4,
       kPassTwiceZeroStart = 5, kPassZeroStart01 = 6 };
// rzp (FP64, one grid, plain or double pass): the pass also writes one
// partial of sum r_i z_i (its new z) per workgroup at rzp[block * R + rhs]
template <typename T>
hipError_t launch_pass(const mgpcg_problem *P, int level, int k, int mode, const T *val, const T *r, T *z,
                       const int *done, T *coarse, hipStream_t s, double *rzp = nullptr);

template <typename T>
hipError_t launch_restrict(const mgpcg_problem *P, int level, const T *val, const T *r, const T *z,
                           T *rc, hipStream_t s);

template <typename T>
hipError_t launch_prolong(const mgpcg_problem *P, int level, const T *zc, T *z, hipStream_t s);

// levels coarse_lc..L-1 of one V-cycle in one persistent launch
hipError_t launch_coarse_vcycle(const mgpcg_problem *P, bool fp32, hipStream_t s);
// levels tail_lw..L-1 of one V-cycle in one single-workgroup launch
hipError_t launch_coarse_tail(const mgpcg_problem *P, bool fp32, hipStream_t s);
int coarse_vcycle_occupancy(int R, bool fp32, int cf, int order);  // resident workgroups per CU

// delta-code a single-grid level's columns (L.dbase and L.dcol allocated);
// flags[0] (device) becomes nonzero if some delta does not fit in int8,
// flags[1] if some real entry has a nonzero delta
hipError_t launch_delta_encode(const mgpcg_problem *P, int level, const int64_t *coff_dev, int *flags,
                               hipStream_t s);

// sequential smoother (FP64): wavefront-major copy of a level's values, and
// one symmetric sweep of Eq. (1) over the level's wavefront schedule
hipError_t launch_wave_gather(const mgpcg_problem *P, int level, hipStream_t s);
hipError_t launch_lex_sweep(const mgpcg_problem *P, int level, const double *r, double *z, hipStream_t s);

hipError_t launch_cast_d2f(const double *src, float *dst, int64_t n, hipStream_t s);
hipError_t launch_cast_f2d(const float *src, double *dst, int64_t n, hipStream_t s);
hipError_t launch_fill_d(double *p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_i(int *p, int64_t n, int v, hipStream_t s);
hipError_t launch_fill_u(unsigned *p, int64_t n, unsigned v, hipStream_t s);

// CG kernels on level 0 (FP64, internal layout), with per-system scalars
hipError_t launch_init_residual(const mgpcg_problem *P, hipStream_t s);
hipError_t launch_dot_rz(const mgpcg_problem *P, hipStream_t s);
// FP32 V-cycle: widen its level-0 z into P->z and form <r, z> in one pass
hipError_t launch_cast_dot_rz(const mgpcg_problem *P, hipStream_t s);
hipError_t launch_finalize_rz(const mgpcg_problem *P, hipStream_t s);  // rho from the fused partials
hipError_t launch_update_p(const mgpcg_problem *P, hipStream_t s);
hipError_t launch_spmv_pq(const mgpcg_problem *P, hipStream_t s);
// r32 (FP32 V-cycle, may be NULL): also store the new r narrowed there
hipError_t launch_update_r(const mgpcg_problem *P, double tol, int hist_cap, hipStream_t s, float *r32 = nullptr);
hipError_t launch_flush_x(const mgpcg_problem *P, hipStream_t s);  // x += pending alpha p, after the last iteration

hipError_t launch_theta_grad(const double *lam, const double *x, const double *theta, double *grad,
                             int64_t n, hipStream_t s);

}  // namespace mg
