// gfx950 kernels of the MG-PCG hot path.
//
// Every kernel is HBM-bound (about 0.16 flop per byte), so the design goals
// are: stream the ELL operator exactly once per pass with coalesced,
// non-temporal loads; keep the vectors (which fit in the Infinity Cache) in
// the cache hierarchy; hand each XCD a contiguous range of rows so that the
// neighbour gathers of one XCD hit its own L2; and make every reduction
// deterministic (fixed-shape wave/LDS trees plus an ordered final pass in the
// last workgroup of each grid).
//
// Floating-point contraction is disabled for this library, so that the
// per-row arithmetic is exactly the sequence of IEEE operations the method
// states: sums over the row in ascending column order, the Gauss-Seidel update
// (r - s + z*d)/d with a true division, and the CG vector updates.
#include "kernels.h"

namespace mg {

namespace {

constexpr int kXcd = 8;  // XCDs per MI355X; workgroups are dealt round-robin

// Workgroup b of nb is dispatched to XCD b % 8.  Return the logical block so
// that each XCD receives one contiguous range of logical blocks.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    int per = nb / kXcd, rem = nb % kXcd;
    int x = b % kXcd, q = b / kXcd;
    return x * per + (x < rem ? x : rem) + q;
}

template <typename T>
__device__ __forceinline__ T ld_nt(const T *p) {
    return __builtin_nontemporal_load(p);
}

__device__ __forceinline__ double softplus_d(double t) {
    return fmax(t, 0.0) + log1p(exp(-fabs(t)));
}

__device__ __forceinline__ double logistic_d(double t) {
    return 1.0 / (1.0 + exp(-t));
}

__device__ __forceinline__ int find_grid(const int64_t *off, int G, int64_t q) {
    int lo = 0, hi = G;  // off[lo] <= q < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= q) lo = mid; else hi = mid;
    }
    return lo;
}

inline int nblocks(int64_t work) { return (int)((work + kBlock - 1) / kBlock); }

}  // namespace

// ------------------------------------------------------------------ setup

// One thread per internal row: recover the grid point, then write the 27
// slots in direction order (ascending natural column order).
__global__ __launch_bounds__(kBlock) void k_build_ell(
    int64_t n, int G, const int32_t *__restrict__ iperm, const int32_t *__restrict__ perm,
    const int64_t *__restrict__ natoff, const int *__restrict__ dims0, int shift,
    const int64_t *__restrict__ natoff0, const double *__restrict__ theta,
    double *__restrict__ val64, float *__restrict__ val32, int32_t *__restrict__ col) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int64_t q = iperm[i];
    int g = G > 1 ? find_grid(natoff, G, q) : 0;
    int nx0 = dims0[3 * g], ny0 = dims0[3 * g + 1];
    int nx = nx0 >> shift, ny = dims0[3 * g + 1] >> shift, nz = dims0[3 * g + 2] >> shift;
    int64_t loc = q - natoff[g];
    int ix = (int)(loc % nx), iy = (int)((loc / nx) % ny), iz = (int)(loc / ((int64_t)nx * ny));
    double d = 26.0;
    if (theta) {
        int64_t f = natoff0[g] + ((int64_t)ix << shift) +
                    (int64_t)nx0 * (((int64_t)iy << shift) + (int64_t)ny0 * ((int64_t)iz << shift));
        d += softplus_d(theta[f]);
    }
#pragma unroll
    for (int s = 0; s < kW; ++s) {
        int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
        int jx = ix + dx, jy = iy + dy, jz = iz + dz;
        bool in = jx >= 0 && jx < nx && jy >= 0 && jy < ny && jz >= 0 && jz < nz;
        double v = in ? (s == kCentre ? d : -1.0) : 0.0;
        int32_t c = in ? perm[natoff[g] + jx + (int64_t)nx * (jy + (int64_t)ny * jz)] : (int32_t)i;
        int64_t e = (int64_t)s * n + i;
        if (val64) val64[e] = v;
        if (val32) val32[e] = (float)v;
        col[e] = c;
    }
}

hipError_t launch_build_ell(const mgpcg_problem *P, int level, const double *theta, hipStream_t s) {
    const Level &L = P->lev[level];
    if (L.n == 0) return hipSuccess;
    k_build_ell<<<nblocks(L.n), kBlock, 0, s>>>(L.n, P->G, L.iperm, L.perm, P->d_natoff[level],
                                                P->d_dims0, level, P->d_natoff0, theta, L.val64,
                                                L.val32, L.col);
    return hipGetLastError();
}

// natural packed layout: grid g block at R*natoff[g], rhs v at + v*n_g
template <int R, bool TO_INT>
__global__ __launch_bounds__(kBlock) void k_permute(int64_t n, int G, const int32_t *__restrict__ iperm,
                                                    const int64_t *__restrict__ natoff,
                                                    const double *__restrict__ src,
                                                    double *__restrict__ dst) {
    int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gid >= n * R) return;
    int64_t i = gid / R;
    int v = (int)(gid % R);
    int64_t q = iperm[i];
    int g = G > 1 ? find_grid(natoff, G, q) : 0;
    int64_t ng = natoff[g + 1] - natoff[g];
    int64_t nat = (int64_t)R * natoff[g] + (int64_t)v * ng + (q - natoff[g]);
    if (TO_INT) dst[gid] = src[nat];
    else dst[nat] = src[gid];
}

#define MG_DISPATCH_R(R, CALL)                 \
    switch (R) {                               \
        case 1: { constexpr int RR = 1; CALL; } break;  \
        case 2: { constexpr int RR = 2; CALL; } break;  \
        case 4: { constexpr int RR = 4; CALL; } break;  \
        case 8: { constexpr int RR = 8; CALL; } break;  \
        case 16: { constexpr int RR = 16; CALL; } break; \
        default: return hipErrorInvalidValue;  \
    }

hipError_t launch_permute(const mgpcg_problem *P, int level, const double *src, double *dst,
                          bool to_internal, hipStream_t s) {
    const Level &L = P->lev[level];
    int64_t work = L.n * P->R;
    if (work == 0) return hipSuccess;
    if (to_internal) {
        MG_DISPATCH_R(P->R, (k_permute<RR, true><<<nblocks(work), kBlock, 0, s>>>(
                                L.n, P->G, L.iperm, P->d_natoff[level], src, dst)));
    } else {
        MG_DISPATCH_R(P->R, (k_permute<RR, false><<<nblocks(work), kBlock, 0, s>>>(
                                L.n, P->G, L.iperm, P->d_natoff[level], src, dst)));
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------- SpMV

// y = A x over all rows; one thread per (row, rhs).  The R lanes of a row
// load the same operator entry (one transaction) and R consecutive x values.
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_spmv(int64_t n, const T *__restrict__ val,
                                                 const int32_t *__restrict__ col,
                                                 const T *__restrict__ x, T *__restrict__ y) {
    int64_t gid = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (gid >= n * R) return;
    int64_t i = gid / R;
    int v = (int)(gid % R);
    T acc = 0;
#pragma unroll
    for (int sl = 0; sl < kW; ++sl) {
        int64_t e = (int64_t)sl * n + i;
        T a = ld_nt(val + e);
        int32_t c = ld_nt(col + e);
        if (a != T(0)) acc = acc + a * x[(int64_t)c * R + v];
    }
    y[gid] = acc;
}

template <typename T>
hipError_t launch_spmv(const mgpcg_problem *P, int level, const T *val, const T *x, T *y, hipStream_t s) {
    const Level &L = P->lev[level];
    int64_t work = L.n * P->R;
    if (work == 0) return hipSuccess;
    MG_DISPATCH_R(P->R, (k_spmv<T, RR><<<nblocks(work), kBlock, 0, s>>>(L.n, val, L.col, x, y)));
    return hipGetLastError();
}
template hipError_t launch_spmv<double>(const mgpcg_problem *, int, const double *, const double *,
                                        double *, hipStream_t);
template hipError_t launch_spmv<float>(const mgpcg_problem *, int, const float *, const float *,
                                       float *, hipStream_t);

// ------------------------------------------------------------ colour pass

// One colour of the coloured Gauss-Seidel pass (Listing 3 of the paper, the
// masked product and the update fused).  Rows of one colour are independent,
// so the update is done in place: a row reads only other colours and itself.
// ZS (zero start): z is all zeros before this sweep, so only neighbours
// already written in this sweep (colours < k) are read; `skip` holds the
// slots whose neighbour cannot have been written yet (including the
// diagonal), and z_i itself is taken as 0.  The z array needs no clearing.
template <typename T, int R, bool ZS>
__global__ __launch_bounds__(kBlock) void k_pass(int64_t n, const T *__restrict__ val,
                                                 const int32_t *__restrict__ col,
                                                 const T *__restrict__ r, T *z,
                                                 const Seg *__restrict__ tab, uint32_t skip,
                                                 const int *__restrict__ done) {
    Seg e = tab[xcd_remap(blockIdx.x, gridDim.x)];
    int rl = threadIdx.x / R, v = threadIdx.x % R;
    if (rl >= e.count) return;
    if (done && done[e.grid * R + v]) return;
    int64_t i = e.row0 + rl;
    T acc = 0, d = 0;
#pragma unroll
    for (int sl = 0; sl < kW; ++sl) {
        int64_t ei = (int64_t)sl * n + i;
        if (ZS && ((skip >> sl) & 1u)) {
            if (sl == kCentre) d = ld_nt(val + ei);
            continue;
        }
        T a = ld_nt(val + ei);
        int32_t c = ld_nt(col + ei);
        if (sl == kCentre) d = a;
        if (a != T(0)) acc = acc + a * z[(int64_t)c * R + v];
    }
    int64_t o = i * R + v;
    T zi = ZS ? T(0) : z[o];
    z[o] = (r[o] - acc + zi * d) / d;
}

template <typename T>
hipError_t launch_pass(const mgpcg_problem *P, int level, int k, bool zero_start, const T *val,
                       const T *r, T *z, const int *done, hipStream_t s) {
    const Level &L = P->lev[level];
    int first = L.pass_first[k], cnt = L.pass_first[k + 1] - first;
    if (cnt == 0) return hipSuccess;
    const Seg *tab = L.pass_tab + first;
    if (zero_start) {
        MG_DISPATCH_R(P->R, (k_pass<T, RR, true><<<cnt, kBlock, 0, s>>>(L.n, val, L.col, r, z, tab,
                                                                         L.zi_skip[k], done)));
    } else {
        MG_DISPATCH_R(P->R, (k_pass<T, RR, false><<<cnt, kBlock, 0, s>>>(L.n, val, L.col, r, z, tab,
                                                                          0u, done)));
    }
    return hipGetLastError();
}
template hipError_t launch_pass<double>(const mgpcg_problem *, int, int, bool, const double *,
                                        const double *, double *, const int *, hipStream_t);
template hipError_t launch_pass<float>(const mgpcg_problem *, int, int, bool, const float *,
                                       const float *, float *, const int *, hipStream_t);

// ------------------------------------------------------------- transfers

// rc = inject(r - A z): only the injection rows of the residual are formed.
// Threads walk the injection rows in fine order (coalesced operator reads)
// and scatter into the coarse vector.
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_restrict(int64_t n, const T *__restrict__ val,
                                                     const int32_t *__restrict__ col,
                                                     const T *__restrict__ r, const T *__restrict__ z,
                                                     T *__restrict__ rc,
                                                     const int32_t *__restrict__ inj_fine,
                                                     const int32_t *__restrict__ inj_coarse,
                                                     int64_t n_inj) {
    int64_t gid = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (gid >= n_inj * R) return;
    int64_t t = gid / R;
    int v = (int)(gid % R);
    int64_t i = inj_fine[t];
    T acc = 0;
#pragma unroll
    for (int sl = 0; sl < kW; ++sl) {
        int64_t e = (int64_t)sl * n + i;
        T a = ld_nt(val + e);
        int32_t c = ld_nt(col + e);
        if (a != T(0)) acc = acc + a * z[(int64_t)c * R + v];
    }
    rc[(int64_t)inj_coarse[t] * R + v] = r[i * R + v] - acc;
}

template <typename T>
hipError_t launch_restrict(const mgpcg_problem *P, int level, const T *val, const T *r, const T *z,
                           T *rc, hipStream_t s) {
    const Level &L = P->lev[level];
    int64_t work = L.n_inj * P->R;
    if (work == 0) return hipSuccess;
    MG_DISPATCH_R(P->R, (k_restrict<T, RR><<<nblocks(work), kBlock, 0, s>>>(
                            L.n, val, L.col, r, z, rc, L.inj_fine, L.inj_coarse, L.n_inj)));
    return hipGetLastError();
}
template hipError_t launch_restrict<double>(const mgpcg_problem *, int, const double *, const double *,
                                            const double *, double *, hipStream_t);
template hipError_t launch_restrict<float>(const mgpcg_problem *, int, const float *, const float *,
                                           const float *, float *, hipStream_t);

// z += refine(zc): the coarse values are added at the injection points.
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_prolong(const T *__restrict__ zc, T *__restrict__ z,
                                                    const int32_t *__restrict__ inj_fine,
                                                    const int32_t *__restrict__ inj_coarse,
                                                    int64_t n_inj) {
    int64_t gid = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (gid >= n_inj * R) return;
    int64_t t = gid / R;
    int v = (int)(gid % R);
    int64_t o = (int64_t)inj_fine[t] * R + v;
    z[o] = z[o] + zc[(int64_t)inj_coarse[t] * R + v];
}

template <typename T>
hipError_t launch_prolong(const mgpcg_problem *P, int level, const T *zc, T *z, hipStream_t s) {
    const Level &L = P->lev[level];
    int64_t work = L.n_inj * P->R;
    if (work == 0) return hipSuccess;
    MG_DISPATCH_R(P->R, (k_prolong<T, RR><<<nblocks(work), kBlock, 0, s>>>(zc, z, L.inj_fine,
                                                                          L.inj_coarse, L.n_inj)));
    return hipGetLastError();
}
template hipError_t launch_prolong<double>(const mgpcg_problem *, int, const double *, double *,
                                           hipStream_t);
template hipError_t launch_prolong<float>(const mgpcg_problem *, int, const float *, float *,
                                          hipStream_t);

// ------------------------------------------------------------ elementwise

__global__ __launch_bounds__(kBlock) void k_cast_d2f(const double *__restrict__ a, float *__restrict__ b,
                                                     int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
__global__ __launch_bounds__(kBlock) void k_cast_f2d(const float *__restrict__ a, double *__restrict__ b,
                                                     int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *__restrict__ p, int64_t n, T v) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_cast_d2f(const double *src, float *dst, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_cast_d2f<<<nblocks(n), kBlock, 0, s>>>(src, dst, n);
    return hipGetLastError();
}
hipError_t launch_cast_f2d(const float *src, double *dst, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_cast_f2d<<<nblocks(n), kBlock, 0, s>>>(src, dst, n);
    return hipGetLastError();
}
hipError_t launch_fill_d(double *p, int64_t n, double v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_fill<double><<<nblocks(n), kBlock, 0, s>>>(p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_i(int *p, int64_t n, int v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_fill<int><<<nblocks(n), kBlock, 0, s>>>(p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u(unsigned *p, int64_t n, unsigned v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_fill<unsigned><<<nblocks(n), kBlock, 0, s>>>(p, n, v);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_theta_grad(const double *__restrict__ lam,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ th,
                                                       double *__restrict__ g, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) g[i] = -lam[i] * x[i] * logistic_d(th[i]);
}
hipError_t launch_theta_grad(const double *lam, const double *x, const double *theta, double *grad,
                             int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_theta_grad<<<nblocks(n), kBlock, 0, s>>>(lam, x, theta, grad, n);
    return hipGetLastError();
}

// ----------------------------------------------------- CG with reductions
//
// Reduction kernels walk the level-0 reduction table: each workgroup owns a
// grid-homogeneous segment of rows, and the segments of one grid are
// consecutive table entries [gb[g], gb[g+1]).  A workgroup reduces its
// per-rhs partial sums with a fixed wave-shuffle/LDS tree and publishes them;
// the last workgroup of each grid (ticket counter per grid) then adds that
// grid's partials in a fixed order and updates the CG scalars of its R
// systems.  Results are therefore identical from run to run.

enum Kind { kInit = 0, kRz = 1, kPq = 2, kRr = 3 };

struct RedArgs {
    const Seg *tab;
    const int *gb;
    double *partials;
    unsigned *tickets;  // this kind's G counters
    int G;
};

// Returns true in the last workgroup of grid g; then tot[v] (shared) holds
// the grid's total for rhs v.  Every thread of the workgroup must call it.
template <int R>
__device__ bool reduce_last(double acc, int blk, int g, const RedArgs &ra, double *tot) {
    __shared__ double sh[(kBlock / 64) * R];
    __shared__ int is_last;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= R; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane < R) sh[w * R + lane] = acc;
    __syncthreads();
    if (threadIdx.x < R) {
        double s = sh[threadIdx.x];
#pragma unroll
        for (int k = 1; k < kBlock / 64; ++k) s += sh[k * R + threadIdx.x];
        __hip_atomic_store(&ra.partials[(int64_t)blk * R + threadIdx.x], s, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = atomicAdd(&ra.tickets[g], 1u);
        is_last = (t == (unsigned)(ra.gb[g + 1] - ra.gb[g] - 1));
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    const int v = threadIdx.x % R;
    double s = 0.0;
    for (int b = ra.gb[g] + threadIdx.x / R; b < ra.gb[g + 1]; b += kBlock / R)
        s += __hip_atomic_load(&ra.partials[(int64_t)b * R + v], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int off = 32; off >= R; off >>= 1) s += __shfl_xor(s, off, 64);
    __syncthreads();
    if (lane < R) sh[w * R + lane] = s;
    __syncthreads();
    if (threadIdx.x < R) {
        double t = sh[threadIdx.x];
#pragma unroll
        for (int k = 1; k < kBlock / 64; ++k) t += sh[k * R + threadIdx.x];
        tot[threadIdx.x] = t;
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(&ra.tickets[g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return true;
}

// all R systems of grid g finished?
template <int R>
__device__ __forceinline__ bool grid_done(const int *done, int g) {
    bool all = true;
#pragma unroll
    for (int v = 0; v < R; ++v) all = all && done[g * R + v];
    return all;
}

// r = b - A x; ||r|| becomes the reference norm of each system.
template <int R>
__global__ __launch_bounds__(kBlock) void k_init_residual(int64_t n, const double *__restrict__ val,
                                                          const int32_t *__restrict__ col,
                                                          const double *__restrict__ b,
                                                          const double *__restrict__ x,
                                                          double *__restrict__ r, RedArgs ra,
                                                          Scalars sc) {
    __shared__ double tot[R];
    int blk = xcd_remap(blockIdx.x, gridDim.x);
    Seg e = ra.tab[blk];
    const int v = threadIdx.x % R;
    double acc = 0.0;
    for (int rl = threadIdx.x / R; rl < e.count; rl += kBlock / R) {
        int64_t i = e.row0 + rl;
        double s = 0.0;
#pragma unroll
        for (int sl = 0; sl < kW; ++sl) {
            int64_t ei = (int64_t)sl * n + i;
            double a = ld_nt(val + ei);
            int32_t c = ld_nt(col + ei);
            if (a != 0.0) s = s + a * x[(int64_t)c * R + v];
        }
        double ri = b[i * R + v] - s;
        r[i * R + v] = ri;
        acc += ri * ri;
    }
    if (!reduce_last<R>(acc, blk, e.grid, ra, tot)) return;
    if (threadIdx.x < R) {
        int sys = e.grid * R + threadIdx.x;
        double nr0 = sqrt(tot[threadIdx.x]);
        sc.nr0[sys] = nr0;
        if (nr0 == 0.0) {
            sc.done[sys] = 1;
            sc.status[sys] = 1;
            atomicAdd(sc.ndone, 1);
        }
    }
}

// rho = <r, z>; beta = rho / rho_old (0 at the first iteration).
template <int R>
__global__ __launch_bounds__(kBlock) void k_dot_rz(const double *__restrict__ r,
                                                   const double *__restrict__ z, RedArgs ra,
                                                   Scalars sc) {
    __shared__ double tot[R];
    int blk = xcd_remap(blockIdx.x, gridDim.x);
    Seg e = ra.tab[blk];
    if (grid_done<R>(sc.done, e.grid)) return;
    const int v = threadIdx.x % R;
    double acc = 0.0;
    for (int rl = threadIdx.x / R; rl < e.count; rl += kBlock / R) {
        int64_t o = (e.row0 + rl) * R + v;
        acc += r[o] * z[o];
    }
    if (!reduce_last<R>(acc, blk, e.grid, ra, tot)) return;
    if (threadIdx.x < R) {
        int sys = e.grid * R + threadIdx.x;
        if (!sc.done[sys]) {
            double rho = tot[threadIdx.x];
            sc.beta[sys] = (sc.iter[sys] == 0) ? 0.0 : rho / sc.rho_old[sys];
            sc.rho[sys] = rho;
            sc.rho_old[sys] = rho;
        }
    }
}

// p = z + beta p
template <int R>
__global__ __launch_bounds__(kBlock) void k_update_p(const double *__restrict__ z, double *__restrict__ p,
                                                     const Seg *__restrict__ tab, Scalars sc) {
    Seg e = tab[xcd_remap(blockIdx.x, gridDim.x)];
    const int v = threadIdx.x % R;
    const int sys = e.grid * R + v;
    if (sc.done[sys]) return;
    const double beta = sc.beta[sys];
    for (int rl = threadIdx.x / R; rl < e.count; rl += kBlock / R) {
        int64_t o = (e.row0 + rl) * R + v;
        p[o] = z[o] + beta * p[o];
    }
}

// q = A p; alpha = rho / <p, q>, or a breakdown flag.
template <int R>
__global__ __launch_bounds__(kBlock) void k_spmv_pq(int64_t n, const double *__restrict__ val,
                                                    const int32_t *__restrict__ col,
                                                    const double *__restrict__ p,
                                                    double *__restrict__ q, RedArgs ra, Scalars sc) {
    __shared__ double tot[R];
    int blk = xcd_remap(blockIdx.x, gridDim.x);
    Seg e = ra.tab[blk];
    if (grid_done<R>(sc.done, e.grid)) return;
    const int v = threadIdx.x % R;
    double acc = 0.0;
    for (int rl = threadIdx.x / R; rl < e.count; rl += kBlock / R) {
        int64_t i = e.row0 + rl;
        double s = 0.0;
#pragma unroll
        for (int sl = 0; sl < kW; ++sl) {
            int64_t ei = (int64_t)sl * n + i;
            double a = ld_nt(val + ei);
            int32_t c = ld_nt(col + ei);
            if (a != 0.0) s = s + a * p[(int64_t)c * R + v];
        }
        q[i * R + v] = s;
        acc += p[i * R + v] * s;
    }
    if (!reduce_last<R>(acc, blk, e.grid, ra, tot)) return;
    if (threadIdx.x < R) {
        int sys = e.grid * R + threadIdx.x;
        if (!sc.done[sys]) {
            double pq = tot[threadIdx.x];
            sc.pq[sys] = pq;
            if (!(pq > 0.0) || !isfinite(pq)) {
                sc.alpha[sys] = 0.0;
                sc.status[sys] = MGPCG_ERR_BREAKDOWN;
                sc.done[sys] = 1;
                atomicAdd(sc.ndone, 1);
            } else {
                sc.alpha[sys] = sc.rho[sys] / pq;
            }
        }
    }
}

// x += alpha p; r -= alpha q; record ||r|| / ||r0|| and test convergence.
template <int R>
__global__ __launch_bounds__(kBlock) void k_update_xr(double *__restrict__ x, const double *__restrict__ p,
                                                      double *__restrict__ r,
                                                      const double *__restrict__ q, RedArgs ra,
                                                      Scalars sc, double *__restrict__ hist,
                                                      int hist_cap, double tol) {
    __shared__ double tot[R];
    int blk = xcd_remap(blockIdx.x, gridDim.x);
    Seg e = ra.tab[blk];
    if (grid_done<R>(sc.done, e.grid)) return;
    const int v = threadIdx.x % R;
    const int sys = e.grid * R + v;
    const bool live = !sc.done[sys];
    const double alpha = sc.alpha[sys];
    double acc = 0.0;
    if (live) {
        for (int rl = threadIdx.x / R; rl < e.count; rl += kBlock / R) {
            int64_t o = (e.row0 + rl) * R + v;
            x[o] = x[o] + alpha * p[o];
            double ri = r[o] - alpha * q[o];
            r[o] = ri;
            acc += ri * ri;
        }
    }
    if (!reduce_last<R>(acc, blk, e.grid, ra, tot)) return;
    if (threadIdx.x < R) {
        int s2 = e.grid * R + threadIdx.x;
        if (!sc.done[s2]) {
            int k = sc.iter[s2] + 1;
            sc.iter[s2] = k;
            double rel = sqrt(tot[threadIdx.x]) / sc.nr0[s2];
            if (k <= hist_cap) hist[(int64_t)s2 * hist_cap + (k - 1)] = rel;
            if (tol > 0.0 && rel <= tol) {
                sc.done[s2] = 1;
                sc.status[s2] = 1;
                atomicAdd(sc.ndone, 1);
            }
        }
    }
}

static RedArgs red_args(const mgpcg_problem *P, int kind) {
    RedArgs ra;
    ra.tab = P->red_tab;
    ra.gb = P->red_gb;
    ra.partials = P->sc.partials;
    ra.tickets = P->sc.tickets + (int64_t)kind * P->G;
    ra.G = P->G;
    return ra;
}

hipError_t launch_init_residual(const mgpcg_problem *P, hipStream_t s) {
    const Level &L = P->lev[0];
    RedArgs ra = red_args(P, kInit);
    MG_DISPATCH_R(P->R, (k_init_residual<RR><<<P->n_red, kBlock, 0, s>>>(L.n, L.val64, L.col, P->b,
                                                                         P->x, P->r, ra, P->sc)));
    return hipGetLastError();
}
hipError_t launch_dot_rz(const mgpcg_problem *P, hipStream_t s) {
    RedArgs ra = red_args(P, kRz);
    MG_DISPATCH_R(P->R, (k_dot_rz<RR><<<P->n_red, kBlock, 0, s>>>(P->r, P->z, ra, P->sc)));
    return hipGetLastError();
}
hipError_t launch_update_p(const mgpcg_problem *P, hipStream_t s) {
    MG_DISPATCH_R(P->R, (k_update_p<RR><<<P->n_red, kBlock, 0, s>>>(P->z, P->p, P->red_tab, P->sc)));
    return hipGetLastError();
}
hipError_t launch_spmv_pq(const mgpcg_problem *P, hipStream_t s) {
    const Level &L = P->lev[0];
    RedArgs ra = red_args(P, kPq);
    MG_DISPATCH_R(P->R, (k_spmv_pq<RR><<<P->n_red, kBlock, 0, s>>>(L.n, L.val64, L.col, P->p, P->q,
                                                                   ra, P->sc)));
    return hipGetLastError();
}
hipError_t launch_update_xr(const mgpcg_problem *P, double tol, int hist_cap, hipStream_t s) {
    RedArgs ra = red_args(P, kRr);
    MG_DISPATCH_R(P->R, (k_update_xr<RR><<<P->n_red, kBlock, 0, s>>>(P->x, P->p, P->r, P->q, ra, P->sc,
                                                                     P->hist, hist_cap, tol)));
    return hipGetLastError();
}

}  // namespace mg
