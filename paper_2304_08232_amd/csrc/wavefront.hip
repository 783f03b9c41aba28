// Sequential symmetric Gauss-Seidel (Sec. II-E, Eq. (1)) on the GPU by level
// scheduling.
//
// Eq. (1) in increasing natural row order makes z_i depend on every updated
// z_j with j < i and a_ij != 0.  For the 27-point stencil those neighbours
// are (dx, dy, dz) with dz = -1, or dz = 0 and dy = -1, or dz = dy = 0 and
// dx = -1.  Give point (ix, iy, iz) the wavefront number t = ix + 2 iy + 4 iz:
// each such neighbour has t' = t + dx + 2 dy + 4 dz < t (the largest value
// of dx + 2 dy with dz = -1 is 3 < 4), and two points of one wavefront are
// never neighbours (dx + 2 dy + 4 dz = 0 forces d = 0).  Sweeping wavefronts
// in increasing t, all rows of a wavefront at once, therefore reproduces the
// sequential forward sweep exactly; decreasing t reproduces the backward one.
//
// A level's rows are kept in a wavefront-major copy of its operator: the rows
// of wavefront t occupy positions woff[t] .. woff[t+1] (padded to a multiple
// of 64, padding positions have row -1), stored as ELL blocked by 64
// positions, so one wavefront of the GPU reads its 27 slots as contiguous
// runs.  Columns and the vectors stay in the library's internal row order.
//
// Large wavefronts get one launch each (one workgroup per 64 rows); runs of
// consecutive small wavefronts are swept by a single workgroup that separates
// them by workgroup barriers instead of kernel boundaries (kRunThreads rows
// at most per wavefront).
#include "kernels.h"

namespace mg {

namespace {

constexpr int kWaveWG = 64;  // threads per workgroup of a single-wavefront launch

// Eq. (1): z_i = (r_i - sum_{j != i} a_ij z_j) / a_ii, the sum over the row's
// slots in ascending column order; padding slots (a = 0) add nothing.
template <typename T>
__device__ __forceinline__ void lex_row(const T *__restrict__ wval, const int32_t *__restrict__ wcol, int64_t p,
                                        int32_t i, const T *__restrict__ r, T *z) {
    T a[kW];
    int32_t c[kW];
#pragma unroll
    for (int s = 0; s < kW; ++s) {
        a[s] = wval[ell_index(s, p)];
        c[s] = wcol[ell_index(s, p)];
    }
    T x[kW];
#pragma unroll
    for (int s = 0; s < kW; ++s) x[s] = s == kCentre ? T(0) : z[c[s]];
    const T rv = r[i];
    T acc = 0;
#pragma unroll
    for (int s = 0; s < kW; ++s)
        if (s != kCentre && a[s] != T(0)) acc = acc + a[s] * x[s];
    z[i] = (rv - acc) / a[kCentre];
}

// the rows of one wavefront: positions [p0, p1)
template <typename T>
__global__ __launch_bounds__(kWaveWG) void k_wave(const T *__restrict__ wval, const int32_t *__restrict__ wcol,
                                                  const int32_t *__restrict__ wrow, const T *__restrict__ r, T *z,
                                                  int64_t p0, int64_t p1) {
    const int64_t p = p0 + (int64_t)blockIdx.x * kWaveWG + threadIdx.x;
    if (p >= p1) return;
    const int32_t i = wrow[p];
    if (i >= 0) lex_row<T>(wval, wcol, p, i, r, z);
}

// ---------------------------------------------------- single-workgroup runs
//
// A run sweeps consecutive small wavefronts in one workgroup of at most
// kRunThreads threads, one row per thread, with a workgroup barrier between
// wavefronts.  It is software-pipelined: while step k updates its wavefront,
// each thread already loads its row of step k+1 and gathers every neighbour
// of that row that step k does not write.  A row's neighbours on the
// wavefront swept just before it (t - 1 going forward, t + 1 going backward)
// are the only ones written by the previous step: dx + 2 dy + 4 dz = -1 has
// the solutions (-1,0,0), (1,-1,0), (1,1,-1), i.e. slots 12, 11, 8, and
// +1 the slots 14, 15, 18.  Those three ("late" slots) are read after the
// barrier.  The sum keeps ascending slot order: the products of the slots
// below the first late slot are summed ahead, the rest are added in order
// once the late values are in.

constexpr int kRunThreads = 512;

__host__ __device__ constexpr int late_slot(bool fwd, int j) {
    return fwd ? (j == 0 ? 8 : j == 1 ? 11 : 12) : (j == 0 ? 14 : j == 1 ? 15 : 18);
}
__host__ __device__ constexpr int late_of(bool fwd, int s) {
    return s == late_slot(fwd, 0) ? 0 : s == late_slot(fwd, 1) ? 1 : s == late_slot(fwd, 2) ? 2 : -1;
}

template <typename T>
struct RawRow {  // a thread's row of the next step, as loaded
    int32_t i;   // internal row, -1: none
    T a[kW];
    int32_t c[kW];
    T x[kW];     // neighbour values of the early slots
    T rv;
};

template <typename T>
struct ReadyRow {  // a row that waits only for its late neighbours
    int32_t i;
    T rv, d, pre;  // pre: sum over the slots below the first late slot
    T p[kW];       // a_s x_s of the early slots above the first late slot
    T al[3];
    int32_t cl[3];
    uint32_t nz;   // slots with a_s != 0
};

template <typename T>
__device__ __forceinline__ void run_load(RawRow<T> &N, const T *__restrict__ wval, const int32_t *__restrict__ wcol,
                                         const int32_t *__restrict__ wrow, int64_t p, bool valid) {
    N.i = valid ? wrow[p] : -1;
    if (N.i < 0) return;
#pragma unroll
    for (int s = 0; s < kW; ++s) {
        N.a[s] = wval[ell_index(s, p)];
        N.c[s] = wcol[ell_index(s, p)];
    }
}

template <typename T, bool FWD>
__device__ __forceinline__ void run_gather(RawRow<T> &N, const T *__restrict__ r, const T *z) {
    if (N.i < 0) return;
#pragma unroll
    for (int s = 0; s < kW; ++s)
        if (s != kCentre && late_of(FWD, s) < 0) N.x[s] = z[N.c[s]];
    N.rv = r[N.i];
}

template <typename T, bool FWD>
__device__ __forceinline__ void run_ready(ReadyRow<T> &R, const RawRow<T> &N) {
    R.i = N.i;
    if (R.i < 0) return;
    constexpr int first = late_slot(FWD, 0);
    R.rv = N.rv;
    R.d = N.a[kCentre];
    uint32_t nz = 0;
    T pre = 0;
#pragma unroll
    for (int s = 0; s < kW; ++s) {
        if (N.a[s] != T(0)) nz |= 1u << s;
        if (s == kCentre) continue;
        if (s < first) {
            if (N.a[s] != T(0)) pre = pre + N.a[s] * N.x[s];
        } else if (late_of(FWD, s) >= 0) {
            R.al[late_of(FWD, s)] = N.a[s];
            R.cl[late_of(FWD, s)] = N.c[s];
        } else {
            R.p[s] = N.a[s] * N.x[s];
        }
    }
    R.nz = nz;
    R.pre = pre;
}

template <typename T, bool FWD>
__device__ __forceinline__ void run_finish(const ReadyRow<T> &R, const T (&xl)[3], T *z) {
    constexpr int first = late_slot(FWD, 0);
    T acc = R.pre;
#pragma unroll
    for (int s = first; s < kW; ++s) {
        if (s == kCentre || !((R.nz >> s) & 1u)) continue;
        const int j = late_of(FWD, s);
        acc = acc + (j >= 0 ? R.al[j] * xl[j] : R.p[s]);
    }
    z[R.i] = (R.rv - acc) / R.d;
}

// wavefronts w0 .. w1-1 (blockDim.x >= the padded size of each of them):
// dirs 1 forward, 2 backward, 3 forward and then backward (the last
// wavefront is not repeated: its neighbours did not change, so a second
// update would give the same values)
template <typename T>
__global__ __launch_bounds__(kRunThreads) void k_wave_run(const T *__restrict__ wval,
                                                          const int32_t *__restrict__ wcol,
                                                          const int32_t *__restrict__ wrow, const T *__restrict__ r,
                                                          T *z, const int64_t *__restrict__ woff, int w0, int w1,
                                                          int dirs) {
    const int nw = w1 - w0;
    const int steps = dirs == 3 ? 2 * nw - 1 : nw;
    auto wave_at = [&](int k) { return dirs == 1 ? w0 + k : dirs == 2 ? w1 - 1 - k : (k < nw ? w0 + k : w1 - 2 - (k - nw)); };
    auto fwd_at = [&](int k) { return dirs == 1 || (dirs == 3 && k < nw); };
    RawRow<T> N;
    ReadyRow<T> R;
    auto load_step = [&](int k) {
        const int w = wave_at(k);
        const int64_t p = woff[w] + threadIdx.x;
        run_load<T>(N, wval, wcol, wrow, p, p < woff[w + 1]);
    };
    auto gather_step = [&](int k) {
        if (fwd_at(k)) run_gather<T, true>(N, r, z);
        else run_gather<T, false>(N, r, z);
    };
    auto ready_step = [&](int k) {
        if (fwd_at(k)) run_ready<T, true>(R, N);
        else run_ready<T, false>(R, N);
    };
    load_step(0);
    gather_step(0);
    ready_step(0);
    for (int k = 0; k < steps; ++k) {
        // late neighbours of this step's row: final since the last barrier
        T xl[3] = {T(0), T(0), T(0)};
        if (R.i >= 0)
#pragma unroll
            for (int j = 0; j < 3; ++j) xl[j] = z[R.cl[j]];
        asm volatile("" ::: "memory");
        const bool more = k + 1 < steps;
        if (more) load_step(k + 1);
        asm volatile("" ::: "memory");
        if (R.i >= 0) {
            if (fwd_at(k)) run_finish<T, true>(R, xl, z);
            else run_finish<T, false>(R, xl, z);
        }
        // early neighbours of the next row: this step writes none of them
        if (more) gather_step(k + 1);
        __syncthreads();
        if (more) ready_step(k + 1);
    }
}

// wavefront-major copy of a level's values (padding positions: identity row)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_wave_gather(const int32_t *__restrict__ wrow, const T *__restrict__ val,
                                                        T *__restrict__ wval, int64_t npos) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= npos) return;
    const int32_t i = wrow[p];
#pragma unroll
    for (int s = 0; s < kW; ++s)
        wval[ell_index(s, p)] = i >= 0 ? val[ell_index(s, i)] : (s == kCentre ? T(1) : T(0));
}

hipError_t launch_segment(const mgpcg_problem *P, const Level &L, const WaveSeg &g, int dirs, const double *r,
                          double *z, hipStream_t s) {
    const double *wval = L.wval;
    if (g.run) {
        if (g.threads > kRunThreads || g.threads % kEllRows) return hipErrorInvalidConfiguration;
        k_wave_run<double><<<1, g.threads, 0, s>>>(wval, L.wcol, L.wrow, r, z, L.woff_dev, g.w0, g.w1, dirs);
    } else {
        const int64_t p0 = L.woff[g.w0], p1 = L.woff[g.w0 + 1];
        const int nb = (int)((p1 - p0 + kWaveWG - 1) / kWaveWG);
        if (nb > 0) k_wave<double><<<nb, kWaveWG, 0, s>>>(wval, L.wcol, L.wrow, r, z, p0, p1);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_wave_gather(const mgpcg_problem *P, int level, hipStream_t s) {
    const Level &L = P->lev[level];
    if (L.npos == 0) return hipSuccess;
    k_wave_gather<double><<<(int)((L.npos + kBlock - 1) / kBlock), kBlock, 0, s>>>(L.wrow, L.val64, L.wval, L.npos);
    return hipGetLastError();
}

// One symmetric sweep: the segments of the plan forward, then backward.
hipError_t launch_lex_sweep(const mgpcg_problem *P, int level, const double *r, double *z, hipStream_t s) {
    const Level &L = P->lev[level];
    const int ns = (int)L.wplan.size();
    if (ns == 0) return hipSuccess;
    hipError_t e;
    // a final run does its forward and backward sweep in one launch
    const bool merge = L.wplan[ns - 1].run;
    for (int q = 0; q < ns; ++q) {
        const bool last = q == ns - 1;
        if ((e = launch_segment(P, L, L.wplan[q], last && merge ? 3 : 1, r, z, s)) != hipSuccess) return e;
    }
    // a final single wavefront is not repeated either
    for (int q = ns - 2; q >= 0; --q)
        if ((e = launch_segment(P, L, L.wplan[q], 2, r, z, s)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace mg
