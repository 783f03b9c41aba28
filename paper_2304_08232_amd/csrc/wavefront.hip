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
// them by workgroup barriers instead of kernel boundaries.
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

// wavefronts w0 .. w1-1 in one workgroup (blockDim.x >= the padded size of
// each of them): dirs 1 forward, 2 backward, 3 forward and then backward
// (the last wavefront is not repeated: its neighbours did not change, so a
// second update would give the same values)
template <typename T>
__global__ __launch_bounds__(1024) void k_wave_run(const T *__restrict__ wval, const int32_t *__restrict__ wcol,
                                                   const int32_t *__restrict__ wrow, const T *__restrict__ r, T *z,
                                                   const int64_t *__restrict__ woff, int w0, int w1, int dirs) {
    const int nw = w1 - w0;
    const int steps = dirs == 3 ? 2 * nw - 1 : nw;
    for (int k = 0; k < steps; ++k) {
        int w;
        if (dirs == 1) w = w0 + k;
        else if (dirs == 2) w = w1 - 1 - k;
        else w = k < nw ? w0 + k : w1 - 2 - (k - nw);
        const int64_t p = woff[w] + threadIdx.x;
        if (p < woff[w + 1]) {
            const int32_t i = wrow[p];
            if (i >= 0) lex_row<T>(wval, wcol, p, i, r, z);
        }
        __syncthreads();
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
