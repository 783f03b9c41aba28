// gfx950 kernels of the MG-PCG hot path.
//
// Every kernel is bound by HBM bandwidth (about 0.16 flop per byte) or, on the
// small levels, by latency.  The design goals: stream the ELL operator once
// per pass in wavefront-contiguous blocks (non-temporal loads on levels larger
// than the caches) with the column data as compact as the level allows; issue
// a row's neighbour gathers as soon as its columns are known; hand each XCD a
// contiguous range of rows so that its gathers hit its own L2; and make every
// reduction deterministic (fixed-shape wave/LDS trees, then a one-workgroup
// finalize per grid that sums the partials in a fixed order).
//
// Floating-point contraction is disabled for this library, so that the
// per-row arithmetic is exactly the sequence of IEEE operations the method
// states: sums over the row in ascending column order, the Gauss-Seidel update
// (r - s + z*d)/d with a true division, and the CG vector updates.
#include "kernels.h"

namespace mg {

namespace {

constexpr int kXcd = kXcdCount;  // XCDs per MI355X; workgroups are dealt round-robin

// Workgroup b of nb is dispatched to XCD b % 8.  Return the logical block so
// that each XCD receives one contiguous range of logical blocks.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    int per = nb / kXcd, rem = nb % kXcd;
    int x = b % kXcd, q = b / kXcd;
    return x * per + (x < rem ? x : rem) + q;
}

// Kernel arguments arrive by scalar loads, which complete out of order, so
// each use of one waits for every scalar load issued before it.  Left alone,
// the compiler issues the arguments in the groups the code needs next, with a
// wait after each group: several round trips before a kernel's first memory
// load.  Naming the arguments the first loads need in one empty asm statement
// at the top makes it issue all of them before the first wait.  (Naming
// every argument instead was slower: the compiler then reloads some of them
// one word at a time.)
#define MG_ARGS_FIRST(...) asm volatile("" ::__VA_ARGS__)
// the upper column bases (the lower 16 come in one wide load anyway)
#define MG_BASES_FIRST(B)                                                                            \
    asm volatile("" ::"s"((B).v[16]), "s"((B).v[17]), "s"((B).v[18]), "s"((B).v[19]), "s"((B).v[20]), \
                 "s"((B).v[21]), "s"((B).v[22]), "s"((B).v[23]), "s"((B).v[24]), "s"((B).v[25]),      \
                 "s"((B).v[26]))

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

// colour row ranges of a level, passed by value
struct CoffTable {
    int64_t coff[9];
    int ncol;
};
inline CoffTable coff_table(const Level &L) {
    CoffTable t;
    t.ncol = L.ncol;
    for (int k = 0; k <= 8; ++k) t.coff[k] = L.coff[k < L.ncol ? k : L.ncol];
    return t;
}

// Load helper: streaming (non-temporal) loads for operators far larger than
// the caches, ordinary loads otherwise so that coarse operators stay resident.
template <bool NT, typename T>
__device__ __forceinline__ T ld(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// The 27 column bases of one colour, passed by value in the kernel arguments
// of a colour pass (no separate load of the base table).
struct Base27 {
    int32_t v[27];
    __device__ __forceinline__ int32_t operator[](int s) const { return v[s]; }
};

// The stored operator of one row, as loaded: the 27 values (0 for padding
// slots and for slots in a compile-time SKIP mask) and the column data in
// storage form (packed 8-bit deltas, or 32-bit columns).  Keeping the raw
// words lets a load be in flight across a barrier: nothing uses them until
// the columns are decoded.
template <typename T, int CF>
struct RawRow {
    T a[kW];
    uint32_t w[CF ? kDeltaWords : kW];
};

template <uint32_t SKIP, int q>
constexpr bool word_needed() {
    // a word of deltas is needed if any of its real slots is read
    return ((~SKIP >> (4 * q)) & 0xFu & ((1u << (kW - 4 * q < 4 ? kW - 4 * q : 4)) - 1u)) != 0u;
}

// The column data are loaded first: the gathers need only them (not the
// values), so they can leave while the value loads are still streaming.
// VS: the values were staged in LDS by the workgroup; slot s of this row is
// at vs[s * vstride].
template <typename T, uint32_t SKIP, bool NT, int CF, bool VS = false>
__device__ __forceinline__ void load_raw(const T *__restrict__ val, const int32_t *__restrict__ col,
                                         const int8_t *__restrict__ dcol, int64_t i, RawRow<T, CF> &rw,
                                         const T *vs = nullptr, int vstride = 0) {
    if constexpr (CF == 2) {
        // every delta is zero: the columns are implied by the bases
#pragma unroll
        for (int q = 0; q < kDeltaWords; ++q) rw.w[q] = 0u;
    } else if constexpr (CF == 1) {
        const uint32_t *dw = (const uint32_t *)dcol;
#define MG_LOAD_WORD(q) rw.w[q] = word_needed<SKIP, q>() ? ld<NT>(dw + delta_word(q, i)) : 0u;
        MG_LOAD_WORD(0) MG_LOAD_WORD(1) MG_LOAD_WORD(2) MG_LOAD_WORD(3)
        MG_LOAD_WORD(4) MG_LOAD_WORD(5) MG_LOAD_WORD(6)
#undef MG_LOAD_WORD
    } else {
#pragma unroll
        for (int s = 0; s < kW; ++s) {
            const bool sk = (SKIP >> s) & 1u;
            rw.w[s] = sk ? 0u : (uint32_t)ld<NT>(col + ell_index(s, i));
        }
    }
#pragma unroll
    for (int s = 0; s < kW; ++s) {
        const bool sk = (SKIP >> s) & 1u;
        if constexpr (VS) rw.a[s] = (!sk || s == kCentre) ? vs[s * vstride] : T(0);
        else rw.a[s] = (!sk || s == kCentre) ? ld<NT>(val + ell_index(s, i)) : T(0);
    }
}

// absolute column of slot s of row i
template <int CF, typename T, class SB>
__device__ __forceinline__ int32_t slot_col(const RawRow<T, CF> &rw, const SB &sb, int64_t i, int s) {
    if constexpr (CF) {
        const int32_t dl = (int32_t)(rw.w[s / 4] << (24 - 8 * (s % 4))) >> 24;  // sign-extended byte
        return (int32_t)(i + sb[s] + dl);
    } else {
        return (int32_t)rw.w[s];
    }
}

// Absolute columns of the row (0 for skipped slots), each a valid row of the
// level: a padding slot's delta-coded column (i + base) may fall outside
// [0, n), so delta-coded columns are clamped.  Real columns are unchanged
// by the clamp; a padding slot's gather then reads some valid row and its
// value is never used (the sums skip slots whose value is 0).
template <uint32_t SKIP, int CF, typename T, class SB>
__device__ __forceinline__ void decode_cols(const RawRow<T, CF> &rw, const SB &sb, int64_t n, int64_t i,
                                            int32_t (&c)[kW]) {
#pragma unroll
    for (int s = 0; s < kW; ++s) {
        int32_t cs = ((SKIP >> s) & 1u) ? 0 : slot_col<CF>(rw, sb, i, s);
        if constexpr (CF) cs = min(max(cs, 0), (int32_t)(n - 1));
        c[s] = cs;
    }
}

// Operator values a[s] and absolute columns c[s] of the 27 slots of row i.
// All value and column loads of the row are issued before anything uses
// them: 27 value loads plus 7 delta words (int8 deltas), 27 columns (int32),
// or none (implied columns, whose gathers can then leave at once).
template <typename T, int R, uint32_t SKIP, bool NT, int CF, class SB, bool VS = false>
__device__ __forceinline__ void load_slots(const T *__restrict__ val, const int32_t *__restrict__ col,
                                           const int8_t *__restrict__ dcol, const SB &sb, int64_t n, int64_t i,
                                           T (&a)[kW], int32_t (&c)[kW], const T *vs = nullptr,
                                           int vstride = 0) {
    RawRow<T, CF> rw;
    load_raw<T, SKIP, NT, CF, VS>(val, col, dcol, i, rw, vs, vstride);
#pragma unroll
    for (int s = 0; s < kW; ++s) a[s] = rw.a[s];
    decode_cols<SKIP, CF>(rw, sb, n, i, c);
}

// x at the 27 columns (0 for skipped slots).  The gathers depend on the
// columns only, not on the values: a padding slot gathers a valid row whose
// value the sums ignore.
template <typename T, int R, uint32_t SKIP>
__device__ __forceinline__ void gather_slots(const T *x, int v, const T (&a)[kW], const int32_t (&c)[kW],
                                             T (&xv)[kW]) {
    (void)a;
#pragma unroll
    for (int s = 0; s < kW; ++s) {
        const bool sk = (SKIP >> s) & 1u;
        xv[s] = !sk ? x[(int64_t)c[s] * R + v] : T(0);
    }
}

// Operator values a[s] and x at the columns xv[s] of row i.  The column
// words are loaded first and the gathers leave as soon as they arrive, while
// the value loads are still streaming.  (Predicting the columns and gathering
// together with the operator loads, with a check afterwards, was measured
// slower on the latency-bound levels: ~4.45 against ~4.0 us per level-2 pass.)
template <typename T, int R, uint32_t SKIP, bool NT, int CF, class SB, bool VS = false>
__device__ __forceinline__ void load_row(const T *__restrict__ val, const int32_t *__restrict__ col,
                                         const int8_t *__restrict__ dcol, const SB &sb, int64_t n, int64_t i,
                                         const T *x, int v, T (&a)[kW], T (&xv)[kW], const T *vs = nullptr,
                                         int vstride = 0) {
    int32_t c[kW];
    load_slots<T, R, SKIP, NT, CF, SB, VS>(val, col, dcol, sb, n, i, a, c, vs, vstride);
    gather_slots<T, R, SKIP>(x, v, a, c, xv);
}

// sum_j a_ij x_j over the 27 slots of row i, in slot order (ascending natural
// column order), skipping padding slots (value 0).  Slots whose bit is set in
// the compile-time SKIP mask are left out entirely (their x is known to be
// zero); the diagonal value is always loaded and returned in d.
template <typename T, int R, uint32_t SKIP, bool NT, int CF, bool VS = false, class SB = const int32_t *>
__device__ __forceinline__ T row_sum(const T *__restrict__ val, const int32_t *__restrict__ col,
                                     const int8_t *__restrict__ dcol, const SB &sb, int64_t n,
                                     int64_t i, const T *x, int v, T &d, const T *vs = nullptr, int vstride = 0) {
    T a[kW], xv[kW];
    load_row<T, R, SKIP, NT, CF, SB, VS>(val, col, dcol, sb, n, i, x, v, a, xv, vs, vstride);
    d = a[kCentre];
    T acc = 0;
#pragma unroll
    for (int s = 0; s < kW; ++s) {
        const bool sk = (SKIP >> s) & 1u;
        if (!sk && a[s] != T(0)) acc = acc + a[s] * xv[s];
    }
    return acc;
}

// With R >= kStageR right-hand sides, R lanes share each row: rather than
// each loading the row's 27 values (R times the address work for the same
// bytes, which made these kernels bound by address processing), the
// workgroup stages the values of its `rows` rows (from row0, `count` of them
// real) in LDS with coalesced loads, slot-major: slot s of row j at
// sv[s * rows + j].  Slots in SKIP (other than the diagonal) are not loaded,
// and nothing reads them.  Ends with a workgroup barrier.  With R = 2 the
// buffer (27 x 128 rows) costs more occupancy than the halved loads save.
constexpr int kStageR = 4;
// A thread's share (at most N = ceil(27 ROWS / BS) words) is loaded into
// registers first and written to LDS afterwards, so that all its loads are in
// flight together; words of rows past `count` and of skipped slots are
// written as 0 and never read.
template <typename T, uint32_t SKIP, bool NT, int ROWS, int BS>
__device__ __forceinline__ void stage_values(const T *__restrict__ val, int64_t row0, int64_t count, T *sv) {
    constexpr int N = (kW * ROWS + BS - 1) / BS;
    T w[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
        const int e = threadIdx.x + u * BS;
        const int s = e / ROWS, j = e - s * ROWS;
        const bool need = e < kW * ROWS && (!((SKIP >> (s & 31)) & 1u) || s == kCentre) && j < count;
        w[u] = need ? ld<NT>(val + ell_index(s, row0 + j)) : T(0);
    }
#pragma unroll
    for (int u = 0; u < N; ++u) {
        const int e = threadIdx.x + u * BS;
        if (e < kW * ROWS) sv[e] = w[u];
    }
    __syncthreads();
}

// colour of row i from the colour ranges (at most 8)
__device__ __forceinline__ int colour_of(const int64_t *coff, int ncol, int64_t i) {
    int k = 0;
    while (k + 1 < ncol && i >= coff[k + 1]) ++k;
    return k;
}

// Zero-start skip mask of colour k for the standard colouring of grids whose
// extents are all >= 2: colour number c has parity code c (order 0) or 7-c
// (order 1), the neighbour in direction d has parity code pc ^ parity(d), and
// a slot is skipped when that neighbour's colour number is >= k (not yet
// written in the forward sweep; this includes the diagonal).
constexpr uint32_t zs_mask(int k, int order) {
    uint32_t m = 0;
    const int pc = order ? 7 - k : k;
    for (int s = 0; s < kW; ++s) {
        const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
        const int pd = (dx != 0 ? 1 : 0) | (dy != 0 ? 2 : 0) | (dz != 0 ? 4 : 0);
        const int nb = pc ^ pd;
        const int nbc = order ? 7 - nb : nb;
        if (nbc >= k) m |= 1u << s;
    }
    return m;
}

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
        int64_t e = ell_index(s, i);
        if (val64) val64[e] = v;
        if (val32) val32[e] = (float)v;
        if (col) col[e] = c;
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

// Delta-code the columns of one (single-grid) level: dcol = col - i - base,
// for real entries only.  flags[0]: some delta does not fit in int8;
// flags[1]: some real entry has a nonzero delta (both reduced per wave
// before one atomic each).
__global__ __launch_bounds__(kBlock) void k_delta_encode(int64_t n, const double *__restrict__ val64,
                                                         const float *__restrict__ val32,
                                                         const int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ base,
                                                         const int64_t *__restrict__ coff, int ncol,
                                                         const int32_t *__restrict__ grow,
                                                         int8_t *__restrict__ dcol, int *__restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool bad = false, nonzero = false;
    if (i < n) {
        const int k = colour_of(coff, ncol, i);
        const int32_t *b = base + ((grow ? grow[i] : 0) * 8 + k) * kW;
#pragma unroll
        for (int s = 0; s < kW; ++s) {
            const int64_t e = ell_index(s, i);
            const bool real = val64 ? val64[e] != 0.0 : val32[e] != 0.0f;
            int64_t dlt = real ? (int64_t)col[e] - i - b[s] : 0;
            nonzero = nonzero || dlt != 0;
            if (dlt < -128 || dlt > 127) {
                bad = true;
                dlt = 0;
            }
            dcol[4 * delta_word(s / 4, i) + s % 4] = (int8_t)dlt;
        }
    }
    const bool any_bad = __any(bad), any_nonzero = __any(nonzero);
    if ((threadIdx.x & 63) == 0) {
        if (any_bad) atomicOr(&flags[0], 1);
        if (any_nonzero) atomicOr(&flags[1], 1);
    }
}

hipError_t launch_delta_encode(const mgpcg_problem *P, int level, const int64_t *coff_dev, int *flags,
                               hipStream_t s) {
    const Level &L = P->lev[level];
    if (L.n == 0) return hipSuccess;
    k_delta_encode<<<nblocks(L.n), kBlock, 0, s>>>(L.n, L.val64, L.val32, L.col, L.dbase, coff_dev, L.ncol,
                                                   L.grid_of_row, L.dcol, flags);
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
template <typename T, int R, int CF>
__global__ __launch_bounds__(kBlock) void k_spmv(int64_t n, const T *__restrict__ val,
                                                 const int32_t *__restrict__ col, const int8_t *__restrict__ dcol,
                                                 const int32_t *__restrict__ dbase,
                                                 const int32_t *__restrict__ grow, CoffTable ct,
                                                 const T *__restrict__ x, T *__restrict__ y) {
    int64_t gid = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (gid >= n * R) return;
    int64_t i = gid / R;
    int v = (int)(gid % R);
    const int32_t *sb = CF ? dbase + ((grow ? grow[i] : 0) * 8 + colour_of(ct.coff, ct.ncol, i)) * kW : nullptr;
    T d;
    y[gid] = row_sum<T, R, 0u, true, CF>(val, col, dcol, sb, n, i, x, v, d);
}

template <int R, int CF, bool PQ>
__global__ void k_spmv_pq(int64_t n, const double *__restrict__ val, const int32_t *__restrict__ col,
                          const int8_t *__restrict__ dcol, const int32_t *__restrict__ dbase,
                          const double *__restrict__ p, double *__restrict__ q, const Seg *__restrict__ tab,
                          double *__restrict__ partials, const int *__restrict__ done, int spc);

template <int R, bool PQ>
__global__ void k_spmv_box(const double *__restrict__ val, const double *__restrict__ p, double *__restrict__ q,
                           double *__restrict__ partials, BoxGeo g);

// the box-tiled level-0 product (P->box_ok); PQ: with the <p, q> partials
template <bool PQ>
hipError_t launch_spmv_box(const mgpcg_problem *P, const double *p, double *q, hipStream_t s) {
    const double *val = P->lev[0].val64;
    double *parts = PQ ? P->sc.partials : nullptr;
    switch (P->R) {
        case 4: k_spmv_box<4, PQ><<<P->n_box, kBlock, 0, s>>>(val, p, q, parts, P->box); break;
        case 8: k_spmv_box<8, PQ><<<P->n_box, kBlock, 0, s>>>(val, p, q, parts, P->box); break;
        case 16: k_spmv_box<16, PQ><<<P->n_box, kBlock, 0, s>>>(val, p, q, parts, P->box); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spmv(const mgpcg_problem *P, int level, const T *val, const T *x, T *y, hipStream_t s) {
    const Level &L = P->lev[level];
    int64_t work = L.n * P->R;
    if (work == 0) return hipSuccess;
    if constexpr (sizeof(T) == 8) {
        // level 0, one grid, R >= 4 on a box-tiled geometry: the CG product
        // kernel without its dot
        if (level == 0 && P->box_ok && (const void *)val == (const void *)L.val64)
            return launch_spmv_box<false>(P, x, y, s);
        // level 0, one grid, one rhs: the CG product kernel without its dot
        if (level == 0 && P->G == 1 && P->R == 1 && (const void *)val == (const void *)L.val64) {
#define MG_SPMV0(CFV)                                                                                   \
    k_spmv_pq<1, CFV, false><<<P->n_red[0], kBlock, 0, s>>>(L.n, L.val64, L.col, L.dcol, L.dbase, x, y,    \
                                                            P->red_tab[0], nullptr, nullptr, P->spc);
            if (L.cf == 2) { MG_SPMV0(2) } else if (L.cf == 1) { MG_SPMV0(1) } else { MG_SPMV0(0) }
#undef MG_SPMV0
            return hipGetLastError();
        }
    }
    const CoffTable ct = coff_table(L);
#define MG_SPMV(CFV)                                                                                   \
    MG_DISPATCH_R(P->R, (k_spmv<T, RR, CFV><<<nblocks(work), kBlock, 0, s>>>(L.n, val, L.col, L.dcol, L.dbase, \
                                                                            L.grid_of_row, ct, x, y)));
    if (L.cf == 2) { MG_SPMV(2) } else if (L.cf == 1) { MG_SPMV(1) } else { MG_SPMV(0) }
#undef MG_SPMV
    return hipGetLastError();
}
template hipError_t launch_spmv<double>(const mgpcg_problem *, int, const double *, const double *,
                                        double *, hipStream_t);
template hipError_t launch_spmv<float>(const mgpcg_problem *, int, const float *, const float *,
                                       float *, hipStream_t);

// ------------------------------------------------------------ colour pass

// sum_s a[s] x(s) in slot order over the real slots not in SKIP; x(s) is the
// neighbour value of slot s (gathered into registers, or read from LDS)
// (CHUNK < 27: x fetches its values CHUNK slots at a time through
// x.load(first slot), which bounds the registers they occupy; the sum is
// the same)
template <typename T, uint32_t SKIP, int CHUNK = kW, class X>
__device__ __forceinline__ T row_dot(const T (&a)[kW], X &x) {
    T acc = 0;
#pragma unroll
    for (int s = 0; s < kW; ++s) {
        if constexpr (CHUNK < kW)
            if (s % CHUNK == 0) x.load(s);
        const bool sk = (SKIP >> s) & 1u;
        if (!sk && a[s] != T(0)) acc = acc + a[s] * x(s);
        if constexpr (CHUNK < kW)
            if (s % CHUNK == CHUNK - 1 || s == kW - 1) asm volatile("" ::: "memory");
    }
    return acc;
}

// Gauss-Seidel update of one row (Eq. (1) in the masked-product form of
// Sec. III-A): z_i = (r_i - sum_j a_ij z_j + z_i d_i) / d_i, where the sum
// runs over the whole row including the diagonal (x(kCentre) = z_i, or
// skipped on a zero start).
template <typename T, uint32_t SKIP, int CHUNK = kW, class X>
__device__ __forceinline__ T gs_update(const T (&a)[kW], X &&x, T rv, T zi) {
    const T d = a[kCentre];
    return (rv - row_dot<T, SKIP, CHUNK>(a, x) + zi * d) / d;
}

// The same colour once more (first pass of the backward sweep right after
// the last pass of the forward sweep): same neighbours, the new z_i on the
// diagonal, the full row in slot order.
template <typename T, class X>
__device__ __forceinline__ T gs_again(const T (&a)[kW], const X &x, T rv, T znew) {
    return gs_update<T, 0u>(a, [&](int s) { return s == kCentre ? znew : x(s); }, rv, znew);
}

// wave-shuffle + LDS tree of per-rhs sums over a workgroup of BS threads;
// thread v < R gets the total of rhs v
template <int R, int BS = kBlock>
__device__ __forceinline__ double block_sum(double acc, double *sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= R; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __syncthreads();
    if (lane < R) sh[w * R + lane] = acc;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < R) {
        t = sh[threadIdx.x];
#pragma unroll
        for (int k = 1; k < BS / 64; ++k) t += sh[k * R + threadIdx.x];
    }
    return t;
}

template <int R, int BS = kBlock>
__device__ __forceinline__ void store_partial(double acc, int blk, double *partials) {
    __shared__ double sh[(BS / 64) * R];
    const double t = block_sum<R, BS>(acc, sh);
    if (threadIdx.x < R) partials[(int64_t)blk * R + threadIdx.x] = t;
}

// Per-workgroup partials of the paired-lane kernels (R >= kPairR, R/2 lanes
// per row, BS threads): lane w holds the sums of right-hand sides 2w and
// 2w+1; partials are written to partials[blk * R + rhs] like store_partial's.
template <int R, int BS = kBlock>
__device__ __forceinline__ void store_partial2(double acc0, double acc1, int blk, double *partials) {
    constexpr int LN = pass_lanes(R);
    __shared__ double sh[(BS / 64) * R];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= LN; off >>= 1) {
        acc0 += __shfl_xor(acc0, off, 64);
        acc1 += __shfl_xor(acc1, off, 64);
    }
    __syncthreads();
    if (lane < LN) {
        sh[wv * R + 2 * lane] = acc0;
        sh[wv * R + 2 * lane + 1] = acc1;
    }
    __syncthreads();
    if (threadIdx.x < R) {
        double t = sh[threadIdx.x];
#pragma unroll
        for (int k = 1; k < BS / 64; ++k) t += sh[k * R + threadIdx.x];
        partials[(int64_t)blk * R + threadIdx.x] = t;
    }
}

// One colour of the coloured Gauss-Seidel pass (Listing 3 of the paper, the
// masked product and the update fused).  Rows of one colour are independent,
// so the update is done in place: a row reads only other colours and itself.
//
// SKIP != 0 (zero start): z is all zeros before this sweep, so only
// neighbours already written in this sweep (colours < k) are read and z_i
// itself is taken as 0; the z array needs no clearing.
//
// MODE 1 (last pass of the pre-smoother when the colour swept last is the
// injection set): after its update, each row is an injection point whose
// neighbours are final, so the thread also forms the restricted residual
// rc = r_i - sum_j a_ij z_j (new z_i at the centre, same slot order as a
// separate residual pass) and writes it to the coarse level.
// MODE 2 (first pass of the post-smoother, same condition): the refinement
// z_i += zc is applied on the fly; the rows of this colour are the only
// readers of the refined values.
//
// Rows come from the segment table when the problem has several grids;
// otherwise workgroup b owns rows [row_base + b*rows, ...) of the colour.
// The update of one (row, rhs) of the pass; shared by the per-pass kernel
// and the persistent coarse-level kernel.  inj_base is the first row of the
// colour (the injection rows start there in MODE 1/2).  dflag (may be NULL)
// is the system's convergence flag: it is loaded with the operator and only
// the stores wait for it, so a pass does not begin with a round trip.  (The
// launches pass NULL: with one grid z is internal, with several a converged
// grid's workgroups return before.  The path stays: without it the compiler
// schedules the latency-bound passes differently, ~11 us per 128^3 CG
// iteration slower, measured.)
// Returns r_i times the stored z_i when DOT (for <r, z>), else 0.
template <typename T, int R, uint32_t SKIP, bool NT, int MODE, int CF, class SB, bool TWICE = false,
          bool DOT = false, bool VS = false>
__device__ __forceinline__ double pass_row(int64_t n, const T *__restrict__ val, const int32_t *__restrict__ col,
                                         const int8_t *__restrict__ dcol, const SB &sb,
                                         const T *__restrict__ r, T *z, int64_t i, int v, int64_t inj_base,
                                         T *__restrict__ coarse, const int32_t *__restrict__ inj_coarse,
                                         const int *__restrict__ dflag = nullptr, const T *vs = nullptr,
                                         int vstride = 0) {
    const int64_t o = i * R + v;
    const int dv = dflag ? *dflag : 0;
    // the transfer map and the coarse value travel with the operator loads
    // and the gathers, so none of them adds a round trip of its own
    const T rv = r[o];
    int64_t co = 0;
    if (MODE != 0) co = (int64_t)inj_coarse[i - inj_base] * R + v;
    T a[kW], xv[kW];
    load_row<T, R, SKIP, NT, CF, SB, VS>(val, col, dcol, sb, n, i, z, v, a, xv, vs, vstride);
    T zc = T(0);
    if (MODE == 2) zc = coarse[co];
    // z_i before this pass (refined in MODE 2); 0 on a zero start
    const T zi = SKIP ? T(0) : (MODE == 2 ? xv[kCentre] + zc : xv[kCentre]);
    if (MODE == 2) xv[kCentre] = zi;
    const auto x = [&](int s) { return xv[s]; };
    const T znew = gs_update<T, SKIP>(a, x, rv, zi);
    if (dv) return 0.0;  // converged system: leave its vectors alone
    if constexpr (TWICE) {
        const T z2 = gs_again(a, x, rv, znew);
        z[o] = z2;
        return DOT ? (double)rv * (double)z2 : 0.0;
    }
    z[o] = znew;
    if (MODE == 1) {
        xv[kCentre] = znew;
        coarse[co] = rv - row_dot<T, 0u>(a, x);
    }
    return DOT ? (double)rv * (double)znew : 0.0;
}

// N consecutive values (N = 1 or 2) as one access
template <typename T, int N>
__device__ __forceinline__ void ld_lanes(const T *p, T (&v)[N]) {
    if constexpr (N == 2) {
        typedef T V2 __attribute__((ext_vector_type(2)));
        const V2 t = *(const V2 *)p;
        v[0] = t.x;
        v[1] = t.y;
    } else {
        v[0] = *p;
    }
}
template <typename T, int N>
__device__ __forceinline__ void st_lanes(T *p, const T (&v)[N]) {
    if constexpr (N == 2) {
        typedef T V2 __attribute__((ext_vector_type(2)));
        *(V2 *)p = V2{v[0], v[1]};
    } else {
        *p = v[0];
    }
}

// The update of one row for two right-hand sides (2w and 2w+1) in one lane
// (R >= kPairR, values staged in LDS): r, z, the gathers and the coarse
// values move as 16-byte pairs, which halves the per-lane address work of a
// pass whose texture unit is otherwise its bottleneck.  Each right-hand
// side's arithmetic is exactly pass_row's.
// DOT: rz[u] = r times the stored z of right-hand side 2w+u (for <r, z>).
template <typename T, int R, uint32_t SKIP, bool NT, int MODE, int CF, class SB, bool TWICE, bool DOT = false>
__device__ __forceinline__ void pass_row2(int64_t n, const int32_t *__restrict__ col,
                                          const int8_t *__restrict__ dcol, const SB &sb, const T *__restrict__ r,
                                          T *z, int64_t i, int w, int64_t inj_base, T *__restrict__ coarse,
                                          const int32_t *__restrict__ inj_coarse, const T *vs, int vstride,
                                          double (&rz)[2]) {
    typedef T V2 __attribute__((ext_vector_type(2)));
    const int64_t o = i * R + 2 * w;
    const V2 rv = *(const V2 *)(r + o);
    int64_t co = 0;
    if (MODE != 0) co = (int64_t)inj_coarse[i - inj_base] * R + 2 * w;
    T a[kW];
    int32_t c[kW];
    load_slots<T, R, SKIP, NT, CF, SB, true>(nullptr, col, dcol, sb, n, i, a, c, vs, vstride);
    V2 xv[kW];
#pragma unroll
    for (int s = 0; s < kW; ++s) {
        const bool sk = (SKIP >> s) & 1u;
        xv[s] = !sk ? *(const V2 *)(z + (int64_t)c[s] * R + 2 * w) : V2{T(0), T(0)};
    }
    V2 zc = {T(0), T(0)};
    if (MODE == 2) zc = *(const V2 *)(coarse + co);
    V2 zi = SKIP ? V2{T(0), T(0)} : (MODE == 2 ? xv[kCentre] + zc : xv[kCentre]);
    if (MODE == 2) xv[kCentre] = zi;
    const auto x0 = [&](int s) { return xv[s].x; };
    const auto x1 = [&](int s) { return xv[s].y; };
    V2 zn;
    zn.x = gs_update<T, SKIP>(a, x0, rv.x, zi.x);
    zn.y = gs_update<T, SKIP>(a, x1, rv.y, zi.y);
    if constexpr (TWICE) {
        V2 z2;
        z2.x = gs_again(a, x0, rv.x, zn.x);
        z2.y = gs_again(a, x1, rv.y, zn.y);
        *(V2 *)(z + o) = z2;
        if (DOT) {
            rz[0] = (double)rv.x * (double)z2.x;
            rz[1] = (double)rv.y * (double)z2.y;
        }
        return;
    }
    *(V2 *)(z + o) = zn;
    if (DOT) {
        rz[0] = (double)rv.x * (double)zn.x;
        rz[1] = (double)rv.y * (double)zn.y;
    }
    if (MODE == 1) {
        xv[kCentre] = zn;
        V2 rc;
        rc.x = rv.x - row_dot<T, 0u>(a, x0);
        rc.y = rv.y - row_dot<T, 0u>(a, x1);
        *(V2 *)(coarse + co) = rc;
    }
}

// DOT (one grid, no table): each workgroup also writes the sum of r_i z_i
// over its rows to rzp[b * R + rhs].
template <typename T, int R, uint32_t SKIP, bool NT, int MODE, int CF, bool TWICE = false, bool DOT = false>
__global__ __launch_bounds__(pass_block(NT)) void k_pass(int64_t n, const T *__restrict__ val,
                                                 const int32_t *__restrict__ col, const int8_t *__restrict__ dcol,
                                                 const Base27 sb_arg,
                                                 const T *__restrict__ r, T *z,
                                                 const Seg *__restrict__ tab, int64_t row_base,
                                                 int64_t row_end, const int *__restrict__ done,
                                                 T *__restrict__ coarse, const int32_t *__restrict__ inj_coarse,
                                                 double *__restrict__ rzp, const int32_t *__restrict__ gbase) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    // every argument the first loads need, in one batch (see MG_ARGS_FIRST)
    MG_ARGS_FIRST("s"(n), "s"(val), "s"(r), "s"(z), "s"(tab), "s"(row_base), "s"(row_end), "s"(done));
    if constexpr (CF != 0) MG_BASES_FIRST(sb_arg);
    int64_t row0, count;
    int grid;
    Base27 sb = sb_arg;
    if (tab) {
        const Seg e = tab[b];
        row0 = e.row0;
        count = e.count;
        grid = e.grid;
        // several grids: the bases of this segment's grid and colour
        if (CF && gbase) {
            const int32_t *gb = gbase + (e.grid * 8 + e.colour) * kW;
#pragma unroll
            for (int t = 0; t < kW; ++t) sb.v[t] = gb[t];
        }
    } else {
        row0 = row_base + (int64_t)b * pass_rows(NT, R);
        count = row_end - row0;
        grid = 0;
    }
    if constexpr (R >= kPairR) {
        // R/2 lanes per row, two right-hand sides each; the workgroup's
        // values go through LDS once
        constexpr int LN = pass_lanes(R), RW = pass_rows(NT, R);
        __shared__ T sv[kW * RW];
        const int rl = threadIdx.x / LN, w = threadIdx.x % LN;
        if (tab && done) {  // a grid whose systems are all converged: uniform, before the barrier
            bool all = true;
#pragma unroll
            for (int u = 0; u < R; ++u) all = all && done[grid * R + u];
            if (all) return;
        }
        stage_values<T, SKIP, NT, RW, pass_block(NT)>(val, row0, count, sv);
        double rz[2] = {0.0, 0.0};
        // several grids: a lane whose two systems have both converged stores
        // nothing (z is internal: a converged system's z is never used again)
        if (rl < count && !(tab && done && done[grid * R + 2 * w] && done[grid * R + 2 * w + 1]))
            pass_row2<T, R, SKIP, NT, MODE, CF, Base27, TWICE, DOT>(n, col, dcol, sb, r, z, row0 + rl, w, row_base,
                                                                    coarse, inj_coarse, sv + rl, RW, rz);
        // DOT (one grid, no table): every thread takes part in the sum
        if constexpr (DOT) store_partial2<R, pass_block(NT)>(rz[0], rz[1], b, rzp);
        return;
    }
    const int rl = threadIdx.x / R, v = threadIdx.x % R;
    if constexpr (DOT) {
        // every thread takes part in the workgroup's sum
        double rz = 0.0;
        if (rl < count)
            rz = pass_row<T, R, SKIP, NT, MODE, CF, Base27, TWICE, true>(
                n, val, col, dcol, sb, r, z, row0 + rl, v, row_base, coarse, inj_coarse, done ? done + v : nullptr);
        store_partial<R, pass_block(NT)>(rz, b, rzp);
    } else if constexpr (R >= kStageR) {
        // R lanes per row: the workgroup's values go through LDS once
        constexpr int RW = pass_block(NT) / R;
        __shared__ T sv[kW * RW];
        if (tab && done) {  // a grid whose systems are all converged: uniform, before the barrier
            bool all = true;
#pragma unroll
            for (int u = 0; u < R; ++u) all = all && done[grid * R + u];
            if (all) return;
        }
        stage_values<T, SKIP, NT, RW, pass_block(NT)>(val, row0, count, sv);
        if (rl >= count) return;
        if (tab && done && done[grid * R + v]) return;
        pass_row<T, R, SKIP, NT, MODE, CF, Base27, TWICE, false, true>(
            n, val, col, dcol, sb, r, z, row0 + rl, v, row_base, coarse, inj_coarse,
            tab || !done ? nullptr : done + v, sv + rl, RW);
    } else {
        if (rl >= count) return;
        // several grids: a converged grid is skipped before anything is
        // loaded (one grid: the host passes no flag)
        if (tab && done && done[grid * R + v]) return;
        pass_row<T, R, SKIP, NT, MODE, CF, Base27, TWICE>(n, val, col, dcol, sb, r, z, row0 + rl, v, row_base,
                                                         coarse, inj_coarse, tab || !done ? nullptr : done + v);
    }
}

// The first two passes of a zero-start forward sweep in one launch.  Colour
// 0 reads no neighbour (z_i = (r_i - 0 + 0*d_i)/d_i); colour 1 reads only its
// colour-0 neighbours, whose values this kernel forms on the fly with the
// same expression instead of waiting for them.  Rows [coff0, coff2) hold both
// colours contiguously (colour-major layout).
template <typename T, int R, bool NT, int CF, int ORD>
__global__ __launch_bounds__(pass_block(NT)) void k_pass_zs01(int64_t n, const T *__restrict__ val,
                                                      const int32_t *__restrict__ col,
                                                      const int8_t *__restrict__ dcol, const Base27 sb_arg,
                                                      const T *__restrict__ r, T *__restrict__ z,
                                                      const Seg *__restrict__ tab, int64_t coff0, int64_t coff1,
                                                      int64_t coff2, const int *__restrict__ done,
                                                      const int32_t *__restrict__ gbase) {
    MG_ARGS_FIRST("s"(n), "s"(val), "s"(r), "s"(z), "s"(tab), "s"(coff0), "s"(coff1), "s"(coff2), "s"(done),
                  "s"(gridDim.x));
    if constexpr (CF != 0) MG_BASES_FIRST(sb_arg);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    int64_t row0, count;
    int grid;
    Base27 sb1 = sb_arg;  // bases of colour 1
    if (tab) {
        const Seg e = tab[b];
        row0 = e.row0;
        count = e.count;
        grid = e.grid;
        if (CF && gbase) {
            const int32_t *gb = gbase + (e.grid * 8 + 1) * kW;
#pragma unroll
            for (int t = 0; t < kW; ++t) sb1.v[t] = gb[t];
        }
    } else {
        row0 = coff0 + (int64_t)b * pass_rows(NT, R);
        count = coff2 - row0;
        grid = 0;
    }
    // R >= kPairR: each lane updates two right-hand sides (as in k_pass)
    constexpr int LN = pass_lanes(R), NV = R / LN;
    const int rl = threadIdx.x / LN, w = threadIdx.x % LN;
    if (rl >= count) return;
    if (tab && done) {  // as in k_pass
        bool all = true;
#pragma unroll
        for (int u = 0; u < NV; ++u) all = all && done[grid * R + NV * w + u];
        if (all) return;
    }
    // one grid: the host passes no flag (z is internal)
    const int dv = (!tab && done && NV == 1) ? done[w] : 0;
    const int64_t i = row0 + rl;
    const int64_t o = i * R + NV * w;
    T rv[NV], zn[NV];
    ld_lanes(r + o, rv);
    if (i < coff1) {
        const T d = ld<NT>(val + ell_index(kCentre, i));
        const T acc = T(0), zi = T(0);
#pragma unroll
        for (int u = 0; u < NV; ++u) zn[u] = (rv[u] - acc + zi * d) / d;
        if (!dv) st_lanes(z + o, zn);
        return;
    }
    constexpr uint32_t SKIP = zs_mask(1, ORD);
    T a[kW];
    int32_t c[kW];
    load_slots<T, R, SKIP, NT, CF>(val, col, dcol, sb1, n, i, a, c);
    T rj[kW][NV], dj[kW];
#pragma unroll
    for (int s = 0; s < kW; ++s) {
        const bool sk = (SKIP >> s) & 1u;
        const bool use = !sk && a[s] != T(0);
        if (use) {
            ld_lanes(r + (int64_t)c[s] * R + NV * w, rj[s]);
        } else {
#pragma unroll
            for (int u = 0; u < NV; ++u) rj[s][u] = T(0);
        }
        dj[s] = use ? val[ell_index(kCentre, c[s])] : T(1);
    }
    const T d = a[kCentre];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        T acc = 0;
#pragma unroll
        for (int s = 0; s < kW; ++s) {
            const bool sk = (SKIP >> s) & 1u;
            if (!sk && a[s] != T(0)) {
                const T acc0 = T(0), z0 = T(0);
                const T zj = (rj[s][u] - acc0 + z0 * dj[s]) / dj[s];  // the colour-0 value of the first pass
                acc = acc + a[s] * zj;
            }
        }
        const T zi = T(0);
        zn[u] = (rv[u] - acc + zi * d) / d;
    }
    if (!dv) st_lanes(z + o, zn);
}

template <typename T, int R, bool NT, int CF>
static void pass_zs(int k, int order, int cnt, hipStream_t s, int64_t n, const T *val, const int32_t *col,
                    const int8_t *dcol, const Base27 &sb, const T *r, T *z, const Seg *tab, int64_t rb,
                    int64_t re, const int *done, const int32_t *gb) {
#define MG_ZS_CASE(K, O)                                                                              \
    case K + 8 * O:                                                                                   \
        k_pass<T, R, zs_mask(K, O), NT, 0, CF><<<cnt, pass_block(NT), 0, s>>>(n, val, col, dcol, sb, r, z, tab, rb, re, \
                                                                      done, nullptr, nullptr, nullptr, gb); \
        break;
    switch (k + 8 * order) {
        MG_ZS_CASE(0, 0) MG_ZS_CASE(1, 0) MG_ZS_CASE(2, 0) MG_ZS_CASE(3, 0)
        MG_ZS_CASE(4, 0) MG_ZS_CASE(5, 0) MG_ZS_CASE(6, 0) MG_ZS_CASE(7, 0)
        MG_ZS_CASE(0, 1) MG_ZS_CASE(1, 1) MG_ZS_CASE(2, 1) MG_ZS_CASE(3, 1)
        MG_ZS_CASE(4, 1) MG_ZS_CASE(5, 1) MG_ZS_CASE(6, 1) MG_ZS_CASE(7, 1)
        default: break;
    }
#undef MG_ZS_CASE
}

uint32_t standard_zs_mask(int k, int order) { return zs_mask(k, order); }
static_assert(zs_mask(7, 0) == (1u << kCentre) && zs_mask(7, 1) == (1u << kCentre),
              "the last colour of a zero-start sweep reads every neighbour");

template <typename T>
hipError_t launch_pass(const mgpcg_problem *P, int level, int k, int mode, const T *val, const T *r, T *z,
                       const int *done, T *coarse, hipStream_t s, double *rzp) {
    const Level &L = P->lev[level];
    const int R = P->R;
    if (rzp && (sizeof(T) != 8 || P->G != 1 || (mode != kPassPlain && mode != kPassTwice)))
        return hipErrorInvalidValue;
    // With one grid the passes store regardless of convergence: the flag
    // would put a dependent load in front of every pass (the compiler moves
    // the test ahead of the loads, whose results are dead when it fails),
    // and z is internal: after convergence the CG updates leave x, r and p
    // alone and the finalizes leave the scalars alone.  With several grids
    // a converged grid's workgroups return before loading anything.
    if (P->G == 1) done = nullptr;
    // several grids: the kernels read each segment's bases from the device table
    const int32_t *gb = P->G > 1 ? L.dbase : nullptr;
    const Seg *tab = nullptr;
    int cnt;
    const int64_t rb = L.coff[k], re = L.coff[k + 1];
    if (P->G > 1) {
        const int first = L.pass_first[k];
        cnt = L.pass_first[k + 1] - first;
        tab = L.pass_tab + first;
    } else {
        const int rows = pass_rows(L.stream_nt, R);
        cnt = (int)((re - rb + rows - 1) / rows);
    }
    if (cnt == 0) return hipSuccess;
    const int32_t *ic = L.inj_coarse;
    Base27 sb;
    for (int t = 0; t < kW; ++t) sb.v[t] = L.cf ? L.dbase_host[k * kW + t] : 0;
    if (mode == kPassZeroStart01) {
        if (k != 0 || !L.zs_std || L.ncol != 8 || (R != 1 && R != 16)) return hipErrorInvalidValue;
        int cnt01;
        const Seg *tab01 = nullptr;
        if (P->G > 1) {
            tab01 = L.pass_tab + L.pass_first[0];
            cnt01 = L.pass_first[2] - L.pass_first[0];
        } else {
            const int rows = pass_rows(L.stream_nt, R);
            cnt01 = (int)((L.coff[2] - L.coff[0] + rows - 1) / rows);
        }
        Base27 sb1;
        for (int t = 0; t < kW; ++t) sb1.v[t] = L.cf ? L.dbase_host[1 * kW + t] : 0;
#define MG_ZS01(RR, NT, CF)                                                                             \
    if (P->colour_order)                                                                               \
        k_pass_zs01<T, RR, NT, CF, 1><<<cnt01, pass_block(NT), 0, s>>>(L.n, val, L.col, L.dcol, sb1, r, z, tab01,      \
                                                            L.coff[0], L.coff[1], L.coff[2], done, gb);  \
    else                                                                                               \
        k_pass_zs01<T, RR, NT, CF, 0><<<cnt01, pass_block(NT), 0, s>>>(L.n, val, L.col, L.dcol, sb1, r, z, tab01,      \
                                                            L.coff[0], L.coff[1], L.coff[2], done, gb);
#define MG_ZS01_R(NT, CF)                                                                               \
    if (R == 1) { MG_ZS01(1, NT, CF) } else { MG_ZS01(16, NT, CF) }
        if (L.stream_nt) {
            if (L.cf == 2) { MG_ZS01_R(true, 2) } else if (L.cf == 1) { MG_ZS01_R(true, 1) } else { MG_ZS01_R(true, 0) }
        } else {
            if (L.cf == 2) { MG_ZS01_R(false, 2) } else if (L.cf == 1) { MG_ZS01_R(false, 1) } else { MG_ZS01_R(false, 0) }
        }
#undef MG_ZS01_R
#undef MG_ZS01
        return hipGetLastError();
    }
    if (mode == kPassTwice || mode == kPassTwiceZeroStart) {
        // colour k swept twice in a row; on a zero start its first update
        // skips only the diagonal (every other colour is already written)
        if (mode == kPassTwiceZeroStart && (!L.zs_std || k != L.ncol - 1 || L.ncol != 8)) return hipErrorInvalidValue;
#define MG_TWICE_LAUNCH(SKIPM, NT, CF)                                                                  \
    if (rzp && SKIPM == 0u) {                                                                          \
        if constexpr (sizeof(T) == 8)                                                                  \
            MG_DISPATCH_R(R, (k_pass<T, RR, SKIPM, NT, 0, CF, true, true><<<cnt, pass_block(NT), 0, s>>>(  \
                                 L.n, val, L.col, L.dcol, sb, r, z, tab, rb, re, done, nullptr, nullptr, rzp, gb))); \
    } else {                                                                                           \
        MG_DISPATCH_R(R, (k_pass<T, RR, SKIPM, NT, 0, CF, true><<<cnt, pass_block(NT), 0, s>>>(            \
                             L.n, val, L.col, L.dcol, sb, r, z, tab, rb, re, done, nullptr, nullptr, nullptr, gb))); \
    }
#define MG_TWICE_MODE(SKIPM)                                                                            \
    if (L.stream_nt) {                                                                                 \
        if (L.cf == 2) { MG_TWICE_LAUNCH(SKIPM, true, 2) } else if (L.cf == 1) { MG_TWICE_LAUNCH(SKIPM, true, 1) } else { MG_TWICE_LAUNCH(SKIPM, true, 0) }    \
    } else {                                                                                           \
        if (L.cf == 2) { MG_TWICE_LAUNCH(SKIPM, false, 2) } else if (L.cf == 1) { MG_TWICE_LAUNCH(SKIPM, false, 1) } else { MG_TWICE_LAUNCH(SKIPM, false, 0) }  \
    }
        if (mode == kPassTwiceZeroStart) {
            MG_TWICE_MODE(zs_mask(7, 0))
        } else {
            MG_TWICE_MODE(0u)
        }
#undef MG_TWICE_MODE
#undef MG_TWICE_LAUNCH
        return hipGetLastError();
    }
    if (mode == kPassZeroStart) {
        if (!L.zs_std || (R != 1 && R != 16)) return hipErrorInvalidValue;
        const int ord = P->colour_order;
#define MG_ZS_LAUNCH(NT, CF)                                                                           \
    if (R == 1) pass_zs<T, 1, NT, CF>(k, ord, cnt, s, L.n, val, L.col, L.dcol, sb, r, z, tab, rb, re, done, gb); \
    else pass_zs<T, 16, NT, CF>(k, ord, cnt, s, L.n, val, L.col, L.dcol, sb, r, z, tab, rb, re, done, gb);
        if (L.stream_nt) {
            if (L.cf == 2) { MG_ZS_LAUNCH(true, 2) } else if (L.cf == 1) { MG_ZS_LAUNCH(true, 1) } else { MG_ZS_LAUNCH(true, 0) }
        } else {
            if (L.cf == 2) { MG_ZS_LAUNCH(false, 2) } else if (L.cf == 1) { MG_ZS_LAUNCH(false, 1) } else { MG_ZS_LAUNCH(false, 0) }
        }
#undef MG_ZS_LAUNCH
        return hipGetLastError();
    }
#define MG_PASS_LAUNCH(NT, M, CF)                                                                      \
    if (M == 0 && rzp) {                                                                               \
        if constexpr (sizeof(T) == 8)                                                                  \
            MG_DISPATCH_R(R, (k_pass<T, RR, 0u, NT, 0, CF, false, true><<<cnt, pass_block(NT), 0, s>>>(    \
                                 L.n, val, L.col, L.dcol, sb, r, z, tab, rb, re, done, coarse, ic, rzp, gb))); \
    } else {                                                                                           \
        MG_DISPATCH_R(R, (k_pass<T, RR, 0u, NT, M, CF><<<cnt, pass_block(NT), 0, s>>>(L.n, val, L.col, L.dcol, sb, \
                                                                          r, z, tab, rb, re, done, coarse, ic, \
                                                                          nullptr, gb)));         \
    }
#define MG_PASS_MODE(M)                                                                                \
    if (L.stream_nt) {                                                                                 \
        if (L.cf == 2) { MG_PASS_LAUNCH(true, M, 2) } else if (L.cf == 1) { MG_PASS_LAUNCH(true, M, 1) } else { MG_PASS_LAUNCH(true, M, 0) }            \
    } else {                                                                                           \
        if (L.cf == 2) { MG_PASS_LAUNCH(false, M, 2) } else if (L.cf == 1) { MG_PASS_LAUNCH(false, M, 1) } else { MG_PASS_LAUNCH(false, M, 0) }          \
    }
    if (mode == kPassRestrict) {
        if (!L.fuse_transfers) return hipErrorInvalidValue;
        MG_PASS_MODE(1)
    } else if (mode == kPassProlong) {
        if (!L.fuse_transfers) return hipErrorInvalidValue;
        MG_PASS_MODE(2)
    } else {
        MG_PASS_MODE(0)
    }
#undef MG_PASS_LAUNCH
#undef MG_PASS_MODE
    return hipGetLastError();
}
template hipError_t launch_pass<double>(const mgpcg_problem *, int, int, int, const double *,
                                        const double *, double *, const int *, double *, hipStream_t, double *);
template hipError_t launch_pass<float>(const mgpcg_problem *, int, int, int, const float *,
                                       const float *, float *, const int *, float *, hipStream_t, double *);

// --------------------------------------------- persistent coarse V-cycle
//
// Levels lc..L-1 of one V-cycle in a single launch.  Every colour pass of a
// coarse level is small (a few thousand to a few hundred thousand rows), so as
// separate kernels each costs a launch-and-drain latency floor.  Here the
// workgroups stay resident and separate the passes with a grid barrier.
//
// Barrier: workgroup b publishes the epoch it reached in flags[b]; a barrier
// completes when every flag has reached the current epoch.  Epochs count up
// from a device-resident base that the kernel advances itself, so a captured
// graph can replay the launch unchanged.  Flags and base are cleared by the
// host before each solve.  Every wait is bounded: on timeout the waiting
// workgroup raises `err`, every workgroup that sees it stops, and the host
// reports the error.

__device__ __forceinline__ bool grid_barrier(unsigned *flags, int B, unsigned epoch, int *err,
                                             long long spin_limit) {
    __shared__ int s_ok;
    // Every wave first waits until its own stores have completed at its L2
    // (the memory counter is per wave, and the workgroup barrier alone does not
    // wait for it); after the workgroup barrier one release fence then writes
    // that L2 back for the other XCDs.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x < 64) {
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&flags[blockIdx.x], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        long long spins = 0;
        int good = 1;
        for (;;) {
            int mine = 1;
            for (int j = threadIdx.x; j < B; j += 64)
                mine &= __hip_atomic_load(&flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
            if (__all(mine)) break;
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                good = 0;
                break;
            }
            if (++spins > spin_limit) {
                if (threadIdx.x == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        // acquire: the CU's caches and this XCD's L2 drop stale lines
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (threadIdx.x == 0) s_ok = good;
    }
    __syncthreads();
    return s_ok != 0;
}

template <typename T, int R, int CF, uint32_t SKIP, int MODE, bool TWICE = false>
__device__ __forceinline__ void coarse_phase(const CoarseLevel &lv, int k, T *coarse, int bid, int B) {
    const int32_t *sb = CF ? lv.dbase + k * kW : nullptr;
    const int64_t r0 = lv.coff[k], r1 = lv.coff[k + 1];
    const int rpb = blockDim.x / R;
    const int rl = threadIdx.x / R, v = threadIdx.x % R;
    for (int64_t base = r0 + (int64_t)bid * rpb; base < r1; base += (int64_t)B * rpb) {
        const int64_t i = base + rl;
        if (i < r1)
            pass_row<T, R, SKIP, false, MODE, CF, const int32_t *, TWICE>(
                lv.n, (const T *)lv.val, lv.col, lv.dcol, sb, (const T *)lv.r, (T *)lv.z, i, v, r0, coarse,
                lv.inj_coarse);
    }
}

// separate restriction / refinement phases (when they cannot ride on a pass)
template <typename T, int R, int CF>
__device__ __forceinline__ void coarse_restrict(const CoarseLevel &lv, T *rc, int bid, int B) {
    const int rpb = blockDim.x / R;
    const int rl = threadIdx.x / R, v = threadIdx.x % R;
    for (int64_t base = (int64_t)bid * rpb; base < lv.n_inj; base += (int64_t)B * rpb) {
        const int64_t t = base + rl;
        if (t < lv.n_inj) {
            const int64_t i = lv.inj_fine[t];
            const int32_t *sb = CF ? lv.dbase + colour_of(lv.coff, 8, i) * kW : nullptr;
            T d;
            const T acc = row_sum<T, R, 0u, false, CF>((const T *)lv.val, lv.col, lv.dcol, sb, lv.n, i,
                                                      (const T *)lv.z, v, d);
            rc[(int64_t)lv.inj_coarse[t] * R + v] = ((const T *)lv.r)[i * R + v] - acc;
        }
    }
}

template <typename T, int R>
__device__ __forceinline__ void coarse_prolong(const CoarseLevel &lv, const T *zc, int bid, int B) {
    const int rpb = blockDim.x / R;
    const int rl = threadIdx.x / R, v = threadIdx.x % R;
    T *z = (T *)lv.z;
    for (int64_t base = (int64_t)bid * rpb; base < lv.n_inj; base += (int64_t)B * rpb) {
        const int64_t t = base + rl;
        if (t < lv.n_inj) {
            const int64_t o = (int64_t)lv.inj_fine[t] * R + v;
            z[o] = z[o] + zc[(int64_t)lv.inj_coarse[t] * R + v];
        }
    }
}

template <typename T, int R, int CF, int ORD>
__device__ __forceinline__ void coarse_run_phase(const CoarseArgs &A, int ph, int bid, int B) {
    const int l = ph & 15, k = (ph >> 4) & 15, op = ph >> 8;
    const CoarseLevel &lv = A.lev[l];
    switch (op) {
        case kOpPlain:
            coarse_phase<T, R, CF, 0u, 0>(lv, k, nullptr, bid, B);
            break;
        case kOpZeroStart:
            switch (k) {
#define MG_ZS_PHASE(K) \
    case K: coarse_phase<T, R, CF, zs_mask(K, ORD), 0>(lv, K, nullptr, bid, B); break;
                MG_ZS_PHASE(0) MG_ZS_PHASE(1) MG_ZS_PHASE(2) MG_ZS_PHASE(3)
                MG_ZS_PHASE(4) MG_ZS_PHASE(5) MG_ZS_PHASE(6) MG_ZS_PHASE(7)
#undef MG_ZS_PHASE
                default: break;
            }
            break;
        case kOpFusedRestrict:
            coarse_phase<T, R, CF, 0u, 1>(lv, k, (T *)A.lev[l + 1].r, bid, B);
            break;
        case kOpFusedProlong:
            coarse_phase<T, R, CF, 0u, 2>(lv, k, (T *)A.lev[l + 1].z, bid, B);
            break;
        case kOpRestrict:
            coarse_restrict<T, R, CF>(lv, (T *)A.lev[l + 1].r, bid, B);
            break;
        case kOpProlong:
            coarse_prolong<T, R>(lv, (const T *)A.lev[l + 1].z, bid, B);
            break;
        case kOpTwice:
            coarse_phase<T, R, CF, 0u, 0, true>(lv, k, nullptr, bid, B);
            break;
        case kOpTwiceZeroStart:
            coarse_phase<T, R, CF, zs_mask(7, ORD), 0, true>(lv, k, nullptr, bid, B);
            break;
        default:
            break;
    }
}

// Executes the host-built phase program (level, colour, operation) with one
// grid barrier between consecutive phases.
template <typename T, int R, int CF, int ORD>
__global__ __launch_bounds__(kBlock) void k_coarse_vcycle(CoarseArgs A) {
    __shared__ unsigned s_base;
    const int B = gridDim.x;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    if (threadIdx.x == 0) s_base = __hip_atomic_load(A.epoch_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    unsigned epoch = s_base;
    bool ok = true;
    for (int p = 0; p < A.nphases; ++p) {
        if (ok) coarse_run_phase<T, R, CF, ORD>(A, A.phase[p], bid, B);
        if (p + 1 == A.nphases) break;
        ++epoch;
        if (ok) ok = grid_barrier(A.flags, B, epoch, A.err, A.spin_limit);
        // after the first barrier every workgroup has read the base: advance
        // it past this launch's epochs for the next launch
        if (p == 0 && blockIdx.x == 0 && threadIdx.x == 0)
            __hip_atomic_store(A.epoch_base, s_base + (unsigned)(A.nphases - 1), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Coarsest level, one workgroup: its symmetric sweep (zero-start forward
// pass, backward pass) with r and z held in LDS.  The 15 colour passes are
// separated by workgroup barriers instead of kernel launches, and the 27
// gathers of every row read LDS.  The operator rows do not depend on z, so
// the pass is software-pipelined: while one pass computes, each thread's row
// of the next pass is already on its way from memory into registers, and
// the barriers between passes wait for LDS traffic only.

// barrier for LDS data only: prefetches from global memory stay in flight
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T, int CF, uint32_t SKIP>
__device__ __forceinline__ void tail_load(const T *val, const int32_t *col, const int8_t *dcol, const CoffTable &ct,
                                          int k,
                                          RawRow<T, CF> &rw) {
    // unconditional (threads past the colour's end load its last row, or
    // row 0), so that the loads are straight-line code the wait counters
    // track exactly
    int64_t i = ct.coff[k] + threadIdx.x;
    if (i >= ct.coff[k + 1]) i = ct.coff[k + 1] > 0 ? ct.coff[k + 1] - 1 : 0;
    // an opaque copy of the row index per pass: the compiler can then not
    // merge these loads with the other sweep's loads of the same colour
    asm volatile("" : "+v"(i));
    load_raw<T, SKIP, false, CF>(val, col, dcol, i, rw);
    // keep the loads here: without this the compiler sinks them to their
    // use in the next pass, which would put them back on the critical path
    asm volatile("" ::: "memory");
}

// the [8][27] column bases, read through the constant address space: scalar
// loads, which neither wait behind the vector prefetches nor hold registers
// between passes
typedef const __attribute__((address_space(4))) int32_t *ConstBases;

// Neighbour values of one row read from LDS nine slots at a time (the sums
// call load() at the start of each group), the columns decoded from the raw
// row as they are needed; optionally with the diagonal slot replaced by a
// given value.
template <typename T, int CF, uint32_t SKIP, bool CENTRE>
struct LdsGather {
    const T *zs;
    const RawRow<T, CF> &rw;
    ConstBases cb;
    int64_t i;
    T centre;
    T buf[kW];
    __device__ __forceinline__ void load(int s0) {
        // unconditional reads (an unused slot reads row 0), so that the nine
        // are issued together instead of one branch each
#pragma unroll
        for (int s = s0; s < s0 + 9 && s < kW; ++s) {
            const bool use = !((SKIP >> s) & 1u) && rw.a[s] != T(0);
            const T v = zs[use ? slot_col<CF>(rw, cb, i, s) : 0];
            buf[s] = (CENTRE && s == kCentre) ? centre : (use ? v : T(0));
        }
    }
    __device__ __forceinline__ T operator()(int s) const { return buf[s]; }
};

// one row of a pass with z in LDS (rows of one colour never neighbour each
// other, so nothing a row reads changes during the pass)
template <typename T, int CF, uint32_t SKIP, bool TWICE>
__device__ __forceinline__ void tail_row(const RawRow<T, CF> &rw, ConstBases cb, const T *rs, T *zs, int64_t i) {
    const T rv = rs[i];
    const T zi = SKIP ? T(0) : zs[slot_col<CF>(rw, cb, i, kCentre)];
    const T znew = gs_update<T, SKIP, 9>(rw.a, LdsGather<T, CF, SKIP, false>{zs, rw, cb, i, T(0)}, rv, zi);
    // a second pass of the same colour: the full row with the new diagonal value
    zs[i] = TWICE ? gs_update<T, 0u, 9>(rw.a, LdsGather<T, CF, 0u, true>{zs, rw, cb, i, znew}, rv, znew) : znew;
}

// the rows of colour k (one per thread: the level qualifies only if every
// colour fits in the workgroup), operators from the prefetched raw rows
template <typename T, int CF, uint32_t SKIP, bool TWICE>
__device__ __forceinline__ void tail_pass(ConstBases cb, const CoffTable &ct, int k, const RawRow<T, CF> &rw,
                                          const T *rs, T *zs) {
    const int64_t i = ct.coff[k] + threadIdx.x;
    if (i < ct.coff[k + 1]) tail_row<T, CF, SKIP, TWICE>(rw, cb + k * kW, rs, zs, i);
}

// (the operator pointers are deliberately not __restrict__: that lets the
// compiler keep the forward sweep's loads of a colour for its backward pass,
// which does not fit in registers next to the prefetch buffers)
template <typename T, int CF, int ORD>
__global__ __launch_bounds__(kTailBlock) void k_coarse_tail(int64_t n, const T *val, const int32_t *col,
                                                            const int8_t *dcol,
                                                            const int32_t *__restrict__ dbase, CoffTable ct,
                                                            const T *__restrict__ r, T *__restrict__ z) {
    extern __shared__ char tail_lds[];
    const ConstBases tb = (ConstBases)dbase;
    T *rs = (T *)tail_lds;
    T *zs = rs + n;
    // forward, zero start (colour k reads only colours < k); colour 7 is the
    // last forward and the first backward pass in one; then backward 6..0:
    // 15 passes.  Rows of a pass are loaded DEPTH-1 passes ahead: pass p
    // computes from buffer p % DEPTH while later passes' rows are in flight.
    // Three buffers in FP32; in FP64 three rows of 27 values no longer fit
    // in registers next to the working set, so two.
    constexpr int DEPTH = sizeof(T) == 4 ? 3 : 2;
#define MG_TAIL_LOAD(K, SK, B) tail_load<T, CF, SK>(val, col, dcol, ct, K, B);
#define MG_TAIL_PASS(K, SK, TW, B)                                                                      \
    tail_pass<T, CF, SK, TW>(tb, ct, K, B, rs, zs);                                                    \
    lds_barrier();
    if constexpr (DEPTH == 3) {
        RawRow<T, CF> b0, b1, b2;
        MG_TAIL_LOAD(0, zs_mask(0, ORD), b0)
        MG_TAIL_LOAD(1, zs_mask(1, ORD), b1)
        for (int64_t i = threadIdx.x; i < n; i += kTailBlock) rs[i] = r[i];
        __syncthreads();
        MG_TAIL_LOAD(2, zs_mask(2, ORD), b2) MG_TAIL_PASS(0, zs_mask(0, ORD), false, b0)
        MG_TAIL_LOAD(3, zs_mask(3, ORD), b0) MG_TAIL_PASS(1, zs_mask(1, ORD), false, b1)
        MG_TAIL_LOAD(4, zs_mask(4, ORD), b1) MG_TAIL_PASS(2, zs_mask(2, ORD), false, b2)
        MG_TAIL_LOAD(5, zs_mask(5, ORD), b2) MG_TAIL_PASS(3, zs_mask(3, ORD), false, b0)
        MG_TAIL_LOAD(6, zs_mask(6, ORD), b0) MG_TAIL_PASS(4, zs_mask(4, ORD), false, b1)
        MG_TAIL_LOAD(7, zs_mask(7, ORD), b1) MG_TAIL_PASS(5, zs_mask(5, ORD), false, b2)
        MG_TAIL_LOAD(6, 0u, b2) MG_TAIL_PASS(6, zs_mask(6, ORD), false, b0)
        MG_TAIL_LOAD(5, 0u, b0) MG_TAIL_PASS(7, zs_mask(7, ORD), true, b1)
        MG_TAIL_LOAD(4, 0u, b1) MG_TAIL_PASS(6, 0u, false, b2)
        MG_TAIL_LOAD(3, 0u, b2) MG_TAIL_PASS(5, 0u, false, b0)
        MG_TAIL_LOAD(2, 0u, b0) MG_TAIL_PASS(4, 0u, false, b1)
        MG_TAIL_LOAD(1, 0u, b1) MG_TAIL_PASS(3, 0u, false, b2)
        MG_TAIL_LOAD(0, 0u, b2) MG_TAIL_PASS(2, 0u, false, b0)
        MG_TAIL_PASS(1, 0u, false, b1)
        tail_pass<T, CF, 0u, false>(tb, ct, 0, b2, rs, zs);
    } else {
        RawRow<T, CF> b0, b1;
        MG_TAIL_LOAD(0, zs_mask(0, ORD), b0)
        for (int64_t i = threadIdx.x; i < n; i += kTailBlock) rs[i] = r[i];
        __syncthreads();
        MG_TAIL_LOAD(1, zs_mask(1, ORD), b1) MG_TAIL_PASS(0, zs_mask(0, ORD), false, b0)
        MG_TAIL_LOAD(2, zs_mask(2, ORD), b0) MG_TAIL_PASS(1, zs_mask(1, ORD), false, b1)
        MG_TAIL_LOAD(3, zs_mask(3, ORD), b1) MG_TAIL_PASS(2, zs_mask(2, ORD), false, b0)
        MG_TAIL_LOAD(4, zs_mask(4, ORD), b0) MG_TAIL_PASS(3, zs_mask(3, ORD), false, b1)
        MG_TAIL_LOAD(5, zs_mask(5, ORD), b1) MG_TAIL_PASS(4, zs_mask(4, ORD), false, b0)
        MG_TAIL_LOAD(6, zs_mask(6, ORD), b0) MG_TAIL_PASS(5, zs_mask(5, ORD), false, b1)
        MG_TAIL_LOAD(7, zs_mask(7, ORD), b1) MG_TAIL_PASS(6, zs_mask(6, ORD), false, b0)
        MG_TAIL_LOAD(6, 0u, b0) MG_TAIL_PASS(7, zs_mask(7, ORD), true, b1)
        MG_TAIL_LOAD(5, 0u, b1) MG_TAIL_PASS(6, 0u, false, b0)
        MG_TAIL_LOAD(4, 0u, b0) MG_TAIL_PASS(5, 0u, false, b1)
        MG_TAIL_LOAD(3, 0u, b1) MG_TAIL_PASS(4, 0u, false, b0)
        MG_TAIL_LOAD(2, 0u, b0) MG_TAIL_PASS(3, 0u, false, b1)
        MG_TAIL_LOAD(1, 0u, b1) MG_TAIL_PASS(2, 0u, false, b0)
        MG_TAIL_LOAD(0, 0u, b0) MG_TAIL_PASS(1, 0u, false, b1)
        tail_pass<T, CF, 0u, false>(tb, ct, 0, b0, rs, zs);
    }
#undef MG_TAIL_PASS
#undef MG_TAIL_LOAD
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += kTailBlock) z[i] = zs[i];
}

hipError_t launch_coarse_tail(const mgpcg_problem *P, bool fp32, hipStream_t s) {
    const int l = P->L - 1;
    const Level &L = P->lev[l];
    if (P->R != 1 || L.ncol != 8) return hipErrorInvalidValue;
    const CoffTable ct = coff_table(L);
    const size_t lds = (size_t)L.n * 2 * (fp32 ? sizeof(float) : sizeof(double));
#define MG_TAIL(T, VAL, CF)                                                                            \
    if (P->colour_order)                                                                               \
        k_coarse_tail<T, CF, 1><<<1, kTailBlock, lds, s>>>(L.n, VAL, L.col, L.dcol, L.dbase, ct, (const T *)L.r, \
                                                          (T *)L.z);                                    \
    else                                                                                               \
        k_coarse_tail<T, CF, 0><<<1, kTailBlock, lds, s>>>(L.n, VAL, L.col, L.dcol, L.dbase, ct, (const T *)L.r, \
                                                          (T *)L.z);
    if (fp32) {
        if (L.cf == 2) { MG_TAIL(float, L.val32, 2) } else if (L.cf == 1) { MG_TAIL(float, L.val32, 1) } else { MG_TAIL(float, L.val32, 0) }
    } else {
        if (L.cf == 2) { MG_TAIL(double, L.val64, 2) } else if (L.cf == 1) { MG_TAIL(double, L.val64, 1) } else { MG_TAIL(double, L.val64, 0) }
    }
#undef MG_TAIL
    return hipGetLastError();
}

hipError_t launch_coarse_vcycle(const mgpcg_problem *P, bool fp32, hipStream_t s) {
    const CoarseArgs &A = P->coarse_args;
    const int B = P->coarse_blocks;
    if (P->R != 1 || A.nphases < 1) return hipErrorInvalidValue;
#define MG_COARSE(T, CF)                                                                               \
    if (P->colour_order) k_coarse_vcycle<T, 1, CF, 1><<<B, kBlock, 0, s>>>(A);                           \
    else k_coarse_vcycle<T, 1, CF, 0><<<B, kBlock, 0, s>>>(A);
    if (fp32) {
        if (A.cf == 2) { MG_COARSE(float, 2) } else if (A.cf == 1) { MG_COARSE(float, 1) } else { MG_COARSE(float, 0) }
    } else {
        if (A.cf == 2) { MG_COARSE(double, 2) } else if (A.cf == 1) { MG_COARSE(double, 1) } else { MG_COARSE(double, 0) }
    }
#undef MG_COARSE
    return hipGetLastError();
}

int coarse_vcycle_occupancy(int R, bool fp32, int cf, int order) {
    if (R != 1) return 0;
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define MG_OCC(T, CF, O) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_coarse_vcycle<T, 1, CF, O>, kBlock, 0);
#define MG_OCC2(T, CF)                                                                                  \
    if (order) { MG_OCC(T, CF, 1) } else { MG_OCC(T, CF, 0) }
    if (fp32) {
        if (cf == 2) { MG_OCC2(float, 2) } else if (cf == 1) { MG_OCC2(float, 1) } else { MG_OCC2(float, 0) }
    } else {
        if (cf == 2) { MG_OCC2(double, 2) } else if (cf == 1) { MG_OCC2(double, 1) } else { MG_OCC2(double, 0) }
    }
#undef MG_OCC2
#undef MG_OCC
    return e == hipSuccess ? nb : 0;
}

// ------------------------------------------------------------- transfers

// rc = inject(r - A z): only the injection rows of the residual are formed.
// Threads walk the injection rows in fine order (coalesced operator reads)
// and scatter into the coarse vector.
template <typename T, int R, bool NT, int CF>
__global__ __launch_bounds__(kBlock) void k_restrict(int64_t n, const T *__restrict__ val,
                                                     const int32_t *__restrict__ col,
                                                     const int8_t *__restrict__ dcol,
                                                     const int32_t *__restrict__ dbase,
                                                     const int32_t *__restrict__ grow, CoffTable ct,
                                                     const Base27 sb_inj,
                                                     const T *__restrict__ r, const T *__restrict__ z,
                                                     T *__restrict__ rc,
                                                     const int32_t *__restrict__ inj_fine,
                                                     const int32_t *__restrict__ inj_coarse,
                                                     int64_t n_inj) {
    MG_ARGS_FIRST("s"(n), "s"(val), "s"(grow), "s"(r), "s"(z), "s"(rc), "s"(inj_fine), "s"(inj_coarse), "s"(n_inj),
                  "s"(gridDim.x));
    if constexpr (CF != 0) MG_BASES_FIRST(sb_inj);
    int64_t gid = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (gid >= n_inj * R) return;
    int64_t t = gid / R;
    int v = (int)(gid % R);
    int64_t i = inj_fine[t];
    T d;
    T acc;
    if (CF && grow) {
        // several grids: the bases of the row's grid and colour, per lane
        const int32_t *sb = dbase + (grow[i] * 8 + colour_of(ct.coff, ct.ncol, i)) * kW;
        acc = row_sum<T, R, 0u, NT, CF>(val, col, dcol, sb, n, i, z, v, d);
    } else {
        // one grid: every injection point has the same colour, whose bases
        // come with the arguments (no dependent table load)
        acc = row_sum<T, R, 0u, NT, CF>(val, col, dcol, sb_inj, n, i, z, v, d);
    }
    rc[(int64_t)inj_coarse[t] * R + v] = r[i * R + v] - acc;
}

template <typename T>
hipError_t launch_restrict(const mgpcg_problem *P, int level, const T *val, const T *r, const T *z,
                           T *rc, hipStream_t s) {
    const Level &L = P->lev[level];
    int64_t work = L.n_inj * P->R;
    if (work == 0) return hipSuccess;
    const CoffTable ct = coff_table(L);
    Base27 sb_inj;  // one grid: the bases of the injection colour
    const int kinj = P->G == 1 ? L.grids[0].inj_colour : 0;
    for (int t = 0; t < kW; ++t) sb_inj.v[t] = L.cf ? L.dbase_host[kinj * kW + t] : 0;
#define MG_RESTRICT(NT, CF)                                                                             \
    MG_DISPATCH_R(P->R, (k_restrict<T, RR, NT, CF><<<nblocks(work), kBlock, 0, s>>>(                    \
                            L.n, val, L.col, L.dcol, L.dbase, L.grid_of_row, ct, sb_inj, r, z, rc, L.inj_fine,  \
                            L.inj_coarse, L.n_inj)));
    if (L.stream_nt) {
        if (L.cf == 2) { MG_RESTRICT(true, 2) } else if (L.cf == 1) { MG_RESTRICT(true, 1) } else { MG_RESTRICT(true, 0) }
    } else {
        if (L.cf == 2) { MG_RESTRICT(false, 2) } else if (L.cf == 1) { MG_RESTRICT(false, 1) } else { MG_RESTRICT(false, 0) }
    }
#undef MG_RESTRICT
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
    MG_ARGS_FIRST("s"(zc), "s"(z), "s"(inj_fine), "s"(inj_coarse), "s"(n_inj), "s"(gridDim.x));
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
    MG_ARGS_FIRST("s"(a), "s"(b), "s"(n));
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
__global__ __launch_bounds__(kBlock) void k_cast_f2d(const float *__restrict__ a, double *__restrict__ b,
                                                     int64_t n) {
    MG_ARGS_FIRST("s"(a), "s"(b), "s"(n));
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
// Reduction kernels walk a level-0 reduction table: each workgroup owns a
// grid-homogeneous segment of rows, and the segments of one grid are
// consecutive table entries [gb[g], gb[g+1]).  A workgroup reduces its
// per-rhs partial sums with a fixed wave-shuffle/LDS tree and stores them.
// A finalize kernel with one workgroup per grid then adds that grid's
// partials in a fixed order and updates the CG scalars of its R systems.
// No atomics: results are identical from run to run, and thousands of
// workgroups never contend on one counter.

enum Kind { kInit = 0, kRz = 1, kPq = 2, kRr = 3 };


// all R systems of grid g finished?
template <int R>
__device__ __forceinline__ bool grid_done(const int *done, int g) {
    bool all = true;
#pragma unroll
    for (int v = 0; v < R; ++v) all = all && done[g * R + v];
    return all;
}

// Rows of one block of a vector kernel: from the segment table (several
// grids), or, for one grid (tab == NULL), the blk-th chunk of `rows` rows of
// [0, nrows), so that no table load precedes the data loads.
__device__ __forceinline__ Seg vec_seg(const Seg *__restrict__ tab, int blk, int64_t nrows, int rows) {
    if (tab) return tab[blk];
    Seg e;
    e.row0 = (int64_t)blk * rows;
    e.count = (int32_t)(nrows - e.row0 < rows ? nrows - e.row0 : rows);
    e.grid = 0;
    e.colour = 0;
    return e;
}

// sum_j a_ij x_j of row i for right-hand sides 2w and 2w+1 (values staged in
// LDS), each in row_sum's slot order
template <int R, int CF, class SB>
__device__ __forceinline__ void row_sum2(const int32_t *__restrict__ col, const int8_t *__restrict__ dcol,
                                         const SB &sb, int64_t n, int64_t i, const double *x, int w,
                                         const double *vs, int vstride, double (&s2)[2]) {
    double a[kW];
    int32_t c[kW];
    load_slots<double, R, 0u, true, CF, SB, true>(nullptr, col, dcol, sb, n, i, a, c, vs, vstride);
    double xv[kW][2];
#pragma unroll
    for (int t = 0; t < kW; ++t) ld_lanes(x + (int64_t)c[t] * R + 2 * w, xv[t]);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        double acc = 0;
#pragma unroll
        for (int t = 0; t < kW; ++t)
            if (a[t] != 0.0) acc = acc + a[t] * xv[t][u];
        s2[u] = acc;
    }
}

// SpMV-type kernels (one row per R threads, table 0): with one right-hand
// side a workgroup takes one table entry of kBlock rows.  With R > 1 an entry
// holds only kBlock/R rows, so a workgroup takes `spc` consecutive entries of
// one grid (the table pads every grid to a multiple of spc with empty
// entries).  That keeps the workgroup count, and the partials the finalize
// sums, at the one-rhs level.

// r = b - A x, partial ||r||^2
template <int R, int CF>
__global__ __launch_bounds__(kBlock) void k_init_residual(int64_t n, const double *__restrict__ val,
                                                          const int32_t *__restrict__ col,
                                                          const int8_t *__restrict__ dcol,
                                                          const int32_t *__restrict__ dbase,
                                                          const double *__restrict__ b,
                                                          const double *__restrict__ x,
                                                          double *__restrict__ r, const Seg *__restrict__ tab,
                                                          double *__restrict__ partials, int spc) {
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    if constexpr (R >= kPairR) {
        // R/2 lanes per row, two right-hand sides each; values through LDS
        constexpr int LN = pass_lanes(R), RW = kBlock / LN;
        __shared__ double sv2[kW * RW];
        const int w = threadIdx.x % LN, rl = threadIdx.x / LN;
        double acc0 = 0.0, acc1 = 0.0;
        for (int it = 0; it < spc; ++it) {
            const Seg e = tab[(int64_t)blk * spc + it];
            stage_values<double, 0u, true, RW, kBlock>(val, e.row0, e.count, sv2);
            if (rl < e.count) {
                const int64_t i = e.row0 + rl;
                const int32_t *sb = CF ? dbase + (e.grid * 8 + e.colour) * kW : nullptr;
                double s2[2], bv[2], ri[2];
                row_sum2<R, CF>(col, dcol, sb, n, i, x, w, sv2 + rl, RW, s2);
                ld_lanes(b + i * R + 2 * w, bv);
                ri[0] = bv[0] - s2[0];
                ri[1] = bv[1] - s2[1];
                st_lanes(r + i * R + 2 * w, ri);
                acc0 += ri[0] * ri[0];
                acc1 += ri[1] * ri[1];
            }
            __syncthreads();  // the next entry overwrites sv2
        }
        store_partial2<R>(acc0, acc1, blk, partials);
        return;
    }
    const int v = threadIdx.x % R, rl = threadIdx.x / R;
    double acc = 0.0;
    for (int it = 0; it < (R == 1 ? 1 : spc); ++it) {
        const Seg e = tab[(int64_t)blk * (R == 1 ? 1 : spc) + it];
        if constexpr (R < kStageR) {
            if (rl < e.count) {
                const int64_t i = e.row0 + rl;
                double d;
                const int32_t *sb = CF ? dbase + (e.grid * 8 + e.colour) * kW : nullptr;
                const double s = row_sum<double, R, 0u, true, CF>(val, col, dcol, sb, n, i, x, v, d);
                const double ri = b[i * R + v] - s;
                r[i * R + v] = ri;
                if constexpr (R == 1) acc = ri * ri;
                else acc += ri * ri;
            }
        } else {
            // R lanes per row: the entry's values go through LDS once
            __shared__ double sv[kW * (kBlock / R)];
            stage_values<double, 0u, true, kBlock / R, kBlock>(val, e.row0, e.count, sv);
            if (rl < e.count) {
                const int64_t i = e.row0 + rl;
                double d;
                const int32_t *sb = CF ? dbase + (e.grid * 8 + e.colour) * kW : nullptr;
                const double s = row_sum<double, R, 0u, true, CF, true>(val, col, dcol, sb, n, i, x, v, d,
                                                                         sv + rl, kBlock / R);
                const double ri = b[i * R + v] - s;
                r[i * R + v] = ri;
                acc += ri * ri;
            }
            __syncthreads();  // the next entry overwrites sv
        }
    }
    store_partial<R>(acc, blk, partials);
}

// partial <r, z>
// (done: NULL for one grid, whose converged state the finalize checks)
template <int R>
__global__ __launch_bounds__(kBlock) void k_dot_rz(const double *__restrict__ r, const double *__restrict__ z,
                                                   const Seg *__restrict__ tab, int64_t nrows,
                                                   double *__restrict__ partials, const int *__restrict__ done) {
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const Seg e = vec_seg(tab, blk, nrows, kVecRows * kBlock / R);
    if (done && grid_done<R>(done, e.grid)) return;
    const int v = threadIdx.x % R;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kVecRows; ++u) {
        const int rl = threadIdx.x / R + u * (kBlock / R);
        if (rl < e.count) {
            const int64_t o = (e.row0 + rl) * R + v;
            acc += r[o] * z[o];
        }
    }
    store_partial<R>(acc, blk, partials);
}

// FP32 V-cycle: z = (double) z32 and the partial <r, z> in one pass (the
// widening is exact, so the products and their order are k_dot_rz's on the
// widened z; one pass over the vectors less than the cast and the dot)
template <int R>
__global__ __launch_bounds__(kBlock) void k_cast_dot_rz(const double *__restrict__ r, const float *__restrict__ z32,
                                                        double *__restrict__ z, const Seg *__restrict__ tab,
                                                        int64_t nrows, double *__restrict__ partials,
                                                        const int *__restrict__ done) {
    MG_ARGS_FIRST("s"(r), "s"(z32), "s"(z), "s"(tab), "s"(nrows), "s"(partials), "s"(done), "s"(gridDim.x));
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const Seg e = vec_seg(tab, blk, nrows, kVecRows * kBlock / R);
    if (done && grid_done<R>(done, e.grid)) return;
    const int v = threadIdx.x % R;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kVecRows; ++u) {
        const int rl = threadIdx.x / R + u * (kBlock / R);
        if (rl < e.count) {
            const int64_t o = (e.row0 + rl) * R + v;
            const double zo = (double)z32[o];
            z[o] = zo;
            acc += r[o] * zo;
        }
    }
    store_partial<R>(acc, blk, partials);
}

// The vector kernels' loads of one thread: its kVecRows rows (a row past the
// chunk's end is read as its last row, and not stored).  The values are
// consumed by an empty asm statement that runs on every path, so that the
// compiler cannot move the loads behind a test of the convergence flag:
// otherwise, the loads being dead when the flag is set, it tests the flag
// first, and every kernel begins with a dependent load of it.
template <int R, int N>
__device__ __forceinline__ void vec_rows(const Seg &e, int v, int64_t (&o)[kVecRows], const double *(&src)[N],
                                         double (&val)[N][kVecRows]) {
#pragma unroll
    for (int u = 0; u < kVecRows; ++u) {
        const int rl = threadIdx.x / R + u * (kBlock / R);
        o[u] = (e.row0 + (rl < e.count ? rl : e.count - 1)) * R + v;
    }
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int u = 0; u < kVecRows; ++u) val[a][u] = src[a][o[u]];
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int u = 0; u < kVecRows; ++u) asm volatile("" ::"v"(val[a][u]));
}

// x += apend p (the previous iteration's x update, deferred to here, where
// p is read anyway), then p = z + beta p.  apend is that iteration's alpha,
// or 0 when nothing is pending (first iteration, or a system that had
// converged before it); a system that converged in it still gets its x
// update, but keeps its p.
// (several grids: a grid whose systems had all converged before the previous
// iteration has nothing pending and returns before loading)
template <int R>
__global__ __launch_bounds__(kBlock) void k_update_p(const double *__restrict__ z, double *__restrict__ p,
                                                     double *__restrict__ x, const Seg *__restrict__ tab,
                                                     int64_t nrows, Scalars sc) {
    MG_ARGS_FIRST("s"(z), "s"(p), "s"(x), "s"(tab), "s"(nrows), "s"(sc.beta), "s"(sc.apend), "s"(sc.done),
                  "s"(gridDim.x));
    const Seg e = vec_seg(tab, xcd_remap(blockIdx.x, gridDim.x), nrows, kVecRows * kBlock / R);
    const int v = threadIdx.x % R;
    const int sys = e.grid * R + v;
    if (tab && sc.done[sys] && sc.apend[sys] == 0.0) return;
    if (e.count <= 0) return;
    int64_t o[kVecRows];
    const double *src[3] = {z, p, x};
    double val[3][kVecRows];
    vec_rows<R, 3>(e, v, o, src, val);
    const double beta = sc.beta[sys], ap = sc.apend[sys];
    const int dn = sc.done[sys];
#pragma unroll
    for (int u = 0; u < kVecRows; ++u) {
        const int rl = threadIdx.x / R + u * (kBlock / R);
        if (rl < e.count) {
            if (ap != 0.0) x[o[u]] = val[2][u] + ap * val[1][u];
            if (!dn) p[o[u]] = val[0][u] + beta * val[1][u];
        }
    }
}

// After the last iteration: the pending x update, x += apend p.
template <int R>
__global__ __launch_bounds__(kBlock) void k_flush_x(double *__restrict__ x, const double *__restrict__ p,
                                                    const Seg *__restrict__ tab, int64_t nrows, Scalars sc) {
    const Seg e = vec_seg(tab, xcd_remap(blockIdx.x, gridDim.x), nrows, kVecRows * kBlock / R);
    const int v = threadIdx.x % R;
    const double ap = sc.apend[e.grid * R + v];
    if (ap == 0.0) return;
#pragma unroll
    for (int u = 0; u < kVecRows; ++u) {
        const int rl = threadIdx.x / R + u * (kBlock / R);
        if (rl < e.count) {
            const int64_t o = (e.row0 + rl) * R + v;
            x[o] = x[o] + ap * p[o];
        }
    }
}

// q = A p, partial <p, q>
// With one rhs every value load and gather of the row is issued before the
// sum uses any of them (136 instead of 68 VGPRs, 3 instead of 7 waves per
// SIMD): the product's 8192 workgroups take several dispatch rounds at any
// occupancy, and more loads in flight per wave took it from 100 to 92 us at
// 128^3.  (The colour passes, whose 1024 workgroups fit in one round at the
// higher occupancy, and the LDS-staged R >= 4 product became slower.)
// PQ = false: q = A p only (the standalone level-0 SpMV, one grid, one rhs),
// with the same loads and sums as inside the solve.
template <int R, int CF, bool PQ = true>
__global__ __launch_bounds__(kBlock) void k_spmv_pq(int64_t n, const double *__restrict__ val,
                                                    const int32_t *__restrict__ col,
                                                    const int8_t *__restrict__ dcol,
                                                    const int32_t *__restrict__ dbase,
                                                    const double *__restrict__ p, double *__restrict__ q,
                                                    const Seg *__restrict__ tab, double *__restrict__ partials,
                                                    const int *__restrict__ done, int spc) {
    // (its arguments are left to the compiler: naming them up front moved the
    // table-entry load to the vector unit and cost 9 us per CG iteration)
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t first = (int64_t)blk * (R == 1 ? 1 : spc);
    // the entries of a workgroup belong to one grid
    if (done && grid_done<R>(done, tab[first].grid)) return;  // done: NULL for one grid
    if constexpr (R >= kPairR) {
        // R/2 lanes per row, two right-hand sides each; values through LDS
        constexpr int LN = pass_lanes(R), RW = kBlock / LN;
        __shared__ double sv2[kW * RW];
        const int w = threadIdx.x % LN, rl = threadIdx.x / LN;
        double acc0 = 0.0, acc1 = 0.0;
        for (int it = 0; it < spc; ++it) {
            const Seg e = tab[first + it];
            stage_values<double, 0u, true, RW, kBlock>(val, e.row0, e.count, sv2);
            if (rl < e.count) {
                const int64_t i = e.row0 + rl;
                const int32_t *sb = CF ? dbase + (e.grid * 8 + e.colour) * kW : nullptr;
                double s2[2], pv[2];
                row_sum2<R, CF>(col, dcol, sb, n, i, p, w, sv2 + rl, RW, s2);
                st_lanes(q + i * R + 2 * w, s2);
                ld_lanes(p + i * R + 2 * w, pv);
                acc0 += pv[0] * s2[0];
                acc1 += pv[1] * s2[1];
            }
            __syncthreads();  // the next entry overwrites sv2
        }
        store_partial2<R>(acc0, acc1, blk, partials);
        return;
    }
    const int v = threadIdx.x % R, rl = threadIdx.x / R;
    double acc = 0.0;
    for (int it = 0; it < (R == 1 ? 1 : spc); ++it) {
        const Seg e = tab[first + it];
        if constexpr (R < kStageR) {
            if (rl < e.count) {
                const int64_t i = e.row0 + rl;
                double d;
                const int32_t *sb = CF ? dbase + (e.grid * 8 + e.colour) * kW : nullptr;
                double s;
                if constexpr (R == 1) {
                    double a[kW], xv[kW];
                    load_row<double, R, 0u, true, CF>(val, col, dcol, sb, n, i, p, v, a, xv);
                    __builtin_amdgcn_sched_barrier(0);  // all loads issued before the sum
                    s = 0.0;
#pragma unroll
                    for (int t = 0; t < kW; ++t)
                        if (a[t] != 0.0) s = s + a[t] * xv[t];
                } else {
                    s = row_sum<double, R, 0u, true, CF>(val, col, dcol, sb, n, i, p, v, d);
                }
                q[i * R + v] = s;
                if constexpr (!PQ) continue;
                if constexpr (R == 1) acc = p[i * R + v] * s;
                else acc += p[i * R + v] * s;
            }
        } else {
            // R lanes per row: the entry's values go through LDS once
            __shared__ double sv[kW * (kBlock / R)];
            stage_values<double, 0u, true, kBlock / R, kBlock>(val, e.row0, e.count, sv);
            if (rl < e.count) {
                const int64_t i = e.row0 + rl;
                double d;
                const int32_t *sb = CF ? dbase + (e.grid * 8 + e.colour) * kW : nullptr;
                const double s = row_sum<double, R, 0u, true, CF, true>(val, col, dcol, sb, n, i, p, v, d,
                                                                         sv + rl, kBlock / R);
                q[i * R + v] = s;
                acc += p[i * R + v] * s;
            }
            __syncthreads();  // the next entry overwrites sv
        }
    }
    if constexpr (PQ) store_partial<R>(acc, blk, partials);
}

// q = A p and partial <p, q>, one grid, R >= kPairR right-hand sides, all
// level-0 extents even and nx a multiple of 2 box_run(R) (BoxGeo).  A
// workgroup owns BX = box_run(R) consecutive half-points in x at one (Y, Z)
// (16, 8, 4 at R = 4, 8, 16, so that its 8 BX rows fill kBlock threads): a
// 2BX x 2 x 2 box of fine points, BX rows of each of the 8 colours.  It stages
// p on the box and its one-point halo ((2BX+2) x 4 x 4 points) in LDS, and its
// rows read their 27 neighbours there: about 5 staged loads per row instead of
// 27 gathers through the texture unit, which bounds the table-driven product
// at R >= 4.  The rows' operator values are staged as in the other paired
// kernels.  Every right-hand side's sum takes row_sum2's slot order and
// operations (a missing neighbour has value 0 and is skipped, so the halo
// outside the grid holds zeros), so q is bit-identical to the table-driven
// product; only the grouping of the <p, q> partials differs.  PQ = false:
// q = A p only (the standalone level-0 product).
template <int R, bool PQ>
__global__ __launch_bounds__(kBlock) void k_spmv_box(const double *__restrict__ val, const double *__restrict__ p,
                                                     double *__restrict__ q, double *__restrict__ partials,
                                                     BoxGeo g) {
    static_assert(R >= kPairR, "two right-hand sides per lane");
    constexpr int LN = pass_lanes(R), BX = box_run(R), RWS = 8 * BX, BS = kBlock;
    constexpr int TX = 2 * BX + 2, TY = 4, TZ = 4, TP = TX * TY * TZ;
    typedef double V2 __attribute__((ext_vector_type(2)));
    constexpr int NP = (TP + RWS - 1) / RWS, NV = (kW * RWS + BS - 1) / BS;
    // (padded to whole rounds of the staging loops, whose stores are then
    // unconditional: a store under a branch drags its load into the branch)
    __shared__ V2 tile[NP * RWS * LN];  // point-major: tile[pt * LN + w] = rhs 2w, 2w+1
    __shared__ double sv[NV * BS];      // sv[s * RWS + row]
    // Boxes in slabs of 8 half-lines in y: x fastest, then y within the slab,
    // then z, then the slab.  The boxes that share halo points with a box are
    // then at most 8 * nxb workgroups apart, and an XCD (a contiguous range of
    // logical blocks) works through one slab at a time, so that its halo reads
    // hit its L2.  (With y before z, the z-neighbours of a box were hy * nxb
    // blocks away, out of the L2, and p was read 2.7 times from memory.)
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int xb = b % g.nxb, t = b / g.nxb;
    const int hz = g.nz >> 1, slab = t / (kBoxSlab * hz);
    const int sy = min(kBoxSlab, g.hy - kBoxSlab * slab), rem = t - slab * kBoxSlab * hz;
    const int Y = kBoxSlab * slab + rem % sy, Z = rem / sy;
    const int x0 = 2 * BX * xb - 1, y0 = 2 * Y - 1, z0 = 2 * Z - 1;  // fine origin of the tile
    const int64_t run = ((int64_t)Z * g.hy + Y) * g.hx + BX * xb;   // the run's offset within a class
    const int w = threadIdx.x % LN, ps = threadIdx.x / LN;
    // All loads are issued before any is used, unconditionally: a point
    // outside the grid (or past the tile) loads from its clamped position and
    // is replaced by zero afterwards.  (A load under a divergent branch is
    // waited for at the end of the branch, one round trip per load.)
    V2 pv[NP];
    bool inside[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int pt = min(ps + RWS * k, TP - 1);
        const int tx = pt % TX, ty = (pt / TX) % TY, tz = pt / (TX * TY);
        const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
        inside[k] = (unsigned)x < (unsigned)g.nx && (unsigned)y < (unsigned)g.ny && (unsigned)z < (unsigned)g.nz;
        const int xc = min(max(x, 0), g.nx - 1), yc = min(max(y, 0), g.ny - 1), zc = min(max(z, 0), g.nz - 1);
        const int pc = (xc & 1) | (yc & 1) << 1 | (zc & 1) << 2;
        const int64_t i = (int64_t)(pc ^ g.flip) * g.nh + ((int64_t)(zc >> 1) * g.hy + (yc >> 1)) * g.hx + (xc >> 1);
        pv[k] = *(const V2 *)(p + i * R + 2 * w);
    }
    double av[NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const int e = min((int)threadIdx.x + u * BS, kW * RWS - 1);  // e = s * RWS + class * BX + j
        const int s = e / RWS, c = (e % RWS) / BX, j = e % BX;
        av[u] = ld<true>(val + ell_index(s, (int64_t)(c ^ g.flip) * g.nh + run + j));
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) tile[(ps + RWS * k) * LN + w] = inside[k] ? pv[k] : V2{0.0, 0.0};
#pragma unroll
    for (int u = 0; u < NV; ++u) sv[threadIdx.x + u * BS] = av[u];
    __syncthreads();
    // row ps: class c = ps / BX, half-point BX xb + j; its fine point in the tile
    const int c = ps / BX, j = ps % BX;
    const int pt0 = (((c >> 2) + 1) * TY + ((c >> 1) & 1) + 1) * TX + 2 * j + (c & 1) + 1;
    // Each right-hand side's sum in slot order, the two side by side, nine
    // slots' LDS reads issued at a time; a zero value (a missing neighbour)
    // leaves the sum as it is, by a select rather than a branch, so that no
    // read waits behind the test of another.
    double s2[2] = {0.0, 0.0};
#pragma unroll
    for (int t0 = 0; t0 < kW; t0 += 9) {
        double a[9];
        V2 xv[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int t = t0 + k;
            a[k] = sv[t * RWS + ps];
            xv[k] = tile[(pt0 + ((t / 9 - 1) * TY + (t / 3 % 3 - 1)) * TX + (t % 3 - 1)) * LN + w];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double n0 = s2[0] + a[k] * xv[k].x, n1 = s2[1] + a[k] * xv[k].y;
            s2[0] = a[k] != 0.0 ? n0 : s2[0];
            s2[1] = a[k] != 0.0 ? n1 : s2[1];
        }
    }
    st_lanes(q + ((int64_t)(c ^ g.flip) * g.nh + run + j) * R + 2 * w, s2);
    if constexpr (PQ) {
        const V2 pc2 = tile[pt0 * LN + w];
        store_partial2<R>(pc2.x * s2[0], pc2.y * s2[1], b, partials);
    }
}

// r -= alpha q; partial ||r||^2 (the x update x += alpha p is deferred to
// the next k_update_p, or to k_flush_x after the last iteration)
// (converged systems: as in k_update_p; their r is not written)
// W32 (FP32 V-cycle): the new r is also stored narrowed into r32, the next
// V-cycle's level-0 right-hand side, instead of a separate cast pass.
template <int R, bool W32>
__device__ __forceinline__ void update_r_body(double *__restrict__ r, const double *__restrict__ q,
                                              const Seg *__restrict__ tab, int64_t nrows,
                                              double *__restrict__ partials, const Scalars &sc,
                                              float *__restrict__ r32) {
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const Seg e = vec_seg(tab, blk, nrows, kVecRows * kBlock / R);
    if (tab && grid_done<R>(sc.done, e.grid)) return;
    const int v = threadIdx.x % R;
    const int sys = e.grid * R + v;
    double acc = 0.0;
    if (e.count > 0) {
        int64_t o[kVecRows];
        const double *src[2] = {r, q};
        double val[2][kVecRows];
        vec_rows<R, 2>(e, v, o, src, val);
        const double alpha = sc.alpha[sys];
        if (!sc.done[sys]) {
#pragma unroll
            for (int u = 0; u < kVecRows; ++u) {
                const int rl = threadIdx.x / R + u * (kBlock / R);
                if (rl < e.count) {
                    const double ri = val[0][u] - alpha * val[1][u];
                    r[o[u]] = ri;
                    if constexpr (W32) r32[o[u]] = (float)ri;
                    acc += ri * ri;
                }
            }
        }
    }
    store_partial<R>(acc, blk, partials);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_update_r(double *__restrict__ r, const double *__restrict__ q,
                                                     const Seg *__restrict__ tab, int64_t nrows,
                                                     double *__restrict__ partials, Scalars sc) {
    MG_ARGS_FIRST("s"(r), "s"(q), "s"(tab), "s"(nrows), "s"(partials), "s"(sc.alpha), "s"(sc.done),
                  "s"(gridDim.x));
    update_r_body<R, false>(r, q, tab, nrows, partials, sc, nullptr);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_update_r32(double *__restrict__ r, const double *__restrict__ q,
                                                       const Seg *__restrict__ tab, int64_t nrows,
                                                       double *__restrict__ partials, Scalars sc,
                                                       float *__restrict__ r32) {
    MG_ARGS_FIRST("s"(r), "s"(q), "s"(tab), "s"(nrows), "s"(partials), "s"(sc.alpha), "s"(sc.done),
                  "s"(gridDim.x), "s"(r32));
    update_r_body<R, true>(r, q, tab, nrows, partials, sc, r32);
}

// One workgroup per grid: sum the grid's partials in a fixed order, then
// update the scalars of its R systems.
//   kInit: nr0 = ||r0||; a zero residual finishes the system with 0 iterations
//   kRz:   rho = <r,z>; beta = rho/rho_old (0 at the first iteration)
//   kPq:   alpha = rho/<p,q>, or a breakdown when <p,q> is not finite and > 0
//   kRr:   record ||r||/||r0|| and test it against tol
// Threads of a finalize workgroup: with R right-hand sides, kBlock/R threads
// per system would need R times as many round trips, so R > 1 uses 1024.
constexpr int fin_block(int R) { return R == 1 ? kBlock : 1024; }

// The body of k_finalize with KU straight-line partial loads per thread and
// round trip (a load past the end rereads the last partial and adds 0):
// 32 for the long ranges of one workgroup per producing block, 4 for folded
// partials, whose few values would otherwise cost 28 redundant loads a
// thread.
template <int R, int KIND, int KU>
__device__ __forceinline__ void finalize_body(int g, int b0, int b1, const double *__restrict__ partials,
                                              const Scalars &sc, double *__restrict__ hist, int hist_cap,
                                              double tol) {
    constexpr int FB = fin_block(R);
    __shared__ double sh[(FB / 64) * R];
    const int v = threadIdx.x % R;
    constexpr int kStep = FB / R;
    double t[KU];
    int b = b0 + threadIdx.x / R;
    if (b1 > b0) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int bb = b + u * kStep;
            t[u] = partials[(int64_t)(bb < b1 ? bb : b1 - 1) * R + v];
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    const bool gdone = KIND != kInit && grid_done<R>(sc.done, g);
    const int sys = g * R + (threadIdx.x < R ? threadIdx.x : 0);
    const int dn = sc.done[sys];
    const int it0 = (KIND == kRz || KIND == kRr) ? sc.iter[sys] : 0;
    const double rho_old = KIND == kRz ? sc.rho_old[sys] : 0.0;
    const double rho = KIND == kPq ? sc.rho[sys] : 0.0;
    const double nr0 = KIND == kRr ? sc.nr0[sys] : 0.0;
    const double alpha = KIND == kRr ? sc.alpha[sys] : 0.0;
    // the deferred x update of the previous iteration was applied by the
    // k_update_p that ran before this reduction: nothing is pending now
    if (KIND == kPq && threadIdx.x < R) sc.apend[sys] = 0.0;
    double s = 0.0;
    while (b < b1) {
#pragma unroll
        for (int u = 0; u < KU; ++u) s += (b + u * kStep < b1) ? t[u] : 0.0;
        b += KU * kStep;
        if (b < b1) {
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int bb = b + u * kStep;
                t[u] = partials[(int64_t)(bb < b1 ? bb : b1 - 1) * R + v];
            }
        }
    }
    if (gdone) return;  // uniform over the workgroup
    const double tot = block_sum<R, FB>(s, sh);
    if (threadIdx.x >= R) return;
    if (KIND == kInit) {
        const double n0 = sqrt(tot);
        sc.nr0[sys] = n0;
        if (n0 == 0.0) {
            sc.done[sys] = 1;
            sc.status[sys] = 1;
            atomicAdd(sc.ndone, 1);
        }
        return;
    }
    if (dn) return;
    if (KIND == kRz) {
        sc.beta[sys] = (it0 == 0) ? 0.0 : tot / rho_old;
        sc.rho[sys] = tot;
        sc.rho_old[sys] = tot;
    } else if (KIND == kPq) {
        sc.pq[sys] = tot;
        if (!(tot > 0.0) || !isfinite(tot)) {
            sc.alpha[sys] = 0.0;
            sc.status[sys] = MGPCG_ERR_BREAKDOWN;
            sc.done[sys] = 1;
            atomicAdd(sc.ndone, 1);
        } else {
            sc.alpha[sys] = rho / tot;
        }
    } else {
        // this iteration's x update, applied by the next k_update_p (or by
        // k_flush_x), also when the system converges now
        sc.apend[sys] = alpha;
        const int k = it0 + 1;
        sc.iter[sys] = k;
        const double rel = sqrt(tot) / nr0;
        if (k <= hist_cap) hist[(int64_t)sys * hist_cap + (k - 1)] = rel;
        if (tol > 0.0 && rel <= tol) {
            sc.done[sys] = 1;
            sc.status[sys] = 1;
            atomicAdd(sc.ndone, 1);
        }
    }
}

// One grid (gb == NULL): the partials are [0, nblk), so their loads wait for
// no table load.  The convergence flags and the scalars of the update are
// loaded after the partials are on their way, so that both take one memory
// round trip.
template <int R, int KIND>
__global__ __launch_bounds__(fin_block(R)) void k_finalize(const int *__restrict__ gb, int nblk,
                                                           const double *__restrict__ partials, Scalars sc,
                                                           double *__restrict__ hist, int hist_cap, double tol) {
    MG_ARGS_FIRST("s"(gb), "s"(nblk), "s"(partials), "s"(sc.done), "s"(sc.iter));
    const int g = blockIdx.x;
    const int b0 = gb ? gb[g] : 0, b1 = gb ? gb[g + 1] : nblk;
    if (b1 - b0 <= 4 * (fin_block(R) / R))
        finalize_body<R, KIND, 4>(g, b0, b1, partials, sc, hist, hist_cap, tol);
    else
        finalize_body<R, KIND, 32>(g, b0, b1, partials, sc, hist, hist_cap, tol);  // 64 would spill at 1024 threads
}

// One grid with R > 1: the per-workgroup partials of a reduction (nblk * R
// of them, up to 2M at 16 right-hand sides) are more than one finalize
// workgroup reads quickly.  kFoldBlocks workgroups first sum fixed,
// contiguous slices of them, each in a fixed order, into fold[w * R + rhs].
template <int R>
__global__ __launch_bounds__(kBlock) void k_fold(const double *__restrict__ partials, int nblk,
                                                 double *__restrict__ fold) {
    MG_ARGS_FIRST("s"(partials), "s"(nblk), "s"(fold));
    __shared__ double sh[(kBlock / 64) * R];
    const int w = blockIdx.x;
    const int b0 = (int)((int64_t)nblk * w / kFoldBlocks), b1 = (int)((int64_t)nblk * (w + 1) / kFoldBlocks);
    const int v = threadIdx.x % R;
    constexpr int kStep = kBlock / R, kU = 8;
    double s = 0.0;
    for (int b = b0 + threadIdx.x / R; b < b1; b += kU * kStep) {
        double t[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int bb = b + u * kStep;
            t[u] = bb < b1 ? partials[(int64_t)bb * R + v] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) s += t[u];
    }
    const double tot = block_sum<R>(s, sh);
    if (threadIdx.x < R) fold[w * R + threadIdx.x] = tot;
}

template <int KIND>
static hipError_t finalize(const mgpcg_problem *P, int table, double tol, int hist_cap, hipStream_t s,
                           int nparts = 0) {
    const int *gb = P->red_gb[table];
    const double *parts = P->sc.partials;
    // partials of one grid: the workgroups of the producing kernel(s)
    // (nparts > 0: a kernel outside the tables, one grid)
    int nblk = nparts > 0 ? nparts : table == 2 ? (int)P->rz_off[8] : P->n_red[table];
    if (P->fold) {
        MG_DISPATCH_R(P->R, (k_fold<RR><<<kFoldBlocks, kBlock, 0, s>>>(P->sc.partials, nblk, P->fold)));
        parts = P->fold;
        nblk = kFoldBlocks;
    }
    if (P->G == 1) gb = nullptr;  // the range [0, nblk) travels as an argument
    MG_DISPATCH_R(P->R, (k_finalize<RR, KIND><<<P->G, fin_block(RR), 0, s>>>(gb, nblk, parts, P->sc, P->hist,
                                                                              hist_cap, tol)));
    return hipGetLastError();
}

// SpMV-type kernels: one row per R threads, spc table entries per workgroup
// (table 0); vector kernels: kVecRows*kBlock/R rows per workgroup (table 1).
hipError_t launch_init_residual(const mgpcg_problem *P, hipStream_t s) {
    const Level &L = P->lev[0];
#define MG_INITR(CFV)                                                                                  \
    MG_DISPATCH_R(P->R, (k_init_residual<RR, CFV><<<P->n_red[0], kBlock, 0, s>>>(                       \
                            L.n, L.val64, L.col, L.dcol, L.dbase, P->b, P->x, P->r, P->red_tab[0], P->sc.partials, \
                            P->spc)));
    if (L.cf == 2) { MG_INITR(2) } else if (L.cf == 1) { MG_INITR(1) } else { MG_INITR(0) }
#undef MG_INITR
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize<kInit>(P, 0, 0.0, 0, s);
}
hipError_t launch_dot_rz(const mgpcg_problem *P, hipStream_t s) {
    const bool one = P->G == 1;
    MG_DISPATCH_R(P->R, (k_dot_rz<RR><<<P->n_red[1], kBlock, 0, s>>>(P->r, P->z, one ? nullptr : P->red_tab[1],
                                                                     P->lev[0].n, P->sc.partials,
                                                                     one ? nullptr : P->sc.done)));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize<kRz>(P, 1, 0.0, 0, s);
}
hipError_t launch_cast_dot_rz(const mgpcg_problem *P, hipStream_t s) {
    const bool one = P->G == 1;
    MG_DISPATCH_R(P->R, (k_cast_dot_rz<RR><<<P->n_red[1], kBlock, 0, s>>>(
                            P->r, (const float *)P->lev[0].z, P->z, one ? nullptr : P->red_tab[1], P->lev[0].n,
                            P->sc.partials, one ? nullptr : P->sc.done)));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize<kRz>(P, 1, 0.0, 0, s);
}
hipError_t launch_finalize_rz(const mgpcg_problem *P, hipStream_t s) { return finalize<kRz>(P, 2, 0.0, 0, s); }
hipError_t launch_update_p(const mgpcg_problem *P, hipStream_t s) {
    const bool one = P->G == 1;
    MG_DISPATCH_R(P->R, (k_update_p<RR><<<P->n_red[1], kBlock, 0, s>>>(P->z, P->p, P->x,
                                                                       one ? nullptr : P->red_tab[1], P->lev[0].n,
                                                                       P->sc)));
    return hipGetLastError();
}
hipError_t launch_flush_x(const mgpcg_problem *P, hipStream_t s) {
    const bool one = P->G == 1;
    MG_DISPATCH_R(P->R, (k_flush_x<RR><<<P->n_red[1], kBlock, 0, s>>>(P->x, P->p, one ? nullptr : P->red_tab[1],
                                                                      P->lev[0].n, P->sc)));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_fill_d(P->sc.apend, P->S, 0.0, s);
}
hipError_t launch_spmv_pq(const mgpcg_problem *P, hipStream_t s) {
    const Level &L = P->lev[0];
    if (P->box_ok) {
        hipError_t e = launch_spmv_box<true>(P, P->p, P->q, s);
        if (e != hipSuccess) return e;
        return finalize<kPq>(P, 0, 0.0, 0, s, P->n_box);
    }
#define MG_SPMVPQ(CFV)                                                                                 \
    MG_DISPATCH_R(P->R, (k_spmv_pq<RR, CFV><<<P->n_red[0], kBlock, 0, s>>>(                             \
                            L.n, L.val64, L.col, L.dcol, L.dbase, P->p, P->q, P->red_tab[0], P->sc.partials, \
                            P->G == 1 ? nullptr : P->sc.done, P->spc)));
    if (L.cf == 2) { MG_SPMVPQ(2) } else if (L.cf == 1) { MG_SPMVPQ(1) } else { MG_SPMVPQ(0) }
#undef MG_SPMVPQ
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize<kPq>(P, 0, 0.0, 0, s);
}
hipError_t launch_update_r(const mgpcg_problem *P, double tol, int hist_cap, hipStream_t s, float *r32) {
    const bool one = P->G == 1;
    if (r32) {
        MG_DISPATCH_R(P->R, (k_update_r32<RR><<<P->n_red[1], kBlock, 0, s>>>(
                                P->r, P->q, one ? nullptr : P->red_tab[1], P->lev[0].n, P->sc.partials, P->sc, r32)));
    } else {
        MG_DISPATCH_R(P->R, (k_update_r<RR><<<P->n_red[1], kBlock, 0, s>>>(
                                P->r, P->q, one ? nullptr : P->red_tab[1], P->lev[0].n, P->sc.partials, P->sc)));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize<kRr>(P, 1, tol, hist_cap, s);
}

}  // namespace mg
