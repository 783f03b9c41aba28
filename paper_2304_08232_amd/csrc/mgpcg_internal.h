// Internal structures of the MI355X MG-PCG library (not part of the ABI).
//
// Data layout in HBM (per level l, all grids of the problem):
//   rows are colour-major across grids: for colour k = 0..7, for grid g, the
//   points of grid g with colour k in lexicographic order of their half-grid
//   coordinates (ix>>1, iy>>1, iz>>1).  Consecutive rows of one colour are
//   consecutive points along x, so the neighbour in a fixed stencil direction
//   of consecutive rows is again consecutive: every gather of the sweep reads
//   near-contiguous memory.
//   The operator is 27-slot ELL, blocked by wavefront (ell_index below):
//   slot s is direction (dx,dy,dz) = (s%3-1, s/3%3-1, s/9-1), i.e. ascending
//   natural column order; slot 13 is the diagonal; a missing neighbour is a
//   padding slot with value 0.  Columns are stored in one of three formats
//   (Level::cf): int32, int8 deltas against per-colour bases, or implied by
//   the bases alone.
//   Vectors with R right-hand sides are interleaved: element (row i, rhs v) at
//   i*R + v.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "mgpcg.h"

namespace mg {

constexpr int kW = 27;        // ELL width (3x3x3 stencil)
constexpr int kCentre = 13;   // slot of the diagonal
constexpr int kBlock = 256;   // threads per workgroup
constexpr int kVecRows = 4;   // rows per thread in the CG vector kernels
constexpr int kFoldBlocks = 256;  // workgroups that pre-sum the CG partials (one grid, R > 1)
constexpr int kXcdCount = 8;     // XCDs of the part; workgroup b is dispatched to XCD b % 8
// Workgroup size of a colour pass: 256 threads on streamed (large) levels;
// one wavefront on cache-resident levels, whose passes are latency-bound, so
// that their few rows are spread over as many CUs as possible.
constexpr int pass_block(bool streamed) { return streamed ? 256 : 64; }
// With R >= kPairR right-hand sides a colour-pass lane updates two of them
// (16-byte accesses: half the address work per gathered byte), so a row has
// R/2 lanes and a workgroup twice the rows.
constexpr int kPairR = 4;
constexpr int pass_lanes(int R) { return R >= kPairR ? R / 2 : R; }
constexpr int pass_rows(bool streamed, int R) { return pass_block(streamed) / pass_lanes(R); }
// box-tiled CG product (R >= kPairR): half-points in x per box, so that the
// box's 8 * box_run(R) rows fill a kBlock-thread workgroup
constexpr int box_run(int R) { return kBlock / 8 / pass_lanes(R); }
constexpr int kBoxSlab = 8;  // half-lines in y per slab of the box order
// threads of the single-workgroup coarsest-level kernel; it is used only when
// every colour of that level has at most this many rows
constexpr int kTailBlock = 512;

// Operator storage (ELL-27, blocked by wavefront): rows are grouped in blocks
// of 64; a block holds its 27 slots one after another, each as 64 consecutive
// entries.  Slot s of row i is at ell_index(s, i).  A wavefront of 64
// consecutive rows therefore reads its whole operator from one contiguous
// run, and each of its slot loads is 64 consecutive entries.
constexpr int kEllRows = 64;
__host__ __device__ inline int64_t ell_index(int64_t s, int64_t i) {
    return (i / kEllRows) * (kW * kEllRows) + s * kEllRows + (i % kEllRows);
}
inline int64_t ell_size(int64_t n) { return (n + kEllRows - 1) / kEllRows * kEllRows * kW; }
// Delta-coded columns: four 8-bit deltas per 32-bit word, blocked like the
// values.  Word delta_word(q, i) holds slots 4q..4q+3 of row i, slot s in
// byte s % 4, so a row's 27 deltas are 7 coalesced word loads.
constexpr int kDeltaWords = (kW + 3) / 4;
__host__ __device__ inline int64_t delta_word(int64_t q, int64_t i) {
    return (i / kEllRows) * (kDeltaWords * kEllRows) + q * kEllRows + (i % kEllRows);
}
inline int64_t delta_bytes(int64_t n) { return (n + kEllRows - 1) / kEllRows * kEllRows * kDeltaWords * 4; }

// One workgroup's share of rows: [row0, row0+count), all in grid `grid`.
struct Seg {
    int64_t row0;
    int32_t count;
    int16_t grid;
    int16_t colour;
};

// One launch of the sequential smoother's schedule: wavefronts w0 .. w1-1,
// either a run of small wavefronts swept by one workgroup of `threads`
// threads (run), or one wavefront over as many workgroups as it needs.
struct WaveSeg {
    int w0, w1;
    bool run;
    int threads;
};

struct LevelGrid {  // one grid at one level
    int nx, ny, nz;
    int ncol;            // colours of this grid (8 unless a dim is 1)
    int64_t nat_off;     // first row of this grid in the natural packed order
    int64_t seg_off[8];  // first internal row of (colour k, this grid)
    int64_t seg_len[8];  // rows of (colour k, this grid)
    int inj_colour;      // colour holding the injection points (2jx,2jy,2jz)
};

struct Level {
    int64_t n = 0;       // rows, all grids
    int64_t nnz = 0;     // structural nonzeros
    int ncol = 0;        // colour passes (max over grids)
    std::vector<LevelGrid> grids;
    std::vector<int64_t> coff;  // ncol+1: internal row range of each colour (all grids)

    double *val64 = nullptr;  // at ell_index(s, i): FP64 operator (level 0 always; all levels if FP64 V-cycle)
    float *val32 = nullptr;   // at ell_index(s, i): FP32 operator (FP32 V-cycle)
    int32_t *col = nullptr;   // at ell_index(s, i): absolute columns (NULL when delta-coded)
    // delta-coded columns: col(i,s) = i + dbase[grid(i)][colour(i)][s] + delta(s, i),
    // the deltas packed four to a word at delta_word(s / 4, i), byte s % 4;
    // used when every real entry's delta fits in int8
    int8_t *dcol = nullptr;
    // column format: 0 int32 columns (col), 1 int8 deltas (dcol + dbase),
    // 2 every delta zero, the columns implied by the bases (dbase only)
    int cf = 0;
    int32_t *dbase = nullptr; // [G][8][27] column bases (compact formats)
    int32_t *grid_of_row = nullptr;  // internal row -> grid (G > 1, compact formats)
    std::vector<int32_t> dbase_host;
    int32_t *perm = nullptr;  // natural packed row -> internal row
    int32_t *iperm = nullptr; // internal row -> natural packed row
    int32_t *grid_of_nat = nullptr;  // natural packed row -> grid (only when G > 1)

    // colour-pass tables: entries of colour k are pass_tab[pass_first[k] .. pass_first[k+1]);
    // the active pair is variant [stream_nt] of pass_tab_v / pass_first_v
    // (the segment length follows the workgroup size, pass_rows(stream_nt, R))
    Seg *pass_tab = nullptr;
    std::vector<int> pass_first;
    Seg *pass_tab_v[2] = {nullptr, nullptr};
    std::vector<int> pass_first_v[2];
    uint32_t zi_skip[8] = {0};  // zero-start forward pass: slots whose neighbour is not yet written
    bool zs_ok = true;          // the zero-start pass is valid for every grid of the level
    bool zs_std = true;         // ... and its masks are the standard 8-colour ones (compiled in)
    // the colour passes use 256-thread workgroups and stream the operator with
    // non-temporal loads (set by default when it is larger than the caches);
    // otherwise one-wave workgroups and cached loads.  A schedule choice.
    bool stream_nt = true;
    bool fuse_transfers = false;  // colour 0 is exactly the injection set, in injection order, and is
                                  // swept last by the pre- and first by the post-smoother

    // injection to level+1, sorted by fine internal row
    int32_t *inj_fine = nullptr;
    int32_t *inj_coarse = nullptr;
    int64_t n_inj = 0;

    // sequential smoother (Eq. (1)) by wavefronts t = ix + 2 iy + 4 iz:
    // positions woff[t] .. woff[t+1] (multiples of 64) hold the rows of
    // wavefront t; wrow maps a position to its internal row (-1: padding);
    // wval / wcol at ell_index(s, position) are the row's values and internal
    // columns (padding slots: value 0, column = the row itself)
    int nwave = 0;
    int64_t npos = 0;
    std::vector<int64_t> woff;
    std::vector<int64_t> wcnt;   // rows of each wavefront (unpadded)
    int64_t *woff_dev = nullptr;
    int32_t *wrow = nullptr;
    int32_t *wcol = nullptr;
    double *wval = nullptr;
    std::vector<WaveSeg> wplan;  // launches of the forward sweep, in order

    // V-cycle workspaces in the V-cycle precision (n*R elements)
    void *r = nullptr;
    void *z = nullptr;
    // FP64 scratch for the per-level API entry points (n*R elements each)
    double *t0 = nullptr, *t1 = nullptr, *t2 = nullptr;
};

// device view of one level for the persistent coarse-level kernel
struct CoarseLevel {
    int64_t n;
    const void *val;
    const int32_t *col;
    const int8_t *dcol;
    const int32_t *dbase;
    void *r, *z;
    const int32_t *inj_fine;    // injection rows (to level+1), sorted
    const int32_t *inj_coarse;  // their coarse rows
    int64_t n_inj;
    int64_t coff[9];
};
// operations of the persistent coarse-level kernel's phase program; a phase
// is level | colour << 4 | op << 8
enum CoarseOp { kOpPlain = 0, kOpZeroStart = 1, kOpFusedRestrict = 2, kOpFusedProlong = 3,
                kOpRestrict = 4, kOpProlong = 5, kOpTwice = 6, kOpTwiceZeroStart = 7 };
constexpr int kMaxPhases = 320;
struct CoarseArgs {
    CoarseLevel lev[MGPCG_MAX_LEVELS];
    int nphases;
    uint16_t phase[kMaxPhases];
    int cf;               // column format of every coarse level (Level::cf)
    unsigned *flags;       // one per workgroup
    unsigned *epoch_base;  // advanced by the kernel at each launch
    int *err;              // set when a barrier wait times out
    long long spin_limit;
};

// Level-0 geometry of the box-tiled CG product (one grid, R >= kPairR, all
// extents even, nx a multiple of 2 box_run(R)).  Every colour then has nh
// rows, and the points of parity class pc = (x&1) + 2(y&1) + 4(z&1) (colour
// pc, or 7 - pc = pc ^ 7 under colour order 1) start at row (pc ^ flip) * nh;
// within a class, rows follow the half-grid coordinates (x>>1, y>>1, z>>1),
// x fastest.  (Arithmetic, not a table: a table indexed per lane would be
// read from the kernel arguments by a dependent vector load.)
struct BoxGeo {
    int nx, ny, nz;  // fine extents
    int hx, hy;      // half extents in x and y
    int nxb;         // boxes per half-line (hx / box_run(R))
    int32_t nh;      // rows per colour
    int flip;        // 0 or 7
};

struct Scalars {  // per-system CG state, device arrays of S entries
    double *rho, *rho_old, *alpha, *beta, *nr0, *pq;
    double *apend;       // alpha of the x update still pending (0: none)
    int *iter, *done, *status;
    int *ndone;          // one counter: systems finished
    double *partials;    // reduction blocks * R
};

}  // namespace mg

struct mgpcg_problem {
    int device = 0;
    int G = 1, R = 1, S = 1, L = 1;
    int mg_dtype = MGPCG_FP64;
    int colour_order = 0;
    int smoother = MGPCG_SMOOTHER_COLOURED;
    int sweeps = 1;  // symmetric sweeps per smoothing step of the V-cycle
    int lex_run_rows = 256;  // sequential smoother: largest wavefront a single-workgroup run takes
    // most compact column format allowed (Level::cf), 2 by default
    int col_format = 2;
    std::vector<int> dims0;  // 3*G, level 0
    std::vector<mg::Level> lev;

    // device copies of small tables
    int *d_dims0 = nullptr;        // 3*G
    int64_t *d_natoff0 = nullptr;  // G+1 natural offsets at level 0
    std::vector<int64_t *> d_natoff;  // per level, G+1

    // level-0 reduction tables (grid-homogeneous segments, grouped by grid):
    // [0] one row per thread (SpMV-type CG kernels), [1] kVecRows rows per
    // thread (vector kernels).  gb: G+1 first table entry of each grid.
    // red_gb[2] covers the <r,z> partials that the level-0 post-smoother
    // writes when fuse_rz is set (one per workgroup of its last update of
    // each colour; colour k's start at rz_off[k]).
    mg::Seg *red_tab[2] = {nullptr, nullptr};
    int n_red[2] = {0, 0};  // workgroups of the kernels that walk table 0 / table 1
    int spc = 1;            // table-0 entries per workgroup (R > 1: see the table build)
    // one grid with R > 1: the per-workgroup partials are first summed by
    // kFoldBlocks workgroups into fold[w * R + rhs], and the finalize reads
    // those; NULL otherwise
    double *fold = nullptr;
    int *red_gb[3] = {nullptr, nullptr, nullptr};
    bool fuse_rz = false;
    int64_t rz_off[9] = {};
    // box-tiled CG product (k_spmv_box) and its workgroup count
    bool box_ok = false;
    mg::BoxGeo box{};
    int n_box = 0;

    // CG vectors, level 0, internal layout, n0*R doubles
    double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *b = nullptr;
    mg::Scalars sc{};
    double *hist = nullptr;  // S * hist_cap
    int hist_cap = 0;
    int last_max_iters = 0;
    double last_tol = 0.0;

    // Convergence checks of tolerance-driven solves: after an iteration the
    // count of finished systems is copied into a host-pinned slot and an
    // event recorded; the host reads a slot only once a later iteration is
    // queued behind it, so the device never waits for the host.
    static constexpr int kCheckRing = 4;
    int *pinned_ndone = nullptr;  // kCheckRing slots
    hipEvent_t check_ev[kCheckRing] = {};

    // persistent coarse-level V-cycle (levels coarse_lc..L-1 in one launch)
    bool coarse_ok = false;   // supported for this problem
    int coarse_mode = 0;      // 1: use it when supported; 0: one kernel per pass (default: faster here)
    int coarse_lc = 1;
    int coarse_blocks = 0;
    mg::CoarseArgs coarse_args{};
    unsigned *coarse_flags = nullptr;   // coarse_blocks + 1 (last: epoch base)
    // coarsest level in one workgroup with r and z in LDS
    bool tail_ok = false;
    int tail_on = 1;           // schedule choice: use the tail kernel when tail_ok
    int tail_lw = 0;
    int *coarse_err = nullptr;

    // captured iteration graph
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t iter_graph = nullptr;
    int use_graph = 1;
};
