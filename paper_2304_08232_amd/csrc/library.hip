// Host side of the MG-PCG library: hierarchy setup, V-cycle and PCG drivers,
// iteration graph capture, and the C ABI declared in mgpcg.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "kernels.h"

using namespace mg;

namespace {

thread_local std::string g_err;

mgpcg_status fail(mgpcg_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

mgpcg_status hip_fail(hipError_t e, const char *where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return MGPCG_ERR_HIP;
}

#define HIP_TRY(expr)                                              \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);          \
    } while (0)

template <typename T>
mgpcg_status dalloc(T **p, int64_t count) {
    *p = nullptr;
    if (count <= 0) return MGPCG_OK;
    hipError_t e = hipMalloc((void **)p, (size_t)count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(MGPCG_ERR_OOM, std::string("hipMalloc of ") + std::to_string((size_t)count * sizeof(T)) +
                                       " bytes failed: " + hipGetErrorString(e));
    }
    return MGPCG_OK;
}

#define ST_TRY(expr)                         \
    do {                                     \
        mgpcg_status s_ = (expr);            \
        if (s_ != MGPCG_OK) return s_;       \
    } while (0)

template <typename T>
mgpcg_status upload(T **dst, const std::vector<T> &src, hipStream_t s) {
    ST_TRY(dalloc(dst, (int64_t)src.size()));
    if (!src.empty()) {
        HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // src is pageable and about to go away
    }
    return MGPCG_OK;
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

// --------------------------------------------------------------- colouring
//
// Greedy first-fit colouring in ascending row order (Sec. III-A of the paper)
// on the 27-point grid produces the parity code (ix&1) + 2(iy&1) + 4(iz&1)
// over the dimensions of extent >= 2 (bits of extent-1 dimensions are always
// 0 and are dropped from the numbering).  colour_order 1 reverses the
// numbering.  These helpers map parity bits <-> colour numbers for one grid.

struct Colouring {
    int nbits = 0;
    int bitpos[3] = {-1, -1, -1};  // position of the x/y/z parity bit in the colour number
    int ncol = 1;
    int order = 0;
    Colouring(int nx, int ny, int nz, int ord) {
        int d[3] = {nx, ny, nz};
        for (int a = 0; a < 3; ++a)
            if (d[a] >= 2) bitpos[a] = nbits++;
        ncol = 1 << nbits;
        order = ord;
    }
    int colour(int bx, int by, int bz) const {
        int b[3] = {bx, by, bz}, c = 0;
        for (int a = 0; a < 3; ++a)
            if (bitpos[a] >= 0) c |= b[a] << bitpos[a];
        return order ? ncol - 1 - c : c;
    }
    void parity(int k, int *b) const {
        int c = order ? ncol - 1 - k : k;
        for (int a = 0; a < 3; ++a) b[a] = bitpos[a] >= 0 ? (c >> bitpos[a]) & 1 : 0;
    }
};

// points of a dimension of extent `ext` whose coordinate has parity `bit`
inline int64_t half_count(int ext, int bit) { return ext >= 2 ? (ext + 1 - bit) / 2 : (bit ? 0 : 1); }

// <r,z> partials of the level-0 post-smoother: one per workgroup of the last
// update of each colour; colour k's first at off[k] (off[8]: the count)
void rz_layout(const mgpcg_problem *P, bool wide, int64_t *off) {
    const Level &L0 = P->lev[0];
    const int rows = pass_rows(wide, P->R);
    off[0] = 0;
    for (int k = 0; k < 8; ++k) off[k + 1] = off[k] + (L0.coff[k + 1] - L0.coff[k] + rows - 1) / rows;
}

// rz_off and the finalize table red_gb[2] for the current level-0 workgroup size
hipError_t set_rz_layout(mgpcg_problem *P, hipStream_t s) {
    rz_layout(P, P->lev[0].stream_nt, P->rz_off);
    const int gb[2] = {0, (int)P->rz_off[8]};
    hipError_t e = hipMemcpyAsync(P->red_gb[2], gb, sizeof(gb), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);  // gb lives on this stack frame
}

// Forward launch plan of the sequential smoother on one level: each maximal
// run of consecutive wavefronts with at most run_rows rows goes to one
// single-workgroup launch, every larger wavefront gets a launch of its own.
void make_wave_plan(Level &Lv, int run_rows) {
    Lv.wplan.clear();
    WaveSeg run{0, 0, true, 0};
    auto close_run = [&]() {
        if (run.w1 > run.w0) Lv.wplan.push_back(run);
        run = WaveSeg{0, 0, true, 0};
    };
    for (int t = 0; t < Lv.nwave; ++t) {
        const int padded = (int)(Lv.woff[t + 1] - Lv.woff[t]);
        if (run_rows > 0 && Lv.wcnt[t] <= run_rows) {
            if (run.w1 == run.w0) run.w0 = t;
            run.w1 = t + 1;
            run.threads = std::max(run.threads, std::max(padded, kEllRows));
        } else {
            close_run();
            if (Lv.wcnt[t] > 0) Lv.wplan.push_back(WaveSeg{t, t + 1, false, 0});
        }
    }
    close_run();
}

// Tables of the sequential smoother on one level (the wavefront-major copy
// but for its values): every point gets the wavefront number
// t = ix + 2 iy + 4 iz; a wavefront's rows are kept in internal row order and
// its positions are padded to a multiple of 64.
mgpcg_status build_waves(mgpcg_problem *P, int l, const std::vector<int32_t> &perm,
                         const std::vector<int32_t> &iperm, hipStream_t s) {
    Level &Lv = P->lev[l];
    int nw = 0;
    for (const LevelGrid &lg : Lv.grids) nw = std::max(nw, (lg.nx - 1) + 2 * (lg.ny - 1) + 4 * (lg.nz - 1) + 1);
    auto wave_of = [](int ix, int iy, int iz) { return ix + 2 * iy + 4 * iz; };
    std::vector<int64_t> cnt(nw, 0);
    for (const LevelGrid &lg : Lv.grids)
        for (int iz = 0; iz < lg.nz; ++iz)
            for (int iy = 0; iy < lg.ny; ++iy)
                for (int ix = 0; ix < lg.nx; ++ix) ++cnt[wave_of(ix, iy, iz)];
    std::vector<int64_t> woff(nw + 1, 0);
    for (int t = 0; t < nw; ++t) woff[t + 1] = woff[t] + (cnt[t] + kEllRows - 1) / kEllRows * kEllRows;
    const int64_t npos = woff[nw];
    if (ell_size(npos) >= ((int64_t)1 << 31)) return fail(MGPCG_ERR_DIMS, "problem too large for the sequential smoother");
    std::vector<int32_t> wrow(npos, -1);
    std::vector<int64_t> fill(woff.begin(), woff.end() - 1);
    for (const LevelGrid &lg : Lv.grids)
        for (int iz = 0; iz < lg.nz; ++iz)
            for (int iy = 0; iy < lg.ny; ++iy)
                for (int ix = 0; ix < lg.nx; ++ix) {
                    const int64_t q = lg.nat_off + ix + (int64_t)lg.nx * (iy + (int64_t)lg.ny * iz);
                    wrow[fill[wave_of(ix, iy, iz)]++] = perm[q];
                }
    for (int t = 0; t < nw; ++t) std::sort(wrow.begin() + woff[t], wrow.begin() + woff[t] + cnt[t]);
    std::vector<int32_t> wcol(ell_size(npos), 0);
    std::vector<int64_t> natoff;
    for (const LevelGrid &lg : Lv.grids) natoff.push_back(lg.nat_off);
    for (int64_t p = 0; p < npos; ++p) {
        const int32_t i = wrow[p];
        if (i < 0) continue;
        const int64_t q = iperm[i];
        const int g = (int)(std::upper_bound(natoff.begin(), natoff.end(), q) - natoff.begin()) - 1;
        const LevelGrid &lg = Lv.grids[g];
        const int64_t loc = q - lg.nat_off;
        const int ix = (int)(loc % lg.nx), iy = (int)((loc / lg.nx) % lg.ny), iz = (int)(loc / ((int64_t)lg.nx * lg.ny));
        for (int sl = 0; sl < kW; ++sl) {
            const int jx = ix + sl % 3 - 1, jy = iy + (sl / 3) % 3 - 1, jz = iz + sl / 9 - 1;
            const bool in = jx >= 0 && jx < lg.nx && jy >= 0 && jy < lg.ny && jz >= 0 && jz < lg.nz;
            wcol[ell_index(sl, p)] = in ? perm[lg.nat_off + jx + (int64_t)lg.nx * (jy + (int64_t)lg.ny * jz)] : i;
        }
    }
    ST_TRY(upload(&Lv.woff_dev, woff, s));
    ST_TRY(upload(&Lv.wrow, wrow, s));
    ST_TRY(upload(&Lv.wcol, wcol, s));
    Lv.nwave = nw;
    Lv.npos = npos;
    Lv.woff = woff;
    Lv.wcnt = cnt;
    make_wave_plan(Lv, P->lex_run_rows);
    return MGPCG_OK;
}

mgpcg_status build_hierarchy(mgpcg_problem *P, const double *theta, hipStream_t s) {
    const int G = P->G, R = P->R, L = P->L;
    P->lev.resize(L);
    P->d_natoff.assign(L, nullptr);
    std::vector<int> dims0 = P->dims0;
    ST_TRY(upload(&P->d_dims0, dims0, s));

    for (int l = 0; l < L; ++l) {
        Level &Lv = P->lev[l];
        Lv.grids.resize(G);
        int64_t nat = 0;
        Lv.ncol = 0;
        for (int g = 0; g < G; ++g) {
            LevelGrid &lg = Lv.grids[g];
            lg.nx = dims0[3 * g] >> l;
            lg.ny = dims0[3 * g + 1] >> l;
            lg.nz = dims0[3 * g + 2] >> l;
            Colouring C(lg.nx, lg.ny, lg.nz, P->colour_order);
            lg.ncol = C.ncol;
            lg.nat_off = nat;
            nat += (int64_t)lg.nx * lg.ny * lg.nz;
            Lv.nnz += (int64_t)(3 * lg.nx - 2) * (3 * lg.ny - 2) * (3 * lg.nz - 2);
            Lv.ncol = std::max(Lv.ncol, C.ncol);
            for (int k = 0; k < 8; ++k) {
                lg.seg_len[k] = 0;
                if (k < C.ncol) {
                    int b[3];
                    C.parity(k, b);
                    lg.seg_len[k] = half_count(lg.nx, b[0]) * half_count(lg.ny, b[1]) * half_count(lg.nz, b[2]);
                }
            }
            lg.inj_colour = C.colour(0, 0, 0);
        }
        Lv.n = nat;
        // colour-major across grids
        Lv.coff.assign(Lv.ncol + 1, 0);
        int64_t off = 0;
        for (int k = 0; k < Lv.ncol; ++k) {
            Lv.coff[k] = off;
            for (int g = 0; g < G; ++g) {
                Lv.grids[g].seg_off[k] = off;
                off += Lv.grids[g].seg_len[k];
            }
        }
        Lv.coff[Lv.ncol] = off;
        if (off != Lv.n) return fail(MGPCG_ERR_DIMS, "internal: colour classes do not cover the grid");
        if (ell_size(Lv.n) >= ((int64_t)1 << 31) || Lv.n * R >= ((int64_t)1 << 31))
            return fail(MGPCG_ERR_DIMS, "problem too large for 32-bit row indices");

        // permutation natural packed -> internal
        std::vector<int32_t> perm(Lv.n), iperm(Lv.n);
        std::vector<int64_t> natoff(G + 1);
        for (int g = 0; g < G; ++g) {
            const LevelGrid &lg = Lv.grids[g];
            natoff[g] = lg.nat_off;
            Colouring C(lg.nx, lg.ny, lg.nz, P->colour_order);
            for (int iz = 0; iz < lg.nz; ++iz)
                for (int iy = 0; iy < lg.ny; ++iy)
                    for (int ix = 0; ix < lg.nx; ++ix) {
                        int bx = ix & 1, by = iy & 1, bz = iz & 1;
                        int k = C.colour(bx, by, bz);
                        int64_t hx = half_count(lg.nx, bx), hy = half_count(lg.ny, by);
                        int64_t j = (ix >> 1) + hx * ((iy >> 1) + hy * (iz >> 1));
                        int64_t q = lg.nat_off + ix + (int64_t)lg.nx * (iy + (int64_t)lg.ny * iz);
                        int64_t in = lg.seg_off[k] + j;
                        perm[q] = (int32_t)in;
                        iperm[in] = (int32_t)q;
                    }
        }
        natoff[G] = Lv.n;
        ST_TRY(upload(&Lv.perm, perm, s));
        ST_TRY(upload(&Lv.iperm, iperm, s));
        ST_TRY(upload(&P->d_natoff[l], natoff, s));
        if (l == 0) ST_TRY(upload(&P->d_natoff0, natoff, s));
        if (P->smoother == MGPCG_SMOOTHER_SEQUENTIAL) {
            if (l == 0)
                if (const char *env = getenv("MGPCG_LEX_RUN_ROWS"))  // test override, 0..512
                    P->lex_run_rows = std::min(512, std::max(0, atoi(env)));
            ST_TRY(build_waves(P, l, perm, iperm, s));
        }

        // column bases for the compact column formats, per grid and colour:
        // base[g][k][s] = column - row of the first row of colour k of grid g
        // that has a neighbour in slot s
        if (P->col_format >= 1) {
            std::vector<int32_t> base((size_t)G * 8 * kW, 0);
            for (int g = 0; g < G; ++g) {
                const LevelGrid &lg = Lv.grids[g];
                const int64_t no = natoff[g];
                for (int k = 0; k < Lv.ncol; ++k) {
                    int missing = kW;
                    std::vector<char> have(kW, 0);
                    for (int64_t i = lg.seg_off[k]; i < lg.seg_off[k] + lg.seg_len[k] && missing > 0; ++i) {
                        const int64_t q = iperm[i] - no;
                        const int ix = (int)(q % lg.nx), iy = (int)((q / lg.nx) % lg.ny),
                                  iz = (int)(q / ((int64_t)lg.nx * lg.ny));
                        for (int sl = 0; sl < kW; ++sl) {
                            if (have[sl]) continue;
                            const int jx = ix + sl % 3 - 1, jy = iy + (sl / 3) % 3 - 1, jz = iz + sl / 9 - 1;
                            if (jx < 0 || jx >= lg.nx || jy < 0 || jy >= lg.ny || jz < 0 || jz >= lg.nz) continue;
                            base[((size_t)g * 8 + k) * kW + sl] =
                                (int32_t)(perm[no + jx + (int64_t)lg.nx * (jy + (int64_t)lg.ny * jz)] - i);
                            have[sl] = 1;
                            --missing;
                        }
                    }
                }
            }
            ST_TRY(upload(&Lv.dbase, base, s));
            Lv.dbase_host = base;
            if (G > 1) {
                // grid of each internal row, for the kernels that index rows directly
                std::vector<int32_t> grow(Lv.n);
                for (int g = 0; g < G; ++g)
                    for (int k = 0; k < Lv.ncol; ++k)
                        for (int64_t i = 0; i < Lv.grids[g].seg_len[k]; ++i) grow[Lv.grids[g].seg_off[k] + i] = g;
                ST_TRY(upload(&Lv.grid_of_row, grow, s));
            }
        }

        const int64_t opbytes = Lv.n * kW * ((P->mg_dtype == MGPCG_FP32 && l > 0 ? 4 : 8) + 4);
        int64_t nt_bytes = (int64_t)128 << 20;  // operators above half the Infinity Cache are streamed
        if (const char *env = getenv("MGPCG_NT_BYTES")) nt_bytes = atoll(env);  // tuning override
        Lv.stream_nt = opbytes > nt_bytes;
        // colour-pass tables, for both workgroup sizes: one workgroup per
        // pass_rows rows, grid-homogeneous
        for (int v = 0; v < 2; ++v) {
            std::vector<Seg> tab;
            std::vector<int> &first = Lv.pass_first_v[v];
            first.assign(Lv.ncol + 1, 0);
            const int rows_per_block = pass_rows(v == 1, R);
            for (int k = 0; k < Lv.ncol; ++k) {
                first[k] = (int)tab.size();
                for (int g = 0; g < G; ++g) {
                    const LevelGrid &lg = Lv.grids[g];
                    for (int64_t a = 0; a < lg.seg_len[k]; a += rows_per_block) {
                        Seg e;
                        e.row0 = lg.seg_off[k] + a;
                        e.count = (int32_t)std::min<int64_t>(rows_per_block, lg.seg_len[k] - a);
                        e.grid = (int16_t)g;
                        e.colour = (int16_t)k;
                        tab.push_back(e);
                    }
                }
            }
            first[Lv.ncol] = (int)tab.size();
            ST_TRY(upload(&Lv.pass_tab_v[v], tab, s));
        }
        Lv.pass_tab = Lv.pass_tab_v[Lv.stream_nt];
        Lv.pass_first = Lv.pass_first_v[Lv.stream_nt];

        // zero-start forward pass: a colour-k row must skip every slot whose
        // real neighbour has colour >= k (not written yet in this sweep), and
        // may skip padding slots.  One mask per colour serves all grids, so
        // it is the intersection of what each grid allows; if some grid needs
        // a slot skipped that another grid must read, the level falls back to
        // clearing z and a general first pass.
        Lv.zs_ok = true;
        for (int k = 0; k < 8; ++k) {
            uint32_t allowed = ~0u, needed = 0;
            for (int g = 0; g < G; ++g) {
                const LevelGrid &lg = Lv.grids[g];
                if (k >= lg.ncol || lg.seg_len[k] == 0) continue;
                Colouring C(lg.nx, lg.ny, lg.nz, P->colour_order);
                int b[3];
                C.parity(k, b);
                int ext[3] = {lg.nx, lg.ny, lg.nz};
                for (int sl = 0; sl < kW; ++sl) {
                    int d[3] = {sl % 3 - 1, (sl / 3) % 3 - 1, sl / 9 - 1};
                    bool padding = false;
                    for (int a = 0; a < 3; ++a)
                        if (d[a] != 0 && ext[a] < 2) padding = true;
                    if (padding) continue;
                    int nb = C.colour(b[0] ^ (d[0] & 1), b[1] ^ (d[1] & 1), b[2] ^ (d[2] & 1));
                    if (nb >= k) needed |= 1u << sl;
                    else allowed &= ~(1u << sl);
                }
            }
            Lv.zi_skip[k] = allowed & ((1u << kW) - 1);
            if ((needed & ~allowed) != 0) Lv.zs_ok = false;
        }
        // the kernels carry the masks of the standard 8-colour numbering as
        // compile-time constants; any other level clears z and sweeps
        Lv.zs_std = Lv.zs_ok && Lv.ncol == 8;
        for (int k = 0; k < Lv.ncol && Lv.zs_std; ++k)
            if (Lv.zi_skip[k] != standard_zs_mask(k, P->colour_order)) Lv.zs_std = false;
        if (G > 1) {
            std::vector<int32_t> gon(Lv.n);
            for (int g = 0; g < G; ++g)
                for (int64_t q = natoff[g]; q < natoff[g + 1]; ++q) gon[q] = g;
            ST_TRY(upload(&Lv.grid_of_nat, gon, s));
        }
    }

    // injection maps (fine level l -> coarse level l+1), sorted by fine row
    for (int l = 0; l + 1 < L; ++l) {
        Level &F = P->lev[l];
        Level &Cc = P->lev[l + 1];
        std::vector<int32_t> hperm_f(F.n), hperm_c(Cc.n);
        HIP_TRY(hipMemcpyAsync(hperm_f.data(), F.perm, F.n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hperm_c.data(), Cc.perm, Cc.n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        std::vector<std::pair<int32_t, int32_t>> pairs;
        pairs.reserve(Cc.n);
        for (int g = 0; g < G; ++g) {
            const LevelGrid &fg = F.grids[g], &cg = Cc.grids[g];
            for (int jz = 0; jz < cg.nz; ++jz)
                for (int jy = 0; jy < cg.ny; ++jy)
                    for (int jx = 0; jx < cg.nx; ++jx) {
                        int64_t qc = cg.nat_off + jx + (int64_t)cg.nx * (jy + (int64_t)cg.ny * jz);
                        int64_t qf = fg.nat_off + 2 * jx + (int64_t)fg.nx * (2 * jy + (int64_t)fg.ny * 2 * jz);
                        pairs.emplace_back(hperm_f[qf], hperm_c[qc]);
                    }
        }
        std::sort(pairs.begin(), pairs.end());
        std::vector<int32_t> fi(pairs.size()), ci(pairs.size());
        for (size_t t = 0; t < pairs.size(); ++t) {
            fi[t] = pairs[t].first;
            ci[t] = pairs[t].second;
        }
        F.n_inj = (int64_t)pairs.size();
        // colour 0 is exactly the injection set, in injection order, and it is
        // the colour swept last by the backward pass and first by the forward
        // pass: the restriction and the refinement can ride on those passes
        F.fuse_transfers = F.ncol > 0 && F.coff[0] == 0 && F.coff[1] == F.n_inj;
        for (size_t t = 0; t < fi.size() && F.fuse_transfers; ++t)
            if (fi[t] != (int32_t)t) F.fuse_transfers = false;
        ST_TRY(upload(&F.inj_fine, fi, s));
        ST_TRY(upload(&F.inj_coarse, ci, s));
    }

    // operators, workspaces
    const bool fp32 = P->mg_dtype == MGPCG_FP32;
    for (int l = 0; l < L; ++l) {
        Level &Lv = P->lev[l];
        if (l == 0 || !fp32) ST_TRY(dalloc(&Lv.val64, ell_size(Lv.n)));
        if (fp32) ST_TRY(dalloc(&Lv.val32, ell_size(Lv.n)));
        ST_TRY(dalloc(&Lv.col, ell_size(Lv.n)));
        if (fp32) {
            float *r32, *z32;
            ST_TRY(dalloc(&r32, Lv.n * R));
            ST_TRY(dalloc(&z32, Lv.n * R));
            Lv.r = r32;
            Lv.z = z32;
        } else if (l > 0) {
            double *r64, *z64;
            ST_TRY(dalloc(&r64, Lv.n * R));
            ST_TRY(dalloc(&z64, Lv.n * R));
            Lv.r = r64;
            Lv.z = z64;
        }
        HIP_TRY(launch_build_ell(P, l, theta, s));
        if (P->smoother == MGPCG_SMOOTHER_SEQUENTIAL) {
            ST_TRY(dalloc(&Lv.wval, ell_size(Lv.npos)));
            HIP_TRY(launch_wave_gather(P, l, s));
        }
        Lv.cf = 0;
        if (Lv.dbase) {
            // try the compact column formats: implied columns if every delta
            // is zero, int8 deltas if every delta fits, else int32 columns
            ST_TRY(dalloc(&Lv.dcol, delta_bytes(Lv.n)));
            int64_t *coff_dev = nullptr;
            int *flags = nullptr;
            std::vector<int64_t> coffv(Lv.coff.begin(), Lv.coff.end());
            ST_TRY(upload(&coff_dev, coffv, s));
            ST_TRY(dalloc(&flags, 2));
            HIP_TRY(launch_fill_i(flags, 2, 0, s));
            HIP_TRY(launch_delta_encode(P, l, coff_dev, flags, s));
            int hflags[2] = {1, 1};
            HIP_TRY(hipMemcpyAsync(hflags, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            dfree(coff_dev);
            dfree(flags);
            if (hflags[0]) {
                dfree(Lv.dcol);
                dfree(Lv.dbase);
            } else {
                dfree(Lv.col);
                Lv.cf = 1;
                if (!hflags[1] && P->col_format >= 2) {
                    dfree(Lv.dcol);
                    Lv.cf = 2;
                }
            }
        }
    }

    // level-0 reduction tables: grid by grid, chunks of kBlock/R rows (one
    // row per R threads) and of kVecRows*kBlock/R rows.  The workgroups of the
    // one-row table gather from all colours, so its chunks are ordered slab
    // by slab (the j-th slab of every colour, then the next): the contiguous
    // block range an XCD receives is then a run of spatial slabs, whose
    // gathers stay near that XCD, instead of one colour that needs
    // neighbours from the whole grid.  With one rhs a slab is an eighth of the
    // grid, whose 8-byte vector slice fits an XCD's L2.  With R > 1 an entry
    // holds only kBlock/R rows and a point carries 8R bytes, so the rows an
    // XCD has in flight must be a compact region for their gathers to fit
    // its 4 MB L2: a workgroup takes spc = 2 consecutive entries, and the
    // entries run half-plane by half-plane (hz), within one by blocks of 8
    // half-lines (hy), every colour of a block in turn.  At 16 right-hand
    // sides on 128^3 this took the product's HBM reads from 2.26 GB to
    // 1.00 GB (about its 0.99 GB of operator, p and q), with 2 x 16 rows
    // per workgroup instead of 16 x 16 (a z-plane of every colour in turn
    // read 2.26 GB).  Every grid is padded with empty entries to a multiple
    // of spc, so that a workgroup stays within one grid.
    {
        const Level &L0 = P->lev[0];
        int64_t max_blocks = 0;
        P->spc = R == 1 ? 1 : 2;
        for (int t = 0; t < 2; ++t) {
            std::vector<Seg> tab;
            std::vector<int> gb(G + 1, 0);
            // table 0: one row per pass_lanes(R) threads (two right-hand
            // sides per lane from kPairR on, as in the colour passes)
            const int rows = t == 0 ? kBlock / pass_lanes(R) : kVecRows * kBlock / R;
            const int per = t == 0 ? P->spc : 1;  // entries per workgroup
            if (t == 1 && G == 1) {
                // one grid: the vector kernels take contiguous chunks of the
                // whole vector and compute them from the block index
                gb[0] = 0;
                for (int64_t a = 0; a < L0.n; a += rows) {
                    Seg e;
                    e.row0 = a;
                    e.count = (int32_t)std::min<int64_t>(rows, L0.n - a);
                    e.grid = 0;
                    e.colour = 0;
                    tab.push_back(e);
                }
            }
            for (int g = 0; g < G && !(t == 1 && G == 1); ++g) {
                gb[g] = (int)(tab.size() / per);
                const LevelGrid &lg = L0.grids[g];
                if (t == 0 && R > 1) {
                    // half-plane by half-plane; within one, blocks of kYBlock
                    // half-lines, every colour of a block in turn
                    constexpr int64_t kYBlock = 8;
                    Colouring C(lg.nx, lg.ny, lg.nz, P->colour_order);
                    int64_t hx[8] = {}, hy[8] = {}, hz[8] = {};
                    int64_t hzmax = 0, hymax = 0;
                    for (int k = 0; k < lg.ncol; ++k) {
                        int b[3];
                        C.parity(k, b);
                        hx[k] = half_count(lg.nx, b[0]);
                        hy[k] = half_count(lg.ny, b[1]);
                        hz[k] = half_count(lg.nz, b[2]);
                        hzmax = std::max(hzmax, hz[k]);
                        hymax = std::max(hymax, hy[k]);
                    }
                    for (int64_t jz = 0; jz < hzmax; ++jz)
                        for (int64_t y0 = 0; y0 < hymax; y0 += kYBlock)
                            for (int k = 0; k < lg.ncol; ++k) {
                                if (jz >= hz[k] || y0 >= hy[k]) continue;
                                const int64_t y1 = std::min<int64_t>(y0 + kYBlock, hy[k]);
                                const int64_t a0 = lg.seg_off[k] + (jz * hy[k] + y0) * hx[k];
                                const int64_t a1 = lg.seg_off[k] + (jz * hy[k] + y1) * hx[k];
                                for (int64_t a = a0; a < a1; a += rows) {
                                    Seg e;
                                    e.row0 = a;
                                    e.count = (int32_t)std::min<int64_t>(rows, a1 - a);
                                    e.grid = (int16_t)g;
                                    e.colour = (int16_t)k;
                                    tab.push_back(e);
                                }
                            }
                }
                const int slabs = t == 1 ? 1 : R == 1 ? 8 : 0;
                for (int j = 0; j < slabs; ++j)
                    for (int k = 0; k < L0.ncol; ++k) {
                        const int64_t nch = (lg.seg_len[k] + rows - 1) / rows;
                        for (int64_t c = nch * j / slabs; c < nch * (j + 1) / slabs; ++c) {
                            const int64_t a = c * rows;
                            Seg e;
                            e.row0 = lg.seg_off[k] + a;
                            e.count = (int32_t)std::min<int64_t>(rows, lg.seg_len[k] - a);
                            e.grid = (int16_t)g;
                            e.colour = (int16_t)k;
                            tab.push_back(e);
                        }
                    }
                while (tab.size() % per) {
                    Seg e;  // padding: no rows
                    e.row0 = lg.seg_off[0];
                    e.count = 0;
                    e.grid = (int16_t)g;
                    e.colour = 0;
                    tab.push_back(e);
                }
            }
            gb[G] = (int)(tab.size() / per);
            P->n_red[t] = (int)(tab.size() / per);
            max_blocks = std::max<int64_t>(max_blocks, (int64_t)P->n_red[t]);
            ST_TRY(upload(&P->red_tab[t], tab, s));
            ST_TRY(upload(&P->red_gb[t], gb, s));
        }
        // <r,z> fused into the level-0 post-smoother: one grid (several
        // would need per-grid partial ranges; with R > 1 the fold kernel
        // pre-sums the partials), FP64 V-cycle (whose level-0 z is the CG
        // z), the standard sweep with the double pass (the last update of
        // colour c-1 is that pass)
        P->fuse_rz = G == 1 && P->mg_dtype == MGPCG_FP64 && L0.ncol == 8 &&
                     P->smoother == MGPCG_SMOOTHER_COLOURED;
        if (P->fuse_rz) {
            // the partials buffer serves either level-0 workgroup size
            for (int v = 0; v < 2; ++v) {
                int64_t off[9];
                rz_layout(P, v == 1, off);
                max_blocks = std::max<int64_t>(max_blocks, off[8]);
            }
            ST_TRY(dalloc(&P->red_gb[2], 2));
            HIP_TRY(set_rz_layout(P, s));
        }
        // box-tiled product (k_spmv_box): one grid of even extents, two
        // right-hand sides per lane; one workgroup per box of box_run(R)
        // half-points in x at one (Y, Z), i.e. 8 * box_run(R) rows
        {
            const int nx = P->dims0[0], ny = P->dims0[1], nz = P->dims0[2];
            const int bx = R >= kPairR ? box_run(R) : 1;
            P->box_ok = G == 1 && R >= kPairR && L0.ncol == 8 && nx % (2 * bx) == 0 && ny % 2 == 0 && nz % 2 == 0;
            if (P->box_ok) {
                mg::BoxGeo &bg = P->box;
                bg.nx = nx;
                bg.ny = ny;
                bg.nz = nz;
                bg.hx = nx / 2;
                bg.hy = ny / 2;
                bg.nxb = nx / (2 * bx);
                bg.nh = (int32_t)(L0.n / 8);
                bg.flip = P->colour_order ? 7 : 0;
                Colouring C(nx, ny, nz, P->colour_order);
                for (int pc = 0; pc < 8; ++pc)
                    if (L0.coff[C.colour(pc & 1, (pc >> 1) & 1, pc >> 2)] != (int64_t)(pc ^ bg.flip) * bg.nh)
                        return fail(MGPCG_ERR_DIMS, "internal: box geometry does not match the colour ranges");
                P->n_box = (int)(L0.n / (8 * bx));
                max_blocks = std::max<int64_t>(max_blocks, P->n_box);
            }
        }
        const int64_t n0 = L0.n * R;
        ST_TRY(dalloc(&P->x, n0));
        ST_TRY(dalloc(&P->r, n0));
        ST_TRY(dalloc(&P->z, n0));
        ST_TRY(dalloc(&P->p, n0));
        ST_TRY(dalloc(&P->q, n0));
        ST_TRY(dalloc(&P->b, n0));
        const int S = P->S;
        Scalars &sc = P->sc;
        ST_TRY(dalloc(&sc.rho, S));
        ST_TRY(dalloc(&sc.rho_old, S));
        ST_TRY(dalloc(&sc.alpha, S));
        ST_TRY(dalloc(&sc.beta, S));
        ST_TRY(dalloc(&sc.nr0, S));
        ST_TRY(dalloc(&sc.pq, S));
        ST_TRY(dalloc(&sc.apend, S));
        ST_TRY(dalloc(&sc.iter, S));
        ST_TRY(dalloc(&sc.done, S));
        ST_TRY(dalloc(&sc.status, S));
        ST_TRY(dalloc(&sc.ndone, 1));
        ST_TRY(dalloc(&sc.partials, max_blocks * R));
        if (G == 1 && R > 1) {
            ST_TRY(dalloc(&P->fold, (int64_t)kFoldBlocks * R));
        }
    }
    // persistent coarse-level V-cycle (levels 1..L-1 in one launch) and the
    // single-workgroup tail (the smallest levels): one right-hand side,
    // standard 8-colour zero-start masks, one column format
    {
        const bool fp32 = P->mg_dtype == MGPCG_FP32;
        auto eligible = [&](int from) {
            bool ok = from >= 1 && from < L && R == 1 && P->sweeps == 1;
            for (int l = from; l < L && ok; ++l) ok = P->lev[l].zs_std && P->lev[l].ncol == 8;
            const int cf = ok ? P->lev[from].cf : 0;
            for (int l = from; l < L && ok; ++l) ok = P->lev[l].cf == cf;
            // its phases index rows directly: compact columns only for one grid
            if (G > 1 && cf != 0) ok = false;
            return ok;
        };
        // the phase program of the V-cycle of Listing 1 from level `from` down
        auto program = [&](int from, CoarseArgs &A) -> bool {
            std::vector<uint16_t> prog;
            auto ph = [&](int l, int k, int op) { prog.push_back((uint16_t)(l | (k << 4) | (op << 8))); };
            for (int l = from; l < L; ++l) {
                const bool coarser = l + 1 < L;
                const bool fuse = coarser && P->lev[l].fuse_transfers;
                for (int k = 0; k < 7; ++k) ph(l, k, kOpZeroStart);
                ph(l, 7, kOpTwiceZeroStart);
                for (int k = 6; k >= 1; --k) ph(l, k, kOpPlain);
                ph(l, 0, fuse ? kOpFusedRestrict : kOpPlain);
                if (coarser && !fuse) ph(l, 0, kOpRestrict);
            }
            for (int l = L - 2; l >= from; --l) {
                const bool fuse = P->lev[l].fuse_transfers;
                if (!fuse) ph(l, 0, kOpProlong);
                ph(l, 0, fuse ? kOpFusedProlong : kOpPlain);
                for (int k = 1; k < 7; ++k) ph(l, k, kOpPlain);
                ph(l, 7, kOpTwice);
                for (int k = 6; k >= 0; --k) ph(l, k, kOpPlain);
            }
            if ((int)prog.size() > kMaxPhases) return false;
            memset(&A, 0, sizeof(A));
            A.cf = P->lev[from].cf;
            for (int l = from; l < L; ++l) {
                const Level &Lv = P->lev[l];
                CoarseLevel &cl = A.lev[l];
                cl.n = Lv.n;
                cl.val = fp32 ? (const void *)Lv.val32 : (const void *)Lv.val64;
                cl.col = Lv.col;
                cl.dcol = Lv.dcol;
                cl.dbase = Lv.dbase;
                cl.r = Lv.r;
                cl.z = Lv.z;
                cl.inj_fine = Lv.inj_fine;
                cl.inj_coarse = Lv.inj_coarse;
                cl.n_inj = Lv.n_inj;
                for (int k = 0; k <= 8; ++k) cl.coff[k] = Lv.coff[std::min(k, Lv.ncol)];
            }
            A.nphases = (int)prog.size();
            for (size_t t = 0; t < prog.size(); ++t) A.phase[t] = prog[t];
            return true;
        };
        auto max_colour_rows = [&](int l) {
            int64_t m = 0;
            for (int k = 0; k < P->lev[l].ncol; ++k) m = std::max<int64_t>(m, P->lev[l].coff[k + 1] - P->lev[l].coff[k]);
            return m;
        };

        const int lc = 1;
        bool ok = eligible(lc);
        int ncu = 0;
        if (ok && hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess) ok = false;
        const int occ = ok ? coarse_vcycle_occupancy(R, fp32, P->lev[lc].cf, P->colour_order) : 0;
        if (ok && occ < 1) ok = false;
        if (ok) ok = program(lc, P->coarse_args);
        if (ok) {
            const int64_t want = (max_colour_rows(lc) + kBlock / R - 1) / (kBlock / R);
            int B = (int)std::max<int64_t>(1, std::min<int64_t>(want, ncu));
            if (const char *env = getenv("MGPCG_COARSE_BLOCKS")) {  // tuning override
                const int bb = atoi(env);
                if (bb >= 1 && bb <= ncu) B = bb;
            }
            P->coarse_lc = lc;
            P->coarse_blocks = B;
            CoarseArgs &A = P->coarse_args;
            ST_TRY(dalloc(&P->coarse_flags, (int64_t)B + 1));
            ST_TRY(dalloc(&P->coarse_err, 1));
            A.flags = P->coarse_flags;
            A.epoch_base = P->coarse_flags + B;
            A.err = P->coarse_err;
            A.spin_limit = 1ll << 21;
            HIP_TRY(launch_fill_u(P->coarse_flags, (int64_t)B + 1, 0u, s));
            HIP_TRY(launch_fill_i(P->coarse_err, 1, 0, s));
        }
        P->coarse_ok = ok;

        // tail: the coarsest level, when its r and z fit in one workgroup's
        // LDS and it has the standard 8-colour numbering
        int64_t tail_bytes = 64 << 10;
        if (const char *env = getenv("MGPCG_TAIL_BYTES")) tail_bytes = atoll(env);  // tuning override
        const Level &Lt = P->lev[L - 1];
        const int64_t need = Lt.n * 2 * (fp32 ? 4 : 8);
        int64_t widest = 0;
        for (int k = 0; k < Lt.ncol; ++k) widest = std::max<int64_t>(widest, Lt.coff[k + 1] - Lt.coff[k]);
        P->tail_ok = L >= 2 && R == 1 && P->sweeps == 1 && Lt.zs_std && Lt.ncol == 8 && need <= tail_bytes &&
                     need <= (64 << 10) && widest <= kTailBlock && (G == 1 || Lt.cf == 0);
        P->tail_lw = P->tail_ok ? L - 1 : L;
        // default: the tail only while its colours fill at most half the
        // workgroup (measured: at 128^3, 512 rows per colour, the 15 pass
        // kernels are 5 us per CG iteration faster; at 96^3, 216 rows, the
        // tail is 2 us faster); the schedule can choose either
        P->tail_on = widest <= kTailBlock / 2 ? 1 : 0;
    }
    HIP_TRY(hipHostMalloc((void **)&P->pinned_ndone, sizeof(int) * mgpcg_problem::kCheckRing, hipHostMallocDefault));
    for (int j = 0; j < mgpcg_problem::kCheckRing; ++j)
        HIP_TRY(hipEventCreateWithFlags(&P->check_ev[j], hipEventDisableTiming));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    return MGPCG_OK;
}

void free_problem(mgpcg_problem *P) {
    if (!P) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(P->device);
    (void)hipDeviceSynchronize();
    for (auto &Lv : P->lev) {
        dfree(Lv.val64); dfree(Lv.val32); dfree(Lv.col); dfree(Lv.dcol); dfree(Lv.dbase); dfree(Lv.perm);
        dfree(Lv.grid_of_row);
        dfree(Lv.iperm);
        dfree(Lv.grid_of_nat); dfree(Lv.pass_tab_v[0]); dfree(Lv.pass_tab_v[1]); dfree(Lv.inj_fine);
        dfree(Lv.inj_coarse);
        Lv.pass_tab = nullptr;
        dfree(Lv.r); dfree(Lv.z); dfree(Lv.t0); dfree(Lv.t1); dfree(Lv.t2);
        dfree(Lv.woff_dev); dfree(Lv.wrow); dfree(Lv.wcol); dfree(Lv.wval);
    }
    for (auto &p : P->d_natoff) dfree(p);
    dfree(P->d_dims0); dfree(P->d_natoff0);
    for (int t = 0; t < 2; ++t) { dfree(P->red_tab[t]); dfree(P->red_gb[t]); }
    dfree(P->red_gb[2]);
    dfree(P->x); dfree(P->r); dfree(P->z); dfree(P->p); dfree(P->q); dfree(P->b);
    Scalars &sc = P->sc;
    dfree(sc.rho); dfree(sc.rho_old); dfree(sc.alpha); dfree(sc.beta); dfree(sc.nr0); dfree(sc.pq); dfree(sc.apend);
    dfree(sc.iter); dfree(sc.done); dfree(sc.status); dfree(sc.ndone);
    dfree(sc.partials);
    dfree(P->fold);
    dfree(P->hist);
    dfree(P->coarse_flags);
    dfree(P->coarse_err);
    if (P->pinned_ndone) (void)hipHostFree(P->pinned_ndone);
    for (auto &ev : P->check_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (P->iter_graph) (void)hipGraphExecDestroy(P->iter_graph);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    (void)hipSetDevice(cur);
    delete P;
}

// ----------------------------------------------------------------- drivers

// one symmetric sweep: colours 0..c-1 then c-1..0.  first_mode applies to
// the first forward pass, last_mode to the last backward pass.
template <typename T>
hipError_t sweep(const mgpcg_problem *P, int l, const T *val, const T *r, T *z, int first_mode,
                 int last_mode, T *coarse, const int *done, hipStream_t s, double *rzp = nullptr) {
    const Level &Lv = P->lev[l];
    const int c = Lv.ncol;
    hipError_t e;
    // The last forward pass and the first backward pass update the same colour
    // c-1 back to back with unchanged neighbours: one kernel applies both
    // updates (same arithmetic, one read of the rows).
    const bool zs = first_mode == kPassZeroStart;
    const bool twice = c >= 2 && (!zs || (Lv.zs_std && c == 8 && (P->R == 1 || P->R == 16)));
    // a zero start also folds the trivial first pass into the second
    const bool zs01 = zs && twice && c == 8;
    for (int k = 0; k < c; ++k) {
        int mode = k == 0 ? first_mode : (zs ? kPassZeroStart : kPassPlain);
        if (k == c - 1 && twice) mode = zs ? kPassTwiceZeroStart : kPassTwice;
        if (zs01 && k == 0) mode = kPassZeroStart01;
        if (zs01 && k == 1) continue;
        // rzp: the last update of each colour also writes <r,z> partials
        double *kp = rzp && k == c - 1 && twice ? rzp + P->rz_off[k] * P->R : nullptr;
        if ((e = launch_pass<T>(P, l, k, mode, val, r, z, done, coarse, s, kp)) != hipSuccess) return e;
    }
    for (int k = (twice ? c - 2 : c - 1); k >= 0; --k) {
        const int mode = k == 0 ? last_mode : kPassPlain;
        double *kp = rzp ? rzp + P->rz_off[k] * P->R : nullptr;
        if ((e = launch_pass<T>(P, l, k, mode, val, r, z, done, coarse, s, kp)) != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
const T *level_val(const mgpcg_problem *P, int l);
template <>
const double *level_val<double>(const mgpcg_problem *P, int l) { return P->lev[l].val64; }
template <>
const float *level_val<float>(const mgpcg_problem *P, int l) { return P->lev[l].val32; }

// Listing 1: z0 = MG(0, r0); every level starts from z = 0.  With the
// persistent coarse kernel, levels coarse_lc..L-1 run in one launch between
// the level-0 pre- and post-smoothers.
template <typename T>
hipError_t vcycle(const mgpcg_problem *P, const T *r0, T *z0, const int *done, hipStream_t s,
                  double *rzp = nullptr) {
    const bool persistent = P->coarse_ok && P->coarse_mode == 1;
    const bool tail = !persistent && P->tail_ok && P->tail_on;
    // levels below L run one kernel per pass; the rest in one launch
    const int L = persistent ? P->coarse_lc : (tail ? P->tail_lw : P->L);
    auto rl = [&](int l) -> T * { return l == 0 ? const_cast<T *>(r0) : (T *)P->lev[l].r; };
    auto zl = [&](int l) -> T * { return l == 0 ? z0 : (T *)P->lev[l].z; };
    hipError_t e;
    for (int l = 0; l < L; ++l) {
        const Level &Lv = P->lev[l];
        const bool zs = Lv.zs_std && (P->R == 1 || P->R == 16);
        if (!zs) {
            hipError_t fe = sizeof(T) == 8 ? launch_fill_d((double *)zl(l), Lv.n * P->R, 0.0, s)
                                           : launch_fill_u((unsigned *)zl(l), Lv.n * P->R, 0u, s);
            if (fe != hipSuccess) return fe;
        }
        const bool coarser = l + 1 < P->L;
        const bool fuse = coarser && Lv.fuse_transfers;
        // pre-smoothing: P->sweeps symmetric sweeps; the first may start from
        // zero, the last may carry the restriction
        for (int k = 0; k < P->sweeps; ++k)
            if ((e = sweep<T>(P, l, level_val<T>(P, l), rl(l), zl(l), zs && k == 0 ? kPassZeroStart : kPassPlain,
                              fuse && k == P->sweeps - 1 ? kPassRestrict : kPassPlain,
                              coarser ? rl(l + 1) : nullptr, done, s)) != hipSuccess)
                return e;
        if (coarser && !fuse &&
            (e = launch_restrict<T>(P, l, level_val<T>(P, l), rl(l), zl(l), rl(l + 1), s)) != hipSuccess)
            return e;
    }
    if (persistent && (e = launch_coarse_vcycle(P, sizeof(T) == 4, s)) != hipSuccess) return e;
    if (tail && (e = launch_coarse_tail(P, sizeof(T) == 4, s)) != hipSuccess) return e;
    for (int l = (persistent || tail ? L - 1 : L - 2); l >= 0; --l) {
        const bool fuse = P->lev[l].fuse_transfers;
        if (!fuse && (e = launch_prolong<T>(P, l, zl(l + 1), zl(l), s)) != hipSuccess) return e;
        // post-smoothing: the first sweep may carry the refinement, the last
        // writes the <r,z> partials
        for (int k = 0; k < P->sweeps; ++k)
            if ((e = sweep<T>(P, l, level_val<T>(P, l), rl(l), zl(l), fuse && k == 0 ? kPassProlong : kPassPlain,
                              kPassPlain, zl(l + 1), done, s,
                              l == 0 && k == P->sweeps - 1 ? rzp : nullptr)) != hipSuccess)
                return e;
    }
    return hipSuccess;
}

// Listing 1 with the sequential smoother (FP64, one right-hand side): every
// level starts from z = 0, each smoothing step is P->sweeps symmetric sweeps,
// the restriction and refinement run as their own kernels.
hipError_t vcycle_lex(const mgpcg_problem *P, const double *r0, double *z0, hipStream_t s) {
    auto rl = [&](int l) -> double * { return l == 0 ? const_cast<double *>(r0) : (double *)P->lev[l].r; };
    auto zl = [&](int l) -> double * { return l == 0 ? z0 : (double *)P->lev[l].z; };
    hipError_t e;
    for (int l = 0; l < P->L; ++l) {
        const Level &Lv = P->lev[l];
        if ((e = launch_fill_d(zl(l), Lv.n, 0.0, s)) != hipSuccess) return e;
        for (int k = 0; k < P->sweeps; ++k)
            if ((e = launch_lex_sweep(P, l, rl(l), zl(l), s)) != hipSuccess) return e;
        if (l + 1 < P->L && (e = launch_restrict<double>(P, l, Lv.val64, rl(l), zl(l), rl(l + 1), s)) != hipSuccess)
            return e;
    }
    for (int l = P->L - 2; l >= 0; --l) {
        if ((e = launch_prolong<double>(P, l, zl(l + 1), zl(l), s)) != hipSuccess) return e;
        for (int k = 0; k < P->sweeps; ++k)
            if ((e = launch_lex_sweep(P, l, rl(l), zl(l), s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// z = M^{-1} r on the CG vectors (FP64, internal layout)
// fused (FP32 V-cycle inside the CG iteration): the level-0 FP32 r was
// already stored by the previous residual update (or after the initial
// residual), and z is left in the level-0 FP32 workspace for a kernel that
// widens it and forms <r, z> in the same pass
hipError_t precondition(const mgpcg_problem *P, const double *r, double *z, const int *done, hipStream_t s,
                        double *rzp = nullptr, bool fused = false) {
    if (P->smoother == MGPCG_SMOOTHER_SEQUENTIAL) return vcycle_lex(P, r, z, s);
    if (P->mg_dtype == MGPCG_FP64) return vcycle<double>(P, r, z, done, s, rzp);
    const Level &L0 = P->lev[0];
    hipError_t e;
    const int64_t n = L0.n * P->R;
    if (!fused && (e = launch_cast_d2f(r, (float *)L0.r, n, s)) != hipSuccess) return e;
    if ((e = vcycle<float>(P, (const float *)L0.r, (float *)L0.z, done, s)) != hipSuccess) return e;
    return fused ? hipSuccess : launch_cast_f2d((const float *)L0.z, z, n, s);
}

// the FP32 V-cycle's right-hand side and correction are narrowed and widened
// inside the CG kernels (not for the sequential smoother, which is FP64)
static bool fused_fp32(const mgpcg_problem *P) {
    return P->mg_dtype == MGPCG_FP32 && P->smoother != MGPCG_SMOOTHER_SEQUENTIAL;
}

hipError_t cg_iteration(mgpcg_problem *P, double tol, hipStream_t s) {
    hipError_t e;
    // rho = <r, z>: accumulated by the level-0 post-smoother when fuse_rz;
    // with the FP32 V-cycle, formed while its z is widened
    const bool f32 = fused_fp32(P);
    if ((e = precondition(P, P->r, P->z, P->sc.done, s, P->fuse_rz ? P->sc.partials : nullptr, f32)) !=
        hipSuccess)
        return e;
    if ((e = P->fuse_rz ? launch_finalize_rz(P, s) : f32 ? launch_cast_dot_rz(P, s) : launch_dot_rz(P, s)) !=
        hipSuccess)
        return e;
    if ((e = launch_update_p(P, s)) != hipSuccess) return e;
    if ((e = launch_spmv_pq(P, s)) != hipSuccess) return e;
    return launch_update_r(P, tol, P->hist_cap, s, f32 ? (float *)P->lev[0].r : nullptr);
}

// ------------------------------------------------------- argument helpers

mgpcg_status check_problem(const mgpcg_problem *P) {
    if (!P) return fail(MGPCG_ERR_INVALID_ARG, "problem handle is NULL");
    return MGPCG_OK;
}
mgpcg_status check_level(const mgpcg_problem *P, int level, bool need_coarser = false) {
    ST_TRY(check_problem(P));
    if (level < 0 || level >= P->L || (need_coarser && level + 1 >= P->L))
        return fail(MGPCG_ERR_INVALID_ARG, "level " + std::to_string(level) + " out of range");
    return MGPCG_OK;
}
mgpcg_status check_layout(int layout) {
    if (layout != MGPCG_LAYOUT_NATURAL && layout != MGPCG_LAYOUT_INTERNAL)
        return fail(MGPCG_ERR_INVALID_ARG, "layout must be MGPCG_LAYOUT_NATURAL or MGPCG_LAYOUT_INTERNAL");
    return MGPCG_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

mgpcg_status ensure_scratch(mgpcg_problem *P, int l) {
    Level &Lv = P->lev[l];
    if (!Lv.t0) {
        ST_TRY(dalloc(&Lv.t0, Lv.n * P->R));
        ST_TRY(dalloc(&Lv.t1, Lv.n * P->R));
        ST_TRY(dalloc(&Lv.t2, Lv.n * P->R));
    }
    return MGPCG_OK;
}

// bring an FP64 level vector into internal layout (copy into dst when natural)
mgpcg_status in_vec(const mgpcg_problem *P, int l, const double *src, double *dst, int layout, hipStream_t s) {
    if (layout == MGPCG_LAYOUT_NATURAL) HIP_TRY(launch_permute(P, l, src, dst, true, s));
    else HIP_TRY(hipMemcpyAsync(dst, src, P->lev[l].n * P->R * sizeof(double), hipMemcpyDeviceToDevice, s));
    return MGPCG_OK;
}
mgpcg_status out_vec(const mgpcg_problem *P, int l, const double *src, double *dst, int layout, hipStream_t s) {
    if (layout == MGPCG_LAYOUT_NATURAL) HIP_TRY(launch_permute(P, l, src, dst, false, s));
    else HIP_TRY(hipMemcpyAsync(dst, src, P->lev[l].n * P->R * sizeof(double), hipMemcpyDeviceToDevice, s));
    return MGPCG_OK;
}

// clear the persistent kernel's barrier flags, epoch base and error flag
mgpcg_status reset_coarse(mgpcg_problem *P, hipStream_t s) {
    if (!P->coarse_ok) return MGPCG_OK;
    HIP_TRY(launch_fill_u(P->coarse_flags, (int64_t)P->coarse_blocks + 1, 0u, s));
    HIP_TRY(launch_fill_i(P->coarse_err, 1, 0, s));
    return MGPCG_OK;
}

// synchronises; reports a device-side failure of the coarse-level kernel
mgpcg_status device_error(mgpcg_problem *P, hipStream_t s) {
    HIP_TRY(hipStreamSynchronize(s));
    if (!P->coarse_ok) return MGPCG_OK;
    int err = 0;
    HIP_TRY(hipMemcpy(&err, P->coarse_err, sizeof(int), hipMemcpyDeviceToHost));
    if (err) return fail(MGPCG_ERR_HIP, "a grid barrier of the coarse-level kernel timed out");
    return MGPCG_OK;
}

mgpcg_status fetch_result(mgpcg_problem *P, int max_iters, double *history_host, int *iters_host,
                          hipStream_t s) {
    const int S = P->S;
    ST_TRY(device_error(P, s));
    std::vector<int> iters(S), status(S);
    HIP_TRY(hipMemcpyAsync(iters.data(), P->sc.iter, S * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(status.data(), P->sc.status, S * sizeof(int), hipMemcpyDeviceToHost, s));
    std::vector<double> hist;
    if (history_host && max_iters > 0) {
        if (max_iters > P->hist_cap) return fail(MGPCG_ERR_INVALID_ARG, "max_iters exceeds the last solve's");
        hist.resize((size_t)S * P->hist_cap);
        HIP_TRY(hipMemcpyAsync(hist.data(), P->hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (iters_host) memcpy(iters_host, iters.data(), S * sizeof(int));
    for (int i = 0; i < S && !hist.empty(); ++i)
        memcpy(history_host + (size_t)i * max_iters, hist.data() + (size_t)i * P->hist_cap,
               (size_t)max_iters * sizeof(double));
    bool breakdown = false, unconverged = false;
    for (int i = 0; i < S; ++i) {
        if (status[i] == MGPCG_ERR_BREAKDOWN) breakdown = true;
        else if (status[i] != 1 && P->last_tol > 0.0) unconverged = true;
    }
    if (breakdown) return fail(MGPCG_ERR_BREAKDOWN, "<p,Ap> was not finite or not positive for some system");
    return unconverged ? MGPCG_NOT_CONVERGED : MGPCG_OK;
}

// Runs `body(r_internal_T, z_internal_T)` at level l in the V-cycle precision
// with FP64 caller vectors r (read) and z (read/write), any layout.
template <typename F>
mgpcg_status with_level_vectors(mgpcg_problem *p, int l, const double *r, double *z, int layout,
                                       hipStream_t s, bool read_z, F body) {
    ST_TRY(ensure_scratch(p, l));
    Level &Lv = p->lev[l];
    const int64_t n = Lv.n * p->R;
    const double *ri = r;
    double *zi = z;
    if (layout == MGPCG_LAYOUT_NATURAL) {
        HIP_TRY(launch_permute(p, l, r, Lv.t0, true, s));
        if (read_z) HIP_TRY(launch_permute(p, l, z, Lv.t1, true, s));
        ri = Lv.t0;
        zi = Lv.t1;
    }
    if (p->mg_dtype == MGPCG_FP64) {
        HIP_TRY(body((const void *)ri, (void *)zi));
    } else {
        HIP_TRY(launch_cast_d2f(ri, (float *)Lv.r, n, s));
        if (read_z) HIP_TRY(launch_cast_d2f(zi, (float *)Lv.z, n, s));
        HIP_TRY(body((const void *)Lv.r, Lv.z));
        HIP_TRY(launch_cast_f2d((const float *)Lv.z, zi, n, s));
    }
    if (layout == MGPCG_LAYOUT_NATURAL) HIP_TRY(launch_permute(p, l, zi, z, false, s));
    return MGPCG_OK;
}

// ------------------------------------------------------------ schedule

mgpcg_schedule schedule_of(const mgpcg_problem *P) {
    mgpcg_schedule S{};
    S.graph = P->use_graph;
    S.coarse_mode = P->coarse_mode;
    S.coarse_tail = P->tail_on;
    S.wide_levels = 0;
    for (int l = 0; l < P->L; ++l)
        if (P->lev[l].stream_nt) S.wide_levels |= 1u << l;
    S.lex_run_rows = P->lex_run_rows;
    return S;
}

bool same_schedule(const mgpcg_schedule &a, const mgpcg_schedule &b) {
    return a.graph == b.graph && a.coarse_mode == b.coarse_mode && a.coarse_tail == b.coarse_tail &&
           a.wide_levels == b.wide_levels && a.lex_run_rows == b.lex_run_rows;
}

mgpcg_status apply_schedule(mgpcg_problem *P, const mgpcg_schedule &S, hipStream_t s) {
    if (S.graph != 0 && S.graph != 1) return fail(MGPCG_ERR_INVALID_ARG, "schedule.graph must be 0 or 1");
    if (S.coarse_mode != 0 && S.coarse_mode != 1)
        return fail(MGPCG_ERR_INVALID_ARG, "schedule.coarse_mode must be 0 or 1");
    if (S.coarse_tail != 0 && S.coarse_tail != 1)
        return fail(MGPCG_ERR_INVALID_ARG, "schedule.coarse_tail must be 0 or 1");
    if (S.wide_levels >> P->L)
        return fail(MGPCG_ERR_INVALID_ARG, "schedule.wide_levels has bits at or above the level count");
    if (S.lex_run_rows < 0 || S.lex_run_rows > 512)
        return fail(MGPCG_ERR_INVALID_ARG, "schedule.lex_run_rows must be in 0..512");
    bool l0 = false;
    for (int l = 0; l < P->L; ++l) {
        Level &Lv = P->lev[l];
        const bool wide = (S.wide_levels >> l) & 1u;
        if (wide == Lv.stream_nt) continue;
        Lv.stream_nt = wide;
        Lv.pass_tab = Lv.pass_tab_v[wide];
        Lv.pass_first = Lv.pass_first_v[wide];
        if (l == 0) l0 = true;
    }
    if (l0 && P->fuse_rz) HIP_TRY(set_rz_layout(P, s));
    P->use_graph = S.graph;
    P->coarse_mode = S.coarse_mode;
    P->tail_on = S.coarse_tail;
    if (S.lex_run_rows != P->lex_run_rows) {
        P->lex_run_rows = S.lex_run_rows;
        if (P->smoother == MGPCG_SMOOTHER_SEQUENTIAL)
            for (auto &Lv : P->lev) make_wave_plan(Lv, P->lex_run_rows);
    }
    if (P->iter_graph) {
        (void)hipGraphExecDestroy(P->iter_graph);
        P->iter_graph = nullptr;
    }
    return MGPCG_OK;
}

// what a tuned schedule depends on: the device kind and the problem's shape
std::string problem_signature(const mgpcg_problem *P) {
    hipDeviceProp_t prop;
    std::string dev = "unknown";
    if (hipGetDeviceProperties(&prop, P->device) == hipSuccess)
        dev = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
    std::string k = "dev=" + dev + ";dims=";
    for (int g = 0; g < P->G; ++g) {
        if (g) k += ",";
        k += std::to_string(P->dims0[3 * g]) + "x" + std::to_string(P->dims0[3 * g + 1]) + "x" +
             std::to_string(P->dims0[3 * g + 2]);
    }
    k += ";levels=" + std::to_string(P->L) + ";nrhs=" + std::to_string(P->R) + ";mg_dtype=" +
         std::to_string(P->mg_dtype) + ";colour_order=" + std::to_string(P->colour_order) + ";smoother=" +
         std::to_string(P->smoother) + ";sweeps=" + std::to_string(P->sweeps);
    return k;
}

// integer field `name` of one cache line; false if absent
bool cache_field(const std::string &line, const char *name, long long *v) {
    const std::string tag = std::string("\"") + name + "\": ";
    const size_t at = line.find(tag);
    if (at == std::string::npos) return false;
    char *end = nullptr;
    const char *p = line.c_str() + at + tag.size();
    *v = strtoll(p, &end, 10);
    return end != p;
}

// the last entry of the cache file for `key`, if any
bool cache_lookup(const char *path, const std::string &key, mgpcg_schedule *S) {
    std::ifstream f(path);
    if (!f) return false;
    const std::string want = "\"key\": \"" + key + "\"";
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        if (line.find(want) == std::string::npos) continue;
        long long g, cm, ct, wl, lr;
        if (!cache_field(line, "graph", &g) || !cache_field(line, "coarse_mode", &cm) ||
            !cache_field(line, "coarse_tail", &ct) || !cache_field(line, "wide_levels", &wl) ||
            !cache_field(line, "lex_run_rows", &lr))
            continue;
        S->graph = (int)g;
        S->coarse_mode = (int)cm;
        S->coarse_tail = (int)ct;
        S->wide_levels = (unsigned)wl;
        S->lex_run_rows = (int)lr;
        found = true;
    }
    return found;
}

bool cache_append(const char *path, const std::string &key, const mgpcg_schedule &S, double ms, int iters) {
    std::ofstream f(path, std::ios::app);
    if (!f) return false;
    f << "{\"key\": \"" << key << "\", \"graph\": " << S.graph << ", \"coarse_mode\": " << S.coarse_mode
      << ", \"coarse_tail\": " << S.coarse_tail << ", \"wide_levels\": " << S.wide_levels
      << ", \"lex_run_rows\": " << S.lex_run_rows << ", \"ms\": " << ms << ", \"iters\": " << iters << "}\n";
    return (bool)f;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// best time in ms of `reps` runs of `iters` PCG iterations from x = 0 under
// schedule S, after one warm-up run (b and x internal layout)
mgpcg_status time_schedule(mgpcg_problem *P, const mgpcg_schedule &S, const double *b, double *x, int iters,
                           int reps, hipStream_t s, double *best_ms) {
    ST_TRY(apply_schedule(P, S, s));
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    const int64_t n = P->lev[0].n * P->R;
    double best = 1e300;
    for (int r = 0; r <= reps; ++r) {
        HIP_TRY(launch_fill_d(x, n, 0.0, s));
        HIP_TRY(hipEventRecord(ev.a, s));
        ST_TRY(mgpcg_pcg_solve(P, b, x, iters, 0.0, nullptr, nullptr, MGPCG_LAYOUT_INTERNAL, s));
        HIP_TRY(hipEventRecord(ev.b, s));
        HIP_TRY(hipEventSynchronize(ev.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
        if (r > 0) best = std::min(best, (double)ms);
    }
    ST_TRY(device_error(P, s));
    *best_ms = best;
    return MGPCG_OK;
}

}  // namespace

// ----------------------------------- staging of the no-allocation entry point
//
// mgpcg_mg_vcycle_noalloc permutes natural-layout vectors through this array
// instead of buffers it would allocate: r in its first half, z in its second.
// One copy per device, held by the code object until the process ends.  In
// host code the symbol is not a device address: kernels get the address that
// hipGetSymbolAddress returns on each device (kept in g_scratch by device).
constexpr int64_t kScratchDoubles = int64_t(1) << 22;  // 32 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
std::mutex g_scratch_mu;
std::vector<double *> g_scratch;  // by device; NULL until looked up

// the device address of `scratch` on device `dev`, which must be current
mgpcg_status scratch_on_device(int dev, double **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = (double *)ptr;
    }
    *out = g_scratch[dev];
    return MGPCG_OK;
}
}  // namespace

// ====================================================================== C ABI

extern "C" {

const char *mgpcg_last_error(void) { return g_err.c_str(); }

mgpcg_status mgpcg_create(const mgpcg_config *cfg, hipStream_t stream, mgpcg_problem **out) {
    if (!out) return fail(MGPCG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg || !cfg->dims) return fail(MGPCG_ERR_INVALID_ARG, "config or dims is NULL");
    if (cfg->ngrids < 1 || cfg->ngrids > 32767) return fail(MGPCG_ERR_DIMS, "ngrids must be in 1..32767");
    if (cfg->levels < 1 || cfg->levels > MGPCG_MAX_LEVELS)
        return fail(MGPCG_ERR_DIMS, "levels must be in 1.." + std::to_string(MGPCG_MAX_LEVELS));
    const int R = cfg->nrhs;
    if (R != 1 && R != 2 && R != 4 && R != 8 && R != 16)
        return fail(MGPCG_ERR_INVALID_ARG, "nrhs must be 1, 2, 4, 8 or 16");
    if (cfg->mg_dtype != MGPCG_FP64 && cfg->mg_dtype != MGPCG_FP32)
        return fail(MGPCG_ERR_INVALID_ARG, "mg_dtype must be MGPCG_FP64 or MGPCG_FP32");
    if (cfg->colour_order != 0 && cfg->colour_order != 1)
        return fail(MGPCG_ERR_INVALID_ARG, "colour_order must be 0 or 1");
    if (cfg->smoother != MGPCG_SMOOTHER_COLOURED && cfg->smoother != MGPCG_SMOOTHER_SEQUENTIAL)
        return fail(MGPCG_ERR_INVALID_ARG, "smoother must be MGPCG_SMOOTHER_COLOURED or MGPCG_SMOOTHER_SEQUENTIAL");
    if (cfg->sweeps < 0 || cfg->sweeps > MGPCG_MAX_SWEEPS)
        return fail(MGPCG_ERR_INVALID_ARG, "sweeps must be in 0.." + std::to_string(MGPCG_MAX_SWEEPS));
    if (cfg->smoother == MGPCG_SMOOTHER_SEQUENTIAL && (cfg->mg_dtype != MGPCG_FP64 || R != 1))
        return fail(MGPCG_ERR_INVALID_ARG, "the sequential smoother needs mg_dtype MGPCG_FP64 and nrhs 1");
    const int div = 1 << (cfg->levels - 1);
    int64_t total = 0;
    for (int g = 0; g < cfg->ngrids; ++g) {
        for (int a = 0; a < 3; ++a) {
            int d = cfg->dims[3 * g + a];
            if (d < 1) return fail(MGPCG_ERR_DIMS, "grid dimensions must be >= 1");
            if (d % div)
                return fail(MGPCG_ERR_DIMS, "grid " + std::to_string(g) + ": dimension " + std::to_string(d) +
                                                " not divisible by 2^(levels-1) = " + std::to_string(div));
        }
        total += (int64_t)cfg->dims[3 * g] * cfg->dims[3 * g + 1] * cfg->dims[3 * g + 2];
        if (total > ((int64_t)1 << 31) / kW) return fail(MGPCG_ERR_DIMS, "problem too large");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(MGPCG_ERR_NO_DEVICE, "no HIP device available");
    }
    mgpcg_problem *P = new (std::nothrow) mgpcg_problem();
    if (!P) return fail(MGPCG_ERR_OOM, "host allocation failed");
    if (hipGetDevice(&P->device) != hipSuccess) {
        delete P;
        return fail(MGPCG_ERR_NO_DEVICE, "hipGetDevice failed");
    }
    // set-up of the no-allocation entry point on this device (once per device)
    double *scr = nullptr;
    if (mgpcg_status sst = scratch_on_device(P->device, &scr); sst != MGPCG_OK) {
        delete P;
        return sst;
    }
    P->G = cfg->ngrids;
    P->R = R;
    P->S = P->G * R;
    P->L = cfg->levels;
    P->mg_dtype = cfg->mg_dtype;
    P->colour_order = cfg->colour_order;
    P->smoother = cfg->smoother;
    P->sweeps = cfg->sweeps == 0 ? 1 : cfg->sweeps;
    P->dims0.assign(cfg->dims, cfg->dims + 3 * cfg->ngrids);
    // tuning and test override: 0 int32 columns, 1 at most int8 deltas, 2 (default) implied columns allowed
    if (const char *env = getenv("MGPCG_DELTA_COLS")) P->col_format = std::min(2, std::max(0, atoi(env)));
    mgpcg_status st = build_hierarchy(P, cfg->theta, stream);
    if (st != MGPCG_OK) {
        std::string msg = g_err;
        free_problem(P);
        g_err = msg;
        return st;
    }
    *out = P;
    return MGPCG_OK;
}

mgpcg_status mgpcg_destroy(mgpcg_problem *p) {
    free_problem(p);
    return MGPCG_OK;
}

mgpcg_status mgpcg_info(const mgpcg_problem *p, int level, int64_t *n, int64_t *nnz, int64_t *ell_slots) {
    ST_TRY(check_level(p, level));
    const Level &Lv = p->lev[level];
    if (n) *n = Lv.n;
    if (nnz) *nnz = Lv.nnz;
    if (ell_slots) *ell_slots = Lv.n * kW;
    return MGPCG_OK;
}

mgpcg_status mgpcg_set_theta(mgpcg_problem *p, const double *theta, hipStream_t stream) {
    ST_TRY(check_problem(p));
    DeviceGuard dg(p->device);
    for (int l = 0; l < p->L; ++l) {
        HIP_TRY(launch_build_ell(p, l, theta, stream));
        if (p->smoother == MGPCG_SMOOTHER_SEQUENTIAL) HIP_TRY(launch_wave_gather(p, l, stream));
    }
    return MGPCG_OK;
}

mgpcg_status mgpcg_to_internal(const mgpcg_problem *p, int level, const double *src, double *dst,
                               hipStream_t stream) {
    ST_TRY(check_level(p, level));
    if (!src || !dst) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    DeviceGuard dg(p->device);
    HIP_TRY(launch_permute(p, level, src, dst, true, stream));
    return MGPCG_OK;
}

mgpcg_status mgpcg_to_natural(const mgpcg_problem *p, int level, const double *src, double *dst,
                              hipStream_t stream) {
    ST_TRY(check_level(p, level));
    if (!src || !dst) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    DeviceGuard dg(p->device);
    HIP_TRY(launch_permute(p, level, src, dst, false, stream));
    return MGPCG_OK;
}

mgpcg_status mgpcg_spmv(const mgpcg_problem *p_, int level, const double *x, double *y, int layout,
                        hipStream_t s) {
    ST_TRY(check_level(p_, level));
    ST_TRY(check_layout(layout));
    if (!x || !y) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    mgpcg_problem *p = const_cast<mgpcg_problem *>(p_);
    DeviceGuard dg(p->device);
    ST_TRY(ensure_scratch(p, level));
    Level &Lv = p->lev[level];
    const int64_t n = Lv.n * p->R;
    const bool f64 = (level == 0 || p->mg_dtype == MGPCG_FP64);
    const double *xi = x;
    double *yi = y;
    if (layout == MGPCG_LAYOUT_NATURAL) {
        HIP_TRY(launch_permute(p, level, x, Lv.t0, true, s));
        xi = Lv.t0;
        yi = Lv.t1;
    }
    if (f64) {
        HIP_TRY(launch_spmv<double>(p, level, Lv.val64, xi, yi, s));
    } else {
        HIP_TRY(launch_cast_d2f(xi, (float *)Lv.r, n, s));
        HIP_TRY(launch_spmv<float>(p, level, Lv.val32, (const float *)Lv.r, (float *)Lv.z, s));
        HIP_TRY(launch_cast_f2d((const float *)Lv.z, yi, n, s));
    }
    if (layout == MGPCG_LAYOUT_NATURAL) HIP_TRY(launch_permute(p, level, yi, y, false, s));
    return MGPCG_OK;
}

mgpcg_status mgpcg_make_rhs_ones(const mgpcg_problem *p_, double *b, int layout, hipStream_t s) {
    ST_TRY(check_problem(p_));
    ST_TRY(check_layout(layout));
    if (!b) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    mgpcg_problem *p = const_cast<mgpcg_problem *>(p_);
    DeviceGuard dg(p->device);
    ST_TRY(ensure_scratch(p, 0));
    Level &L0 = p->lev[0];
    HIP_TRY(launch_fill_d(L0.t0, L0.n * p->R, 1.0, s));
    if (layout == MGPCG_LAYOUT_NATURAL) {
        HIP_TRY(launch_spmv<double>(p, 0, L0.val64, L0.t0, L0.t1, s));
        HIP_TRY(launch_permute(p, 0, L0.t1, b, false, s));
    } else {
        HIP_TRY(launch_spmv<double>(p, 0, L0.val64, L0.t0, b, s));
    }
    return MGPCG_OK;
}

mgpcg_status mgpcg_gs_sweep(const mgpcg_problem *p_, int level, const double *r, double *z, int layout,
                            hipStream_t s) {
    ST_TRY(check_level(p_, level));
    ST_TRY(check_layout(layout));
    if (!r || !z) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    mgpcg_problem *p = const_cast<mgpcg_problem *>(p_);
    DeviceGuard dg(p->device);
    return with_level_vectors(p, level, r, z, layout, s, true, [&](const void *rv, void *zv) {
        if (p->smoother == MGPCG_SMOOTHER_SEQUENTIAL)
            return launch_lex_sweep(p, level, (const double *)rv, (double *)zv, s);
        if (p->mg_dtype == MGPCG_FP64)
            return sweep<double>(p, level, p->lev[level].val64, (const double *)rv, (double *)zv, kPassPlain,
                                 kPassPlain, (double *)nullptr, nullptr, s);
        return sweep<float>(p, level, p->lev[level].val32, (const float *)rv, (float *)zv, kPassPlain, kPassPlain,
                            (float *)nullptr, nullptr, s);
    });
}

mgpcg_status mgpcg_colour_pass(const mgpcg_problem *p_, int level, int colour, const double *r, double *z,
                               int layout, hipStream_t s) {
    ST_TRY(check_level(p_, level));
    ST_TRY(check_layout(layout));
    if (!r || !z) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    if (colour < 0 || colour >= p_->lev[level].ncol) return fail(MGPCG_ERR_INVALID_ARG, "no such colour at this level");
    mgpcg_problem *p = const_cast<mgpcg_problem *>(p_);
    DeviceGuard dg(p->device);
    return with_level_vectors(p, level, r, z, layout, s, true, [&](const void *rv, void *zv) {
        if (p->mg_dtype == MGPCG_FP64)
            return launch_pass<double>(p, level, colour, kPassPlain, p->lev[level].val64, (const double *)rv,
                                       (double *)zv, nullptr, (double *)nullptr, s);
        return launch_pass<float>(p, level, colour, kPassPlain, p->lev[level].val32, (const float *)rv, (float *)zv,
                                  nullptr, (float *)nullptr, s);
    });
}

mgpcg_status mgpcg_restrict(const mgpcg_problem *p_, int level, const double *r, const double *z, double *rc,
                            int layout, hipStream_t s) {
    ST_TRY(check_level(p_, level, true));
    ST_TRY(check_layout(layout));
    if (!r || !z || !rc) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    mgpcg_problem *p = const_cast<mgpcg_problem *>(p_);
    DeviceGuard dg(p->device);
    ST_TRY(ensure_scratch(p, level));
    ST_TRY(ensure_scratch(p, level + 1));
    Level &F = p->lev[level];
    Level &C = p->lev[level + 1];
    const int64_t nf = F.n * p->R, nc = C.n * p->R;
    ST_TRY(in_vec(p, level, r, F.t0, layout, s));
    ST_TRY(in_vec(p, level, z, F.t1, layout, s));
    if (p->mg_dtype == MGPCG_FP64) {
        HIP_TRY(launch_restrict<double>(p, level, F.val64, F.t0, F.t1, C.t2, s));
    } else {
        HIP_TRY(launch_cast_d2f(F.t0, (float *)F.r, nf, s));
        HIP_TRY(launch_cast_d2f(F.t1, (float *)F.z, nf, s));
        HIP_TRY(launch_restrict<float>(p, level, F.val32, (const float *)F.r, (const float *)F.z, (float *)C.r, s));
        HIP_TRY(launch_cast_f2d((const float *)C.r, C.t2, nc, s));
    }
    return out_vec(p, level + 1, C.t2, rc, layout, s);
}

mgpcg_status mgpcg_prolong_add(const mgpcg_problem *p_, int level, const double *zc, double *z, int layout,
                               hipStream_t s) {
    ST_TRY(check_level(p_, level, true));
    ST_TRY(check_layout(layout));
    if (!zc || !z) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    mgpcg_problem *p = const_cast<mgpcg_problem *>(p_);
    DeviceGuard dg(p->device);
    ST_TRY(ensure_scratch(p, level));
    ST_TRY(ensure_scratch(p, level + 1));
    Level &F = p->lev[level];
    Level &C = p->lev[level + 1];
    const int64_t nf = F.n * p->R, nc = C.n * p->R;
    ST_TRY(in_vec(p, level + 1, zc, C.t0, layout, s));
    ST_TRY(in_vec(p, level, z, F.t1, layout, s));
    if (p->mg_dtype == MGPCG_FP64) {
        HIP_TRY(launch_prolong<double>(p, level, C.t0, F.t1, s));
    } else {
        HIP_TRY(launch_cast_d2f(C.t0, (float *)C.z, nc, s));
        HIP_TRY(launch_cast_d2f(F.t1, (float *)F.z, nf, s));
        HIP_TRY(launch_prolong<float>(p, level, (const float *)C.z, (float *)F.z, s));
        HIP_TRY(launch_cast_f2d((const float *)F.z, F.t1, nf, s));
    }
    return out_vec(p, level, F.t1, z, layout, s);
}

mgpcg_status mgpcg_mg_vcycle(const mgpcg_problem *p_, const double *r, double *z, int layout, hipStream_t s) {
    ST_TRY(check_problem(p_));
    ST_TRY(check_layout(layout));
    if (!r || !z) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    mgpcg_problem *p = const_cast<mgpcg_problem *>(p_);
    DeviceGuard dg(p->device);
    ST_TRY(reset_coarse(p, s));
    return with_level_vectors(p, 0, r, z, layout, s, false, [&](const void *rv, void *zv) {
        if (p->smoother == MGPCG_SMOOTHER_SEQUENTIAL) return vcycle_lex(p, (const double *)rv, (double *)zv, s);
        if (p->mg_dtype == MGPCG_FP64) return vcycle<double>(p, (const double *)rv, (double *)zv, nullptr, s);
        return vcycle<float>(p, (const float *)rv, (float *)zv, nullptr, s);
    });
}

mgpcg_status mgpcg_mg_vcycle_noalloc(const mgpcg_problem *p_, const double *r, double *z, int layout,
                                     hipStream_t s) {
    ST_TRY(check_problem(p_));
    ST_TRY(check_layout(layout));
    if (!r || !z) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    mgpcg_problem *p = const_cast<mgpcg_problem *>(p_);
    const int64_t n = p->lev[0].n * p->R;
    const bool natural = layout == MGPCG_LAYOUT_NATURAL;
    if (natural && 2 * n > kScratchDoubles)
        return fail(MGPCG_ERR_INVALID_ARG, "mgpcg_mg_vcycle_noalloc: " + std::to_string(n) +
                                               " level-0 values exceed the staging limit of " +
                                               std::to_string(kScratchDoubles / 2) +
                                               " in natural layout (use MGPCG_LAYOUT_INTERNAL)");
    DeviceGuard dg(p->device);
    double *scr = nullptr;
    ST_TRY(scratch_on_device(p->device, &scr));
    ST_TRY(reset_coarse(p, s));
    const double *ri = r;
    double *zi = z;
    if (natural) {
        HIP_TRY(launch_permute(p, 0, r, scr, true, s));
        ri = scr;
        zi = scr + n;
    }
    if (p->smoother == MGPCG_SMOOTHER_SEQUENTIAL) {
        HIP_TRY(vcycle_lex(p, ri, zi, s));
    } else if (p->mg_dtype == MGPCG_FP64) {
        HIP_TRY(vcycle<double>(p, ri, zi, nullptr, s));
    } else {
        // the FP32 V-cycle runs in the handle's own level-0 vectors
        Level &L0 = p->lev[0];
        HIP_TRY(launch_cast_d2f(ri, (float *)L0.r, n, s));
        HIP_TRY(vcycle<float>(p, (const float *)L0.r, (float *)L0.z, nullptr, s));
        HIP_TRY(launch_cast_f2d((const float *)L0.z, zi, n, s));
    }
    if (natural) HIP_TRY(launch_permute(p, 0, zi, z, false, s));
    return MGPCG_OK;
}

mgpcg_status mgpcg_pcg_solve(mgpcg_problem *p, const double *b, double *x, int max_iters, double rel_tol,
                             double *history_host, int *iters_host, int layout, hipStream_t s) {
    ST_TRY(check_problem(p));
    ST_TRY(check_layout(layout));
    if (!b || !x) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    if (max_iters < 0) return fail(MGPCG_ERR_INVALID_ARG, "max_iters must be >= 0");
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol)) return fail(MGPCG_ERR_INVALID_ARG, "rel_tol must be finite and >= 0");
    DeviceGuard dg(p->device);
    const int S = p->S;
    const int64_t n = p->lev[0].n * p->R;
    if (max_iters > p->hist_cap) {
        int cap = std::max(max_iters, 64);
        double *h = nullptr;
        ST_TRY(dalloc(&h, (int64_t)S * cap));
        HIP_TRY(hipStreamSynchronize(s));
        dfree(p->hist);
        p->hist = h;
        p->hist_cap = cap;
        if (p->iter_graph) {
            (void)hipGraphExecDestroy(p->iter_graph);
            p->iter_graph = nullptr;
        }
    }
    p->last_max_iters = max_iters;
    if (p->iter_graph && p->last_tol != rel_tol) {
        (void)hipGraphExecDestroy(p->iter_graph);
        p->iter_graph = nullptr;
    }
    p->last_tol = rel_tol;

    ST_TRY(in_vec(p, 0, b, p->b, layout, s));
    ST_TRY(in_vec(p, 0, x, p->x, layout, s));
    Scalars &sc = p->sc;
    ST_TRY(reset_coarse(p, s));
    HIP_TRY(launch_fill_i(sc.done, S, 0, s));
    HIP_TRY(launch_fill_i(sc.status, S, 0, s));
    HIP_TRY(launch_fill_i(sc.iter, S, 0, s));
    HIP_TRY(launch_fill_i(sc.ndone, 1, 0, s));
    HIP_TRY(launch_fill_d(sc.rho_old, S, 0.0, s));
    HIP_TRY(launch_fill_d(sc.apend, S, 0.0, s));
    HIP_TRY(launch_fill_d(p->hist, (int64_t)S * p->hist_cap, 0.0, s));
    HIP_TRY(launch_fill_d(p->p, n, 0.0, s));
    HIP_TRY(launch_init_residual(p, s));
    // the first FP32 V-cycle's right-hand side (later ones are stored by the
    // residual updates)
    if (fused_fp32(p)) HIP_TRY(launch_cast_d2f(p->r, (float *)p->lev[0].r, p->lev[0].n * p->R, s));

    if (p->use_graph && !p->iter_graph && max_iters > 0) {
        if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t ce = cg_iteration(p, rel_tol, p->cap_stream);
        hipError_t ee = hipStreamEndCapture(p->cap_stream, &graph);
        if (ce != hipSuccess) return hip_fail(ce, "capturing the CG iteration");
        if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
        hipError_t ie = hipGraphInstantiate(&p->iter_graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            p->iter_graph = nullptr;
            return hip_fail(ie, "hipGraphInstantiate");
        }
    }
    // Tolerance checks: the count of finished systems is posted after every
    // iteration (every 4th on small problems, whose iterations are short) and
    // read once a later iteration is queued behind it, so the host never
    // drains the stream.  Iterations queued after the last system finished
    // change nothing (converged systems store nothing), they only cost time:
    // at most check_every + 1 of them.
    const bool check = rel_tol > 0.0;
    const int check_every = p->lev[0].n * p->R >= (1 << 20) ? 1 : 4;
    constexpr int kRing = mgpcg_problem::kCheckRing;
    int posted[kRing];  // iteration after which each outstanding slot was posted
    int head = 0, tail = 0;
    bool finished = false;
    for (int it = 0; it < max_iters && !finished; ++it) {
        // read every posted count that has an iteration queued behind it
        // (and the oldest one when the ring is full)
        while (check && tail > head && (posted[head % kRing] <= it - 2 || tail - head == kRing)) {
            const int j = head % kRing;
            HIP_TRY(hipEventSynchronize(p->check_ev[j]));
            ++head;
            if (p->pinned_ndone[j] >= S) {
                finished = true;
                break;
            }
        }
        if (finished) break;
        if (p->iter_graph) HIP_TRY(hipGraphLaunch(p->iter_graph, s));
        else HIP_TRY(cg_iteration(p, rel_tol, s));
        if (check && (it + 1) % check_every == 0 && it + 1 < max_iters) {
            const int j = tail % kRing;
            HIP_TRY(hipMemcpyAsync(p->pinned_ndone + j, sc.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipEventRecord(p->check_ev[j], s));
            posted[j] = it;
            ++tail;
        }
    }
    // the last iteration's x update (each iteration's is applied by the next)
    HIP_TRY(launch_flush_x(p, s));
    ST_TRY(out_vec(p, 0, p->x, x, layout, s));
    if (!history_host && !iters_host && rel_tol == 0.0) return MGPCG_OK;
    return fetch_result(p, max_iters, history_host, iters_host, s);
}

mgpcg_status mgpcg_solve_result(mgpcg_problem *p, int max_iters, double *history_host, int *iters_host,
                                hipStream_t s) {
    ST_TRY(check_problem(p));
    if (max_iters < 0) return fail(MGPCG_ERR_INVALID_ARG, "max_iters must be >= 0");
    DeviceGuard dg(p->device);
    return fetch_result(p, max_iters, history_host, iters_host, s);
}

mgpcg_status mgpcg_theta_grad(const mgpcg_problem *p, const double *lambda, const double *x,
                              const double *theta, double *grad, hipStream_t s) {
    ST_TRY(check_problem(p));
    if (!lambda || !x || !theta || !grad) return fail(MGPCG_ERR_INVALID_ARG, "NULL vector");
    if (p->R != 1) return fail(MGPCG_ERR_INVALID_ARG, "theta_grad needs nrhs == 1");
    DeviceGuard dg(p->device);
    HIP_TRY(launch_theta_grad(lambda, x, theta, grad, p->lev[0].n, s));
    return MGPCG_OK;
}

mgpcg_status mgpcg_set_graph_mode(mgpcg_problem *p, int on) {
    ST_TRY(check_problem(p));
    p->use_graph = on ? 1 : 0;
    if (!on && p->iter_graph) {
        (void)hipGraphExecDestroy(p->iter_graph);
        p->iter_graph = nullptr;
    }
    return MGPCG_OK;
}

mgpcg_status mgpcg_set_coarse_mode(mgpcg_problem *p, int mode) {
    ST_TRY(check_problem(p));
    if (mode != 0 && mode != 1) return fail(MGPCG_ERR_INVALID_ARG, "coarse mode must be 0 or 1");
    p->coarse_mode = mode;
    if (p->iter_graph) {
        (void)hipGraphExecDestroy(p->iter_graph);
        p->iter_graph = nullptr;
    }
    return MGPCG_OK;
}

mgpcg_status mgpcg_get_schedule(const mgpcg_problem *p, mgpcg_schedule *out) {
    ST_TRY(check_problem(p));
    if (!out) return fail(MGPCG_ERR_INVALID_ARG, "out is NULL");
    *out = schedule_of(p);
    return MGPCG_OK;
}

mgpcg_status mgpcg_set_schedule(mgpcg_problem *p, const mgpcg_schedule *sched, hipStream_t stream) {
    ST_TRY(check_problem(p));
    if (!sched) return fail(MGPCG_ERR_INVALID_ARG, "schedule is NULL");
    DeviceGuard dg(p->device);
    return apply_schedule(p, *sched, stream);
}

mgpcg_status mgpcg_autotune(mgpcg_problem *p, const double *b, int iters, int reps, const char *cache_path,
                            mgpcg_schedule *chosen, hipStream_t s) {
    ST_TRY(check_problem(p));
    if (iters < 1 || iters > 1000) return fail(MGPCG_ERR_INVALID_ARG, "iters must be in 1..1000");
    if (reps < 1 || reps > 100) return fail(MGPCG_ERR_INVALID_ARG, "reps must be in 1..100");
    DeviceGuard dg(p->device);
    const std::string key = problem_signature(p);
    mgpcg_schedule S = schedule_of(p);
    if (cache_path && cache_lookup(cache_path, key, &S)) {
        // apply_schedule checks every field before it changes anything; an
        // entry it rejects (an edited file) is ignored and the tuning runs
        if (apply_schedule(p, S, s) == MGPCG_OK) {
            if (chosen) *chosen = schedule_of(p);
            return MGPCG_OK;
        }
        S = schedule_of(p);
    }
    // right-hand side and iterate in the internal layout, owned by this call
    Level &L0 = p->lev[0];
    const int64_t n = L0.n * p->R;
    double *bi = nullptr, *xi = nullptr;
    ST_TRY(dalloc(&bi, n));
    mgpcg_status st = dalloc(&xi, n);
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        dfree(bi);
        dfree(xi);
    };
    if (st != MGPCG_OK) {
        cleanup();
        return st;
    }
    hipError_t e = b ? launch_permute(p, 0, b, bi, true, s) : hipSuccess;
    if (!b && e == hipSuccess) {
        e = launch_fill_d(xi, n, 1.0, s);
        if (e == hipSuccess) e = launch_spmv<double>(p, 0, L0.val64, xi, bi, s);
    }
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "autotune: right-hand side");
    }
    const mgpcg_schedule start = S;
    mgpcg_schedule best = S;
    double best_ms = 0;
    st = time_schedule(p, best, bi, xi, iters, reps, s, &best_ms);
    auto consider = [&](const mgpcg_schedule &c) {
        if (st != MGPCG_OK || same_schedule(c, best)) return;
        double ms = 0;
        st = time_schedule(p, c, bi, xi, iters, reps, s, &ms);
        if (st == MGPCG_OK && ms < best_ms) {
            best = c;
            best_ms = ms;
        }
    };
    // graph replay or eager launches
    {
        mgpcg_schedule c = best;
        c.graph ^= 1;
        consider(c);
    }
    const bool coloured = p->smoother == MGPCG_SMOOTHER_COLOURED;
    if (coloured) {
        // coarse levels: per-pass kernels with or without the tail kernel,
        // or the persistent kernel
        for (int cm = 0; cm < 2; ++cm)
            for (int ct = 0; ct < 2; ++ct) {
                if (cm == 1 && !p->coarse_ok) continue;
                if (ct == 1 && !p->tail_ok) continue;
                mgpcg_schedule c = best;
                c.coarse_mode = cm;
                c.coarse_tail = ct;
                consider(c);
            }
        // each level's workgroup choice; levels that the tail or persistent
        // kernel runs have no colour-pass launches to tune
        const bool persistent = p->coarse_ok && best.coarse_mode == 1;
        const bool tail = !persistent && p->tail_ok && best.coarse_tail == 1;
        const int lmax = persistent ? p->coarse_lc : (tail ? p->tail_lw : p->L);
        for (int l = 0; l < lmax; ++l) {
            if (l == 0 && p->fuse_rz) continue;  // would regroup the <r,z> partials
            mgpcg_schedule c = best;
            c.wide_levels ^= 1u << l;
            consider(c);
        }
    } else {
        for (int rr : {0, 64, 128, 256, 512}) {
            mgpcg_schedule c = best;
            c.lex_run_rows = rr;
            consider(c);
        }
    }
    if (st == MGPCG_OK) st = apply_schedule(p, best, s);
    else (void)apply_schedule(p, start, s);
    cleanup();
    if (st != MGPCG_OK) return st;
    if (cache_path && !cache_append(cache_path, key, best, best_ms, iters))
        return fail(MGPCG_ERR_INVALID_ARG, std::string("autotune: cannot append to ") + cache_path);
    if (chosen) *chosen = schedule_of(p);
    return MGPCG_OK;
}

mgpcg_status mgpcg_check(mgpcg_problem *p, hipStream_t stream) {
    ST_TRY(check_problem(p));
    DeviceGuard dg(p->device);
    return device_error(p, stream);
}

}  // extern "C"
