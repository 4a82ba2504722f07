// The k-marching tile of the sweep, shared by the pseudo-time step
// (sweep.hip) and the record pass of the discrete adjoint (adjoint.hip).
// Included by those two files only; both are built with -ffp-contract=off.
#pragma once

#include "cavity_internal.h"
#include "stencil.h"

namespace cav {

// ---------------------------------------------------------------------------
// The sweep.  Block = one TI x TJ tile of (i, j) columns, i along the lanes
// (64 x 8: one wavefront per j row; narrower tiles put 64 / TI rows in a
// wavefront) marching over a chunk of k planes.  Plane k of
// all five fields lives in LDS with its i/j halo (2 for p, 1 for the rest);
// the k neighbours come from per-thread register queues (p: k-2..k+2,
// others k-1..k+1).  The LDS planes are double-buffered: plane k+1 is
// written into one buffer while plane k is computed from the other, so each
// plane costs one barrier; global loads run two or three planes ahead.  Wall ghosts
// are derived from interior cells (in LDS for the i/j walls, by recurrences
// on the queues for the k walls); no ghost cell is read from HBM.
// LDS of one sweep block of TI x TJ threads: two planes of p (halo 2) and
// of u, v, w, T (halo 1), and one norm slot per wavefront.
template <typename Real, int TI_ = SW_TI, int TJ_ = SW_TJ>
struct SweepLds {
    static constexpr int TI = TI_, TJ = TJ_;
    static constexpr int PW = TI + 4;              // row pitch, p
    static constexpr int UW = TI + 2;              // row pitch, u v w T
    static constexpr int PPL = (TJ + 4) * PW;      // plane, p
    static constexpr int UPL = (TJ + 2) * UW;      // plane, one of u v w T
    static constexpr int NWAVE = TI * TJ / 64;
    Real p[2 * PPL];
    Real u[2 * 4 * UPL];
    double red[NWAVE][NF];
};

// What a sweep does with each cell's stars and residual: the pseudo-time
// update of Sec. 2 (q + dt R, then the centre rescale of p) streamed into
// qn, and R^2 into the norm accumulators.
template <typename Real>
struct StepEpi {
    StateT<Real> qn;
    Real pc_new;
    // New pressure at the centre cell, recomputed with the same arithmetic
    // as its owner, so that every block subtracts the identical value.
    __device__ __forceinline__ void prepare(const Dims& d, const CStateT<Real>& q, const CoefR<Real>& c)
    {
        Star<Real> s;
        gather_global(d, q, c, d.ni / 2, d.nj / 2, d.nk / 2, s);
        Real R[NF], dt;
        cell_residual(c, s, R, dt);
        pc_new = fma(dt, R[FP], s.p);
    }
    __device__ __forceinline__ void cell(const CoefR<Real>&, const Star<Real>& s, const Real R[NF], Real dt, int o,
                                         int, int, int, double acc[NF])
    {
        // the new state is not read again by this launch: stream it out
        __builtin_nontemporal_store(fma(dt, R[FP], s.p) - pc_new, &qn.f[FP][o]);
        __builtin_nontemporal_store(fma(dt, R[FU], s.u), &qn.f[FU][o]);
        __builtin_nontemporal_store(fma(dt, R[FV], s.v), &qn.f[FV][o]);
        __builtin_nontemporal_store(fma(dt, R[FW], s.w), &qn.f[FW][o]);
        __builtin_nontemporal_store(fma(dt, R[FT], s.t), &qn.f[FT][o]);
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] = fma((double)R[f], (double)R[f], acc[f]);
    }
};

// Where one block works: columns [i0, i0+TI) x [j0, j0+TJ), planes
// [k0, k1); its norm partial goes to slot pidx.
struct TileBox {
    int i0, j0, k0, k1, pidx;
};

// Logical tile b of the regular TI x TJ tiling with k chunks of length kc.
template <int TI = SW_TI, int TJ = SW_TJ>
__device__ __forceinline__ TileBox tile_box(const Dims& d, int tiles_i, int tiles_j, int kc, int b)
{
    const int bi = b % tiles_i;
    const int bj = (b / tiles_i) % tiles_j;
    const int bk = b / (tiles_i * tiles_j);
    TileBox t;
    t.i0 = bi * TI;
    t.j0 = bj * TJ;
    t.k0 = bk * kc;
    t.k1 = min(t.k0 + kc, d.nk);
    t.pidx = b;
    return t;
}

// Every cell of the box is updated.  column(i, j): whether any updated cell
// reads column (i, j).
struct OwnAll {
    __device__ __forceinline__ bool operator()(int, int, int) const { return true; }
    __device__ __forceinline__ bool column(int, int) const { return true; }
};

// One tile box: planes of its k range, cells for which own(i, j, k) holds
// are updated (and enter the norm).  Used by the single-cavity sweep, the
// batched kernel and the interior/exterior split.  The block has TI x TJ =
// 512 or 256 threads, launched as SW_TI x (TI TJ / SW_TI): thread t = lane +
// TI * row works on column (i0 + lane, j0 + row); TI >= 16 and TJ >= 4 (the
// halo roles below need 12 threads per row; 4-row tiles give each thread
// two of the eight u v w T halo rows).
template <typename Real, bool NORM, typename Own, typename Epi, int DEPTH = 3, int TI = SW_TI, int TJ = SW_TJ>
__device__ __forceinline__ void sweep_tile(const Dims& d, const CoefR<Real>& c, const TileBox& tb, const Own& own,
                                           const CStateT<Real>& q, Epi& epi, double* partials,
                                           SweepLds<Real, TI, TJ>& L)
{
    static_assert((TI * TJ == 512 || TI * TJ == 256) && TI >= 16 && (TJ >= 8 || TJ == 4),
                  "512- or 256-thread tiles, TI >= 16, TJ = 4 or >= 8");
    constexpr int UR = TJ >= 8 ? 1 : 2;            // u v w T halo rows per thread
    using Lds = SweepLds<Real, TI, TJ>;
    constexpr int PW = Lds::PW, UW = Lds::UW;
    constexpr int PPL = Lds::PPL, UPL = Lds::UPL;
    Real* const sP = L.p;
    Real* const sU = L.u;

    const int i0 = tb.i0, j0 = tb.j0;
    const int k0 = tb.k0, k1 = tb.k1;

    // launched as SW_TI x (TI TJ / SW_TI) threads; other shapes re-split the block
    const int tid = threadIdx.x + SW_TI * threadIdx.y;
    const int lane = TI == SW_TI ? (int)threadIdx.x : tid % TI;
    const int row = TI == SW_TI ? (int)threadIdx.y : tid / TI;
    const int i = i0 + lane, j = j0 + row;
    // columns no owned cell's star reaches are neither loaded nor computed
    const bool active = i < d.ni && j < d.nj && own.column(i, j);


    // ---- what this thread loads (fixed for the whole march) ----
    // Only interior cells are loaded.  LDS cells that hold wall ghosts are
    // filled from interior LDS cells (fix_ghosts), the k neighbours beyond
    // the z walls by recurrences on the register queues.
    auto interior = [&](int ii, int jj) { return ii >= 0 && ii < d.ni && jj >= 0 && jj < d.nj; };
    // p rows j0-2, j0-1, j0+TJ, j0+TJ+1: waves 0..3, one row each
    const bool has_prow = row < 4;
    const int prow_lds = row < 2 ? row : TJ + row;
    const int prow_j = j0 - 2 + prow_lds;
    const bool ld_prow = has_prow && interior(i, prow_j) && own.column(i, prow_j);
    // u v w T rows j0-1, j0+TJ: slot s = 0..7 is field 1 + s/2, side s&1;
    // this thread's slots are row (and row + 4 in 4-row tiles)
    bool has_urow[UR], ld_urow[UR];
    int urow_dst[UR], off_urow[UR];
    const Real* URg[UR];
#pragma unroll
    for (int r = 0; r < UR; ++r) {
        const int sl = row + 4 * r;
        has_urow[r] = sl < 8;
        const int uf = FU + (min(sl, 7) >> 1);
        const int ul = (sl & 1) ? TJ + 1 : 0;
        const int uj = j0 - 1 + ul;
        ld_urow[r] = has_urow[r] && interior(i, uj) && own.column(i, uj);
        urow_dst[r] = (uf - FU) * UPL + ul * UW + lane + 1;
        off_urow[r] = cell_off(d, i, uj, 0);
        URg[r] = q.f[uf];
    }
    // column halos of this wave's row: lanes 0..3 p (i0-2, i0-1, i0+TI,
    // i0+TI+1), lanes 4..11 u v w T (i0-1, i0+TI)
    const bool has_col = lane < 12;
    int col_f, col_lds, col_i;
    if (lane < 4) {
        col_f = FP;
        const int cc = lane < 2 ? lane : TI + lane;
        col_i = i0 - 2 + cc;
        col_lds = (row + 2) * PW + cc;
    } else {
        const int t = min(lane - 4, 7);
        col_f = FU + (t >> 1);
        const int cc = (t & 1) ? TI + 1 : 0;
        col_i = i0 - 1 + cc;
        col_lds = (col_f - FU) * UPL + (row + 1) * UW + cc;
    }
    const bool ld_col = has_col && interior(col_i, j);
    const int prow_dst = prow_lds * PW + lane + 2;
    const int off_c = cell_off(d, i, j, 0);
    const int off_prow = cell_off(d, i, prow_j, 0);
    const int off_col = cell_off(d, col_i, j, 0);
    const Real* const Pg = q.f[FP];
    const Real* const Ug = q.f[FU];
    const Real* const Vg = q.f[FV];
    const Real* const Wg = q.f[FW];
    const Real* const Tg = q.f[FT];
    const Real* const COLg = q.f[col_f];
    const int Z = d.sz;

    // tiles whose LDS planes reach past a wall fix their ghost cells
    const bool bnd = i0 == 0 || j0 == 0 || i0 + TI + 2 > d.ni || j0 + TJ + 2 > d.nj;
    auto fix_ghosts = [&](Real* fP, Real* fU, int k) __attribute__((always_inline)) {
        auto cell = [&](int f, int ci, int cj) -> Real& {
            return f == FP ? fP[(cj - j0 + 2) * PW + (ci - i0 + 2)]
                           : fU[(f - FU) * UPL + (cj - j0 + 1) * UW + (ci - i0 + 1)];
        };
        // y walls: column i0 + lane, fields row, row + TJ, ...
        for (int f = row; f < NF && i < d.ni; f += TJ) {
            const int reach = f == FP ? 2 : 1;
            if (j0 == 0) {
                const Real a = cell(f, i, 0), b = cell(f, i, 1);
                for (int gg = 1; gg <= reach; ++gg) cell(f, i, -gg) = ghost_value(f, gg | (SIDE_OTHER << 2), a, b, c, c.t_hot);
            }
            if (j0 + TJ + reach > d.nj) {
                const Real a = cell(f, i, d.nj - 1), b = cell(f, i, d.nj - 2);
                for (int gg = 1; gg <= reach; ++gg)
                    if (d.nj - 1 + gg < j0 + TJ + reach)
                        cell(f, i, d.nj - 1 + gg) = ghost_value(f, gg | (SIDE_OTHER << 2), a, b, c, c.t_hot);
            }
        }
        // x walls: row j0 + row, field `lane`
        if (lane < NF && j < d.nj) {
            const int f = lane, reach = f == FP ? 2 : 1;
            if (i0 == 0) {
                const Real a = cell(f, 0, j), b = cell(f, 1, j);
                const Real tlo = hot_wall(c, d, j, k);
                for (int gg = 1; gg <= reach; ++gg) cell(f, -gg, j) = ghost_value(f, gg | (SIDE_X_LO << 2), a, b, c, tlo);
            }
            if (i0 + TI + reach > d.ni) {
                const Real a = cell(f, d.ni - 1, j), b = cell(f, d.ni - 2, j);
                for (int gg = 1; gg <= reach; ++gg)
                    if (d.ni - 1 + gg < i0 + TI + reach)
                        cell(f, d.ni - 1 + gg, j) = ghost_value(f, gg | (SIDE_X_HI << 2), a, b, c, c.t_hot);
            }
        }
    };

    // ---- register queues ----
    Real p0, p1, p2, p3;                                 // p at k-2, k-1, k, k+1
    Real u0, u1, v0, v1, w0, w1, t0, t1;                 // at k-1, k
    const int lc_p = (row + 2) * PW + lane + 2;            // this cell in an LDS p plane
    const int lc_u = (row + 1) * UW + lane + 1;            // this cell in an LDS u v w T plane
    {
        // planes k0-2 .. k0+1 of this column; planes beyond the z walls
        // follow from the wall rules (recurrences along k)
        Real P[4], U[2], V[2], W[2], T[2];
        for (int m = 0; m < 4; ++m) {
            const int kk = k0 - 2 + m;
            P[m] = (active && kk >= 0 && kk < d.nk) ? Pg[off_c + kk * Z] : Real(0);
        }
        for (int m = 0; m < 2; ++m) {
            const int kk = k0 - 1 + m;
            const bool in = active && kk >= 0;
            U[m] = in ? Ug[off_c + kk * Z] : Real(0);
            V[m] = in ? Vg[off_c + kk * Z] : Real(0);
            W[m] = in ? Wg[off_c + kk * Z] : Real(0);
            T[m] = in ? Tg[off_c + kk * Z] : Real(0);
        }
        if (k0 + 1 >= d.nk) P[3] = Real(2) * P[2] - P[1];
        for (int m = 1; m >= 0; --m)
            if (k0 - 2 + m < 0) P[m] = Real(2) * P[m + 1] - P[m + 2];
        if (k0 - 1 < 0) { U[0] = -U[1]; V[0] = -V[1]; W[0] = -W[1]; T[0] = T[1]; }
        p0 = P[0]; p1 = P[1]; p2 = P[2]; p3 = P[3];
        u0 = U[0]; u1 = U[1]; v0 = V[0]; v1 = V[1]; w0 = W[0]; w1 = W[1]; t0 = T[0]; t1 = T[1];
    }
    // plane k0 into LDS buffer 0
    sP[lc_p] = p2;
    sU[0 * UPL + lc_u] = u1;
    sU[1 * UPL + lc_u] = v1;
    sU[2 * UPL + lc_u] = w1;
    sU[3 * UPL + lc_u] = t1;
    if (has_prow) sP[prow_dst] = ld_prow ? Pg[off_prow + k0 * Z] : Real(0);
#pragma unroll
    for (int r = 0; r < UR; ++r)
        if (has_urow[r]) sU[urow_dst[r]] = ld_urow[r] ? URg[r][off_urow[r] + k0 * Z] : Real(0);
    if (has_col) (col_f == FP ? sP : sU)[col_lds] = ld_col ? COLg[off_col + k0 * Z] : Real(0);

    // Loads run DEPTH planes ahead: what the iteration for plane k needs
    // from memory (queue heads p(k+2), uvwT(k+1), halo strips of plane k+1)
    // is issued while plane k-DEPTH is computed; DEPTH register sets rotate
    // (3 for the step kernels; 2 where the epilogue needs the registers).
    struct InFlight {
        Real p, u, v, w, t, prow, urow[UR], col;
    };
    auto issue = [&](InFlight& F, int k) __attribute__((always_inline)) {
        if (active) {
            if (k + 2 < d.nk) F.p = Pg[off_c + (k + 2) * Z];
            if (k + 1 < d.nk) {
                F.u = Ug[off_c + (k + 1) * Z];
                F.v = Vg[off_c + (k + 1) * Z];
                F.w = Wg[off_c + (k + 1) * Z];
                F.t = Tg[off_c + (k + 1) * Z];
            }
        }
        if (k + 1 < k1) {
            if (ld_prow) F.prow = Pg[off_prow + (k + 1) * Z];
#pragma unroll
            for (int r = 0; r < UR; ++r)
                if (ld_urow[r]) F.urow[r] = URg[r][off_urow[r] + (k + 1) * Z];
            if (ld_col) F.col = COLg[off_col + (k + 1) * Z];
        }
    };
    static_assert(DEPTH == 2 || DEPTH == 3, "prefetch depth is 2 or 3 planes");
    InFlight X{}, Y{}, Zs{};
    issue(X, k0);
    if (k0 + 1 < k1) issue(Y, k0 + 1);
    if constexpr (DEPTH == 3)
        if (k0 + 2 < k1) issue(Zs, k0 + 2);
    // the epilogue's per-block setup (for the step: the centre cell's new
    // pressure, a star gathered from L2) overlaps the loads in flight
    epi.prepare(d, q, c);
    __syncthreads();

    double acc[NF] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int buf = 0;

    auto plane = [&](InFlight& F, int k) __attribute__((always_inline)) {
        // complete the queues; planes past the top wall follow the wall rules
        const Real p4 = k + 2 < d.nk ? F.p : Real(2) * p3 - p2;
        const bool in1 = k + 1 < d.nk;
        const Real u2 = in1 ? F.u : -u1, v2 = in1 ? F.v : -v1, w2 = in1 ? F.w : -w1, t2 = in1 ? F.t : t1;
        if (k + 1 < k1) {
            // plane k+1 into the other LDS buffer (its last readers finished
            // before the barrier that ended the previous plane)
            Real* const nP = sP + (buf ^ 1) * PPL;
            Real* const nU = sU + (buf ^ 1) * 4 * UPL;
            nP[lc_p] = p3;
            nU[0 * UPL + lc_u] = u2;
            nU[1 * UPL + lc_u] = v2;
            nU[2 * UPL + lc_u] = w2;
            nU[3 * UPL + lc_u] = t2;
            if (has_prow) nP[prow_dst] = F.prow;
#pragma unroll
            for (int r = 0; r < UR; ++r)
                if (has_urow[r]) nU[urow_dst[r]] = F.urow[r];
            if (has_col) (col_f == FP ? nP : nU)[col_lds] = F.col;
        }
        if (k + DEPTH < k1) issue(F, k + DEPTH);

        Real* const cP = sP + buf * PPL;
        Real* const cU = sU + buf * 4 * UPL;
        if (bnd) {
            fix_ghosts(cP, cU, k);
            __syncthreads();
        }
        if (active && own(i, j, k)) {
            Star<Real> s;
            s.p = p2;
            s.pxm = cP[lc_p - 1]; s.pxp = cP[lc_p + 1]; s.pxm2 = cP[lc_p - 2]; s.pxp2 = cP[lc_p + 2];
            s.pym = cP[lc_p - PW]; s.pyp = cP[lc_p + PW]; s.pym2 = cP[lc_p - 2 * PW]; s.pyp2 = cP[lc_p + 2 * PW];
            s.pzm = p1; s.pzp = p3; s.pzm2 = p0; s.pzp2 = p4;
#define STAR_LDS(nm, pl, c0, cm, cp)                                               \
            s.nm = c0; s.nm##zm = cm; s.nm##zp = cp;                               \
            s.nm##xm = cU[pl * UPL + lc_u - 1]; s.nm##xp = cU[pl * UPL + lc_u + 1]; \
            s.nm##ym = cU[pl * UPL + lc_u - UW]; s.nm##yp = cU[pl * UPL + lc_u + UW];
            STAR_LDS(u, 0, u1, u0, u2)
            STAR_LDS(v, 1, v1, v0, v2)
            STAR_LDS(w, 2, w1, w0, w2)
            STAR_LDS(t, 3, t1, t0, t2)
#undef STAR_LDS
            Real R[NF], dt;
            cell_residual(c, s, R, dt);
            epi.cell(c, s, R, dt, off_c + k * Z, i, j, k, acc);
        }
        __syncthreads();
        buf ^= 1;
        p0 = p1; p1 = p2; p2 = p3; p3 = p4;
        u0 = u1; u1 = u2; v0 = v1; v1 = v2; w0 = w1; w1 = w2; t0 = t1; t1 = t2;
    };

    for (int k = k0; k < k1; k += DEPTH) {
        plane(X, k);
        if (k + 1 < k1) plane(Y, k + 1);
        if constexpr (DEPTH == 3)
            if (k + 2 < k1) plane(Zs, k + 2);
    }

    if (NORM) {
        // fixed-order block reduction: butterfly within the wavefront, then
        // the wavefront sums in order
        auto& red = L.red;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            double v = acc[f];
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
            acc[f] = v;
        }
        const int wl = tid & 63, wv = tid >> 6;
        if (wl == 0) {
#pragma unroll
            for (int f = 0; f < NF; ++f) red[wv][f] = acc[f];
        }
        __syncthreads();
        if (tid < NF) {
            double t = 0.0;
#pragma unroll
            for (int r = 0; r < Lds::NWAVE; ++r) t += red[r][tid];
            partials[(size_t)tb.pidx * NF + tid] = t;
        }
    }
}

}  // namespace cav
