// Residual + Euler-update sweep, wall boundary conditions, seeded init and
// the residual-norm finalize for gfx950 (FP64).
//
// The method (Xue & Roy, arXiv:2006.02602): artificial-compressibility
// Boussinesq equations (Sec. 2, Eq. 1-3), second-order central differences
// with a fourth-difference pressure dissipation (5-point p stencil, 3-point
// stencils for u, v, w, T; Sec. 3.1), first-order explicit Euler in pseudo
// time, wall boundary conditions and the pressure rescale at the cavity
// centre in every iteration (Sec. 2).
//
// This file is compiled with -ffp-contract=off: every fused multiply-add is
// written out with fma(), so two inlined copies of the per-cell update round
// identically (the centre-cell rescale relies on that).
#include "cavity_internal.h"
#include "stencil.h"

namespace cav {

// ---------------------------------------------------------------------------
// The sweep.  Block = one 64 x 8 tile of (i, j) columns (one wavefront per
// j row, i along the lanes) marching over a chunk of k planes.  Plane k of
// all five fields lives in LDS with its i/j halo (2 for p, 1 for the rest);
// the k neighbours come from per-thread register queues (p: k-2..k+2,
// others k-1..k+1).  The LDS planes are Real-buffered: plane k+1 is
// written into one buffer while plane k is computed from the other, so each
// plane costs one barrier; global loads run two planes ahead.
// Wall ghosts are derived while loading (Slot), never read from HBM.
// LDS of one sweep block: two double-buffered planes of p (halo 2) and of
// u, v, w, T (halo 1).
template <typename Real>
struct SweepLds {
    static constexpr int TI = SW_TI, TJ = SW_TJ;
    static constexpr int PW = TI + 4;              // row pitch, p
    static constexpr int UW = TI + 2;              // row pitch, u v w T
    static constexpr int PPL = (TJ + 4) * PW;      // plane, p
    static constexpr int UPL = (TJ + 2) * UW;      // plane, one of u v w T
    Real p[2 * PPL];
    Real u[2 * 4 * UPL];
    double red[TJ][NF];
};

// Where one block works: columns [i0, i0+64) x [j0, j0+8), planes
// [k0, k1); its norm partial goes to slot pidx.
struct TileBox {
    int i0, j0, k0, k1, pidx;
};

// Logical tile b of the regular tiling with k chunks of length kc.
__device__ __forceinline__ TileBox tile_box(const Dims& d, int tiles_i, int tiles_j, int kc, int b)
{
    const int bi = b % tiles_i;
    const int bj = (b / tiles_i) % tiles_j;
    const int bk = b / (tiles_i * tiles_j);
    TileBox t;
    t.i0 = bi * SW_TI;
    t.j0 = bj * SW_TJ;
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
// batched kernel and the interior/exterior split.
template <typename Real, bool NORM, typename Own>
__device__ __forceinline__ void sweep_tile(const Dims& d, const CoefR<Real>& c, const TileBox& tb, const Own& own,
                                           const CStateT<Real>& q, const StateT<Real>& qn, double* partials,
                                           SweepLds<Real>& L)
{
    constexpr int TI = SW_TI, TJ = SW_TJ;
    constexpr int PW = SweepLds<Real>::PW, UW = SweepLds<Real>::UW;
    constexpr int PPL = SweepLds<Real>::PPL, UPL = SweepLds<Real>::UPL;
    Real* const sP = L.p;
    Real* const sU = L.u;

    const int i0 = tb.i0, j0 = tb.j0;
    const int k0 = tb.k0, k1 = tb.k1;

    const int lane = threadIdx.x, row = threadIdx.y;
    const int i = i0 + lane, j = j0 + row;
    // columns no owned cell's star reaches are neither loaded nor computed
    const bool active = i < d.ni && j < d.nj && own.column(i, j);

    // New pressure at the centre cell, recomputed with the same arithmetic
    // as its owner, so that every block subtracts the identical value.
    Real pc_new;
    {
        Star<Real> s;
        gather_global(d, q, c, d.ni / 2, d.nj / 2, d.nk / 2, s);
        Real R[NF], dt;
        cell_residual(c, s, R, dt);
        pc_new = fma(dt, R[FP], s.p);
    }

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
    // u v w T rows j0-1, j0+TJ: waves 0..7, field 1 + row/2
    const int urow_f = FU + (row >> 1);
    const int urow_lds = (row & 1) ? TJ + 1 : 0;
    const int urow_j = j0 - 1 + urow_lds;
    const bool ld_urow = interior(i, urow_j) && own.column(i, urow_j);
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
    const int urow_dst = (urow_f - FU) * UPL + urow_lds * UW + lane + 1;
    const int off_c = cell_off(d, i, j, 0);
    const int off_prow = cell_off(d, i, prow_j, 0);
    const int off_urow = cell_off(d, i, urow_j, 0);
    const int off_col = cell_off(d, col_i, j, 0);
    const Real* const Pg = q.f[FP];
    const Real* const Ug = q.f[FU];
    const Real* const Vg = q.f[FV];
    const Real* const Wg = q.f[FW];
    const Real* const Tg = q.f[FT];
    const Real* const URg = q.f[urow_f];
    const Real* const COLg = q.f[col_f];
    const int Z = d.sz;

    // tiles whose LDS planes reach past a wall fix their ghost cells
    const bool bnd = i0 == 0 || j0 == 0 || i0 + TI + 2 > d.ni || j0 + TJ + 2 > d.nj;
    auto fix_ghosts = [&](Real* fP, Real* fU, int k) __attribute__((always_inline)) {
        auto cell = [&](int f, int ci, int cj) -> Real& {
            return f == FP ? fP[(cj - j0 + 2) * PW + (ci - i0 + 2)]
                           : fU[(f - FU) * UPL + (cj - j0 + 1) * UW + (ci - i0 + 1)];
        };
        // y walls: column i0 + lane, field `row`
        if (row < NF && i < d.ni) {
            const int f = row, reach = f == FP ? 2 : 1;
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
    sU[urow_dst] = ld_urow ? URg[off_urow + k0 * Z] : Real(0);
    if (has_col) (col_f == FP ? sP : sU)[col_lds] = ld_col ? COLg[off_col + k0 * Z] : Real(0);

    // Loads run two planes ahead: what the iteration for plane k needs from
    // memory (queue heads p(k+2), uvwT(k+1), halo strips of plane k+1) is
    // issued while plane k-2 is computed.  Two register sets alternate.
    struct InFlight {
        Real p, u, v, w, t, prow, urow, col;
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
            if (ld_urow) F.urow = URg[off_urow + (k + 1) * Z];
            if (ld_col) F.col = COLg[off_col + (k + 1) * Z];
        }
    };
    InFlight X{0, 0, 0, 0, 0, 0, 0, 0}, Y{0, 0, 0, 0, 0, 0, 0, 0};
    issue(X, k0);
    if (k0 + 1 < k1) issue(Y, k0 + 1);
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
            nU[urow_dst] = F.urow;
            if (has_col) (col_f == FP ? nP : nU)[col_lds] = F.col;
        }
        if (k + 2 < k1) issue(F, k + 2);

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
            // the new state is not read again by this launch: stream it out
            const int o = off_c + k * Z;
            __builtin_nontemporal_store(fma(dt, R[FP], s.p) - pc_new, &qn.f[FP][o]);
            __builtin_nontemporal_store(fma(dt, R[FU], s.u), &qn.f[FU][o]);
            __builtin_nontemporal_store(fma(dt, R[FV], s.v), &qn.f[FV][o]);
            __builtin_nontemporal_store(fma(dt, R[FW], s.w), &qn.f[FW][o]);
            __builtin_nontemporal_store(fma(dt, R[FT], s.t), &qn.f[FT][o]);
            if (NORM) {
#pragma unroll
                for (int f = 0; f < NF; ++f) acc[f] = fma((double)R[f], (double)R[f], acc[f]);
            }
        }
        __syncthreads();
        buf ^= 1;
        p0 = p1; p1 = p2; p2 = p3; p3 = p4;
        u0 = u1; u1 = u2; v0 = v1; v1 = v2; w0 = w1; w1 = w2; t0 = t1; t1 = t2;
    };

    for (int k = k0; k < k1; k += 2) {
        plane(X, k);
        if (k + 1 < k1) plane(Y, k + 1);
    }

    if (NORM) {
        // fixed-order block reduction: butterfly within the wavefront, then
        // the 8 wavefront sums in order
        auto& red = L.red;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            double v = acc[f];
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
            acc[f] = v;
        }
        if (lane == 0) {
#pragma unroll
            for (int f = 0; f < NF; ++f) red[row][f] = acc[f];
        }
        __syncthreads();
        if (row == 0 && lane < NF) {
            double t = 0.0;
#pragma unroll
            for (int r = 0; r < TJ; ++r) t += red[r][lane];
            partials[(size_t)tb.pidx * NF + lane] = t;
        }
    }
}

// FIELD = false: the hot wall is the scalar t_hot, known at compile time to
// need no field loads (the kernel the uniform-wall problem runs).
template <typename Real, bool NORM, bool FIELD>
__global__ __launch_bounds__(SW_TI * SW_TJ) void sweep_kernel(Dims d, Coef cd, SweepGeom g, CStateT<Real> q,
                                                              StateT<Real> qn, double* partials)
{
    __shared__ SweepLds<Real> L;
    CoefR<Real> c = coef_as<Real>(cd);
    if constexpr (!FIELD) c.t_hot_field = nullptr;
    const TileBox tb = tile_box(d, g.tiles_i, g.tiles_j, g.kc, xcd_block(blockIdx.x, g.nblocks));
    sweep_tile<Real, NORM>(d, c, tb, OwnAll{}, q, qn, partials, L);
}

SweepGeom sweep_geom(const Dims& d, int slots)
{
    SweepGeom g;
    g.tiles_i = (d.ni + SW_TI - 1) / SW_TI;
    g.tiles_j = (d.nj + SW_TJ - 1) / SW_TJ;
    const int tiles = g.tiles_i * g.tiles_j;
    // Split the k columns into nkc chunks so that the launch finishes
    // earliest: blocks run in rounds of `slots` (one resident block per
    // compute unit), a block costs its planes plus ~3 planes of start-up
    // (the queue and halo planes it loads before its first plane).
    const int overhead = 3;
    long long best_cost = -1;
    int best = 1;
    const int max_nkc = max(1, d.nk / 4);
    for (int nkc = 1; nkc <= max_nkc; ++nkc) {
        const int kc = (d.nk + nkc - 1) / nkc;
        const long long blocks = (long long)tiles * ((d.nk + kc - 1) / kc);
        const long long rounds = (blocks + slots - 1) / slots;
        const long long cost = rounds * (kc + overhead);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = nkc;
        }
    }
    g.kc = (d.nk + best - 1) / best;
    g.nkc = (d.nk + g.kc - 1) / g.kc;
    g.nblocks = tiles * g.nkc;
    return g;
}

template <typename Real>
hipError_t launch_sweep(const Dims& d, const Coef& c, const SweepGeom& g, CStateT<Real> q, StateT<Real> qn,
                        double* partials, bool with_norm, hipStream_t s)
{
    dim3 block(SW_TI, SW_TJ), grid(g.nblocks);
    if (c.t_hot_field) {
        if (with_norm)
            sweep_kernel<Real, true, true><<<grid, block, 0, s>>>(d, c, g, q, qn, partials);
        else
            sweep_kernel<Real, false, true><<<grid, block, 0, s>>>(d, c, g, q, qn, partials);
    } else {
        if (with_norm)
            sweep_kernel<Real, true, false><<<grid, block, 0, s>>>(d, c, g, q, qn, partials);
        else
            sweep_kernel<Real, false, false><<<grid, block, 0, s>>>(d, c, g, q, qn, partials);
    }
    return hipGetLastError();
}
template hipError_t launch_sweep<double>(const Dims&, const Coef&, const SweepGeom&, CStateT<double>,
                                         StateT<double>, double*, bool, hipStream_t);
template hipError_t launch_sweep<float>(const Dims&, const Coef&, const SweepGeom&, CStateT<float>,
                                        StateT<float>, double*, bool, hipStream_t);

// ---------------------------------------------------------------------------
// Interior/exterior split (Sec. 4.7): with a halo exchange in the step, the
// cells whose stars reach no cell the unpack writes (the interior) are
// updated by one launch that may run while the exchange is in flight; the
// rest (the exterior: cells within `m` of a cut) by a second launch after
// it.  Each cell is computed by exactly one launch with the same per-cell
// code as the unsplit sweep, so the new state is bit-identical to it.

// Cell x along `axis` lies within m of a cut between two subdomains.
__device__ __forceinline__ bool near_cut(const SplitGeom& sg, int axis, int x)
{
    const int e = sg.e[axis];
    const int a = x / e, local = x - a * e;
    return (a > 0 && local < sg.m) || (a < sg.P[axis] - 1 && local >= e - sg.m);
}

struct OwnInterior {
    SplitGeom sg;
    __device__ __forceinline__ bool operator()(int i, int j, int k) const
    {
        return !(near_cut(sg, 0, i) || near_cut(sg, 1, j) || near_cut(sg, 2, k));
    }
    __device__ __forceinline__ bool column(int, int) const { return true; }
};

// The slab [cut - m, cut + m) along `axis`; cells also near a cut of a lower
// axis belong to that axis's slab.
struct OwnSlab {
    SplitGeom sg;
    int axis, cut;
    __device__ __forceinline__ bool operator()(int i, int j, int k) const
    {
        const int x = axis == 0 ? i : (axis == 1 ? j : k);
        if (x < cut - sg.m || x >= cut + sg.m) return false;
        if (axis >= 1 && near_cut(sg, 0, i)) return false;
        if (axis == 2 && near_cut(sg, 1, j)) return false;
        return true;
    }
    // an x slab's cells read columns up to 2 cells beyond it
    __device__ __forceinline__ bool column(int i, int) const
    {
        return axis != 0 || (i >= cut - sg.m - 2 && i < cut + sg.m + 2);
    }
};

template <typename Real, bool NORM, bool FIELD>
__global__ __launch_bounds__(SW_TI * SW_TJ) void interior_kernel(Dims d, Coef cd, SweepGeom g, SplitGeom sg,
                                                                 CStateT<Real> q, StateT<Real> qn,
                                                                 double* partials)
{
    __shared__ SweepLds<Real> L;
    CoefR<Real> c = coef_as<Real>(cd);
    if constexpr (!FIELD) c.t_hot_field = nullptr;
    const TileBox tb = tile_box(d, g.tiles_i, g.tiles_j, g.kc, xcd_block(blockIdx.x, g.nblocks));
    sweep_tile<Real, NORM>(d, c, tb, OwnInterior{sg}, q, qn, partials, L);
}

// Exterior work items, block b: first the x slabs (per cut: j tiles x k
// chunks of kce planes), then the y slabs (per cut: i tiles x k chunks),
// then the z slabs (per cut: i x j tiles, the 2m planes around the cut).
// Norm partials follow the interior launch's, at pidx = nblocks + b.
template <typename Real, bool NORM, bool FIELD>
__global__ __launch_bounds__(SW_TI * SW_TJ) void exterior_kernel(Dims d, Coef cd, SweepGeom g, SplitGeom sg,
                                                                 CStateT<Real> q, StateT<Real> qn,
                                                                 double* partials)
{
    __shared__ SweepLds<Real> L;
    CoefR<Real> c = coef_as<Real>(cd);
    if constexpr (!FIELD) c.t_hot_field = nullptr;
    const int b = blockIdx.x;
    const int nkce = (d.nk + sg.kce - 1) / sg.kce;
    const int per0 = g.tiles_j * nkce, per1 = g.tiles_i * nkce, per2 = g.tiles_i * g.tiles_j;
    const int n0 = (sg.P[0] - 1) * per0, n1 = (sg.P[1] - 1) * per1;
    TileBox tb;
    int axis, cut;
    if (b < n0) {
        axis = 0;
        const int r = b % per0;
        cut = (b / per0 + 1) * sg.e[0];
        tb.i0 = cut - sg.m;
        tb.j0 = (r % g.tiles_j) * SW_TJ;
        tb.k0 = (r / g.tiles_j) * sg.kce;
        tb.k1 = min(tb.k0 + sg.kce, d.nk);
    } else if (b < n0 + n1) {
        axis = 1;
        const int r = (b - n0) % per1;
        cut = ((b - n0) / per1 + 1) * sg.e[1];
        tb.i0 = (r % g.tiles_i) * SW_TI;
        tb.j0 = cut - sg.m;
        tb.k0 = (r / g.tiles_i) * sg.kce;
        tb.k1 = min(tb.k0 + sg.kce, d.nk);
    } else {
        axis = 2;
        const int r = (b - n0 - n1) % per2;
        cut = ((b - n0 - n1) / per2 + 1) * sg.e[2];
        tb.i0 = (r % g.tiles_i) * SW_TI;
        tb.j0 = (r / g.tiles_i) * SW_TJ;
        tb.k0 = cut - sg.m;
        tb.k1 = cut + sg.m;
    }
    tb.pidx = g.nblocks + b;
    sweep_tile<Real, NORM>(d, c, tb, OwnSlab{sg, axis, cut}, q, qn, partials, L);
}

int exterior_blocks(const Dims& d, const SweepGeom& g, const SplitGeom& sg)
{
    const int nkce = (d.nk + sg.kce - 1) / sg.kce;
    return (sg.P[0] - 1) * g.tiles_j * nkce + (sg.P[1] - 1) * g.tiles_i * nkce +
           (sg.P[2] - 1) * g.tiles_i * g.tiles_j;
}

template <typename Real>
hipError_t launch_split(const Dims& d, const Coef& c, const SweepGeom& g, const SplitGeom& sg, bool exterior,
                        CStateT<Real> q, StateT<Real> qn, double* partials, bool with_norm, hipStream_t s)
{
    dim3 block(SW_TI, SW_TJ);
    const int nb = exterior ? exterior_blocks(d, g, sg) : g.nblocks;
    if (nb == 0) return hipSuccess;
    const bool fld = c.t_hot_field != nullptr;
#define SPLIT_LAUNCH(K)                                                                                  \
    do {                                                                                                 \
        if (fld) {                                                                                       \
            if (with_norm) K<Real, true, true><<<nb, block, 0, s>>>(d, c, g, sg, q, qn, partials);        \
            else K<Real, false, true><<<nb, block, 0, s>>>(d, c, g, sg, q, qn, partials);                 \
        } else {                                                                                         \
            if (with_norm) K<Real, true, false><<<nb, block, 0, s>>>(d, c, g, sg, q, qn, partials);       \
            else K<Real, false, false><<<nb, block, 0, s>>>(d, c, g, sg, q, qn, partials);                \
        }                                                                                                \
    } while (0)
    if (exterior)
        SPLIT_LAUNCH(exterior_kernel);
    else
        SPLIT_LAUNCH(interior_kernel);
#undef SPLIT_LAUNCH
    return hipGetLastError();
}
template hipError_t launch_split<double>(const Dims&, const Coef&, const SweepGeom&, const SplitGeom&, bool,
                                         CStateT<double>, StateT<double>, double*, bool, hipStream_t);
template hipError_t launch_split<float>(const Dims&, const Coef&, const SweepGeom&, const SplitGeom&, bool,
                                        CStateT<float>, StateT<float>, double*, bool, hipStream_t);

// ---------------------------------------------------------------------------
// Batched form: a persistent grid walks the work list of all members; each
// item is one tile column's k chunk of one member, computed by the same
// sweep_tile as the single-cavity sweep.  `parity` selects which of q and
// q_tmp holds the current state of every member.
template <typename Real, bool NORM>
__global__ __launch_bounds__(SW_TI * SW_TJ) void batch_kernel(const BatchCav* __restrict__ cavs,
                                                              const BatchItem* __restrict__ items, int nitems,
                                                              int parity)
{
    __shared__ SweepLds<Real> L;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BatchItem w = items[it];
        const BatchCav& cv = cavs[w.cav];
        const Dims d = cv.d;
        const CoefR<Real> c = coef_as<Real>(cv.c);
        const Real* cur = static_cast<const Real*>(parity ? cv.q_tmp : cv.q);
        Real* nxt = static_cast<Real*>(parity ? cv.q : cv.q_tmp);
        CStateT<Real> qs;
        StateT<Real> qn;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            qs.f[f] = cur + f * cv.fstride;
            qn.f[f] = nxt + f * cv.fstride;
        }
        const TileBox tb = tile_box(d, cv.tiles_i, cv.tiles_j, cv.kc, w.tile);
        sweep_tile<Real, NORM>(d, c, tb, OwnAll{}, qs, qn, cv.ws + WS_HEAD_DOUBLES, L);
        __syncthreads();                  // LDS is reused by the next item
    }
}

template <typename Real>
hipError_t launch_batch(const BatchCav* cavs, const BatchItem* items, int nitems, int parity, bool with_norm,
                        int nblocks, hipStream_t s)
{
    dim3 block(SW_TI, SW_TJ), grid(nblocks);
    if (with_norm)
        batch_kernel<Real, true><<<grid, block, 0, s>>>(cavs, items, nitems, parity);
    else
        batch_kernel<Real, false><<<grid, block, 0, s>>>(cavs, items, nitems, parity);
    return hipGetLastError();
}
template hipError_t launch_batch<double>(const BatchCav*, const BatchItem*, int, int, bool, int, hipStream_t);
template hipError_t launch_batch<float>(const BatchCav*, const BatchItem*, int, int, bool, int, hipStream_t);

// Residual norms of every member: one block per member, the same
// fixed-order reduction as the single-cavity finalize.
__global__ __launch_bounds__(256) void batch_norm_kernel(const BatchCav* __restrict__ cavs)
{
    __shared__ double red[NF][256];
    const BatchCav& cv = cavs[blockIdx.x];
    const double* part = cv.ws + WS_HEAD_DOUBLES;
    const int t = threadIdx.x;
    for (int f = 0; f < NF; ++f) {
        double s = 0.0;
        for (int b = t; b < cv.ntiles; b += 256) s += part[(size_t)b * NF + f];
        red[f][t] = s;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int f = 0; f < NF; ++f) red[f][t] += red[f][t + w];
        __syncthreads();
    }
    const double ncell = (double)cv.d.ni * cv.d.nj * cv.d.nk;
    if (t < NF) cv.ws[t] = sqrt(red[t][0] / ncell);
}

hipError_t launch_batch_norms(const BatchCav* cavs, int members, hipStream_t s)
{
    batch_norm_kernel<<<members, 256, 0, s>>>(cavs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Wall ghost layers (Sec. 2), written into the state by cavity_init: one
// thread per wall-adjacent line of cells, all five fields, both layers.
template <typename Real>
__global__ __launch_bounds__(256) void bc_kernel(Dims d, Bcs bc, StateT<Real> q)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nx = 2LL * d.nj * d.nk, ny = 2LL * d.ni * d.nk, nz = 2LL * d.ni * d.nj;
    int o, s, axis;
    bool high;
    double tw_lo = bc.t_hot;
    if (t < nx) {                                   // x walls: (j, k, side), j fastest
        axis = 0;
        const int j = (int)(t % d.nj);
        const long long r = t / d.nj;
        const int k = (int)(r % d.nk);
        high = r >= d.nk;
        if (bc.t_hot_field) tw_lo = bc.t_hot_field[j + (long long)d.nj * k];
        o = cell_off(d, high ? d.ni - 1 : 0, j, k);
        s = high ? -1 : 1;
    } else if (t < nx + ny) {                       // y walls: (i, k, side), i fastest
        axis = 1;
        const long long u = t - nx;
        const int i = (int)(u % d.ni);
        const long long r = u / d.ni;
        const int k = (int)(r % d.nk);
        high = r >= d.nk;
        o = cell_off(d, i, high ? d.nj - 1 : 0, k);
        s = high ? -d.sy : d.sy;
    } else if (t < nx + ny + nz) {                  // z walls: (i, j, side), i fastest
        axis = 2;
        const long long u = t - nx - ny;
        const int i = (int)(u % d.ni);
        const long long r = u / d.ni;
        const int j = (int)(r % d.nj);
        high = r >= d.nj;
        o = cell_off(d, i, j, high ? d.nk - 1 : 0);
        s = high ? -d.sz : d.sz;
    } else {
        return;
    }
    // p: one-sided linear extrapolation, second order
    {
        Real* A = q.f[FP];
        const Real a = A[o], b = A[o + s];
        const Real g1 = Real(2) * a - b;
        A[o - s] = g1;
        A[o - 2 * s] = Real(2) * g1 - a;
    }
    // u, v, w: no-slip (odd reflection)
#pragma unroll
    for (int f = FU; f <= FW; ++f) {
        Real* A = q.f[f];
        const Real a = A[o], b = A[o + s];
        A[o - s] = -a;
        A[o - 2 * s] = -b;
    }
    // T: fixed value on the hot/cold walls, zero gradient elsewhere
    {
        Real* A = q.f[FT];
        const Real a = A[o], b = A[o + s];
        if (axis == 0) {
            const Real tw = (Real)(high ? bc.t_cold : tw_lo);
            A[o - s] = Real(2) * tw - a;
            A[o - 2 * s] = Real(2) * tw - b;
        } else {
            A[o - s] = a;
            A[o - 2 * s] = b;
        }
    }
}

template <typename Real>
hipError_t launch_bc(const Dims& d, const Bcs& b, StateT<Real> q, hipStream_t s)
{
    const long long n = 2LL * ((long long)d.nj * d.nk + (long long)d.ni * d.nk + (long long)d.ni * d.nj);
    bc_kernel<Real><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(d, b, q);
    return hipGetLastError();
}
template hipError_t launch_bc<double>(const Dims&, const Bcs&, StateT<double>, hipStream_t);
template hipError_t launch_bc<float>(const Dims&, const Bcs&, StateT<float>, hipStream_t);

// ---------------------------------------------------------------------------
// Seeded initial state: SplitMix64 (Steele, Lea & Flood 2014), output number
// f*2^40 + idx of the stream seeded with `seed`.  Computed in FP64; an FP32
// state stores the rounded values.
__device__ __forceinline__ double noise(uint64_t seed, int f, uint64_t idx, double amp)
{
    uint64_t z = seed + ((((uint64_t)f) << 40) + idx + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    const double r = (double)(z >> 11) * 0x1.0p-53;
    return (2.0 * r - 1.0) * amp;
}

template <typename Real>
__global__ __launch_bounds__(256) void init_kernel(Dims d, double t_hot, double t_cold, uint64_t seed,
                                                   double amp, StateT<Real> q)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)d.ni * d.nj * d.nk) return;
    const int i = (int)(idx % d.ni);
    const long long r = idx / d.ni;
    const int j = (int)(r % d.nj);
    const int k = (int)(r / d.nj);
    const int o = cell_off(d, i, j, k);
    const double xc = ((double)i + 0.5) / (double)d.ni;
    q.f[FP][o] = (Real)0.0;
    q.f[FU][o] = (Real)noise(seed, 1, (uint64_t)idx, amp);
    q.f[FV][o] = (Real)noise(seed, 2, (uint64_t)idx, amp);
    q.f[FW][o] = (Real)noise(seed, 3, (uint64_t)idx, amp);
    q.f[FT][o] = (Real)((t_hot + (t_cold - t_hot) * xc) + noise(seed, 4, (uint64_t)idx, amp));
}

template <typename Real>
hipError_t launch_init(const Dims& d, double t_hot, double t_cold, uint64_t seed, double amp, StateT<Real> q,
                       hipStream_t s)
{
    const long long n = (long long)d.ni * d.nj * d.nk;
    init_kernel<Real><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(d, t_hot, t_cold, seed, amp, q);
    return hipGetLastError();
}
template hipError_t launch_init<double>(const Dims&, double, double, uint64_t, double, StateT<double>, hipStream_t);
template hipError_t launch_init<float>(const Dims&, double, double, uint64_t, double, StateT<float>, hipStream_t);

// ---------------------------------------------------------------------------
// Mean Nusselt number of the hot wall x = 0 in FP64: -dT/dx at the wall from
// the second-order one-sided difference (9 T_0 - T_1 - 8 T_w) / (3h) through
// the wall value and the first two cell centres, averaged over the wall and
// divided by t_hot - t_cold.  The wall value is the hot-wall field where one
// is given.  One block; fixed-order reduction.
template <typename Real>
__global__ __launch_bounds__(1024) void nusselt_kernel(Dims d, Bcs bc, CStateT<Real> q, double* out)
{
    __shared__ double red[1024];
    const int t = threadIdx.x;
    const long long n = (long long)d.nj * d.nk;
    const double three_h = 3.0 / (double)d.ni;
    double acc = 0.0;
    for (long long e = t; e < n; e += 1024) {
        const int j = (int)(e % d.nj), k = (int)(e / d.nj);
        const int o = cell_off(d, 0, j, k);
        const double t0 = (double)q.f[FT][o], t1 = (double)q.f[FT][o + 1];
        const double tw = bc.t_hot_field ? bc.t_hot_field[e] : bc.t_hot;
        acc += -((9.0 * t0 - t1 - 8.0 * tw) / three_h);
    }
    red[t] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[0] = red[0] / ((double)d.nj * (double)d.nk) / (bc.t_hot - bc.t_cold);
}

template <typename Real>
hipError_t launch_nusselt(const Dims& d, const Bcs& b, CStateT<Real> q, double* out, hipStream_t s)
{
    nusselt_kernel<Real><<<1, 1024, 0, s>>>(d, b, q, out);
    return hipGetLastError();
}
template hipError_t launch_nusselt<double>(const Dims&, const Bcs&, CStateT<double>, double*, hipStream_t);
template hipError_t launch_nusselt<float>(const Dims&, const Bcs&, CStateT<float>, double*, hipStream_t);

// ---------------------------------------------------------------------------
// Residual norms: fixed-order sum of the per-block partials (strided
// per-thread sums, then a fixed tree), RMS over the interior.
__global__ __launch_bounds__(256) void norm_finalize_kernel(const double* part, int nb, double ncell,
                                                            double* out)
{
    __shared__ double red[NF][256];
    const int t = threadIdx.x;
    for (int f = 0; f < NF; ++f) {
        double s = 0.0;
        for (int b = t; b < nb; b += 256) s += part[(size_t)b * NF + f];
        red[f][t] = s;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int f = 0; f < NF; ++f) red[f][t] += red[f][t + w];
        __syncthreads();
    }
    if (t < NF) out[t] = sqrt(red[t][0] / ncell);
}

hipError_t launch_norm_finalize(const double* partials, int nblocks, double ncell, double* out,
                                hipStream_t s)
{
    norm_finalize_kernel<<<1, 256, 0, s>>>(partials, nblocks, ncell, out);
    return hipGetLastError();
}

}  // namespace cav
