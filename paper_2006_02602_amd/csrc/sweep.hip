// Residual + Euler-update sweep, wall boundary conditions, seeded init and
// the residual-norm finalize for gfx950 (FP64).
//
// The method (Xue & Roy, arXiv:2006.02602): artificial-compressibility
// Boussinesq equations (Sec. 2, Eq. 1-3), second-order central differences
// with a fourth-difference pressure dissipation (5-point p stencil, 3-point
// stencils for u, v, w, T; Sec. 3.1), first-order explicit Euler in pseudo
// time, pressure rescaled at the cavity centre every iteration (Sec. 2).
//
// This file is compiled with -ffp-contract=off: every fused multiply-add is
// written out with fma(), so two inlined copies of the per-cell update round
// identically (the centre-cell rescale relies on that).
#include "cavity_internal.h"

namespace cav {

// ---------------------------------------------------------------------------
// Per-cell residual.  Inputs: the 13-point pressure star and the 7-point
// stars of u, v, w, T.  Outputs: R_p (Eq. 1 times beta^2, with the
// dissipation -eps4 * lambda_x * F_x p / h_x per axis), R_u, R_v, R_w
// (Eq. 2, advective form, buoyancy +(T - t_inf) along z) and R_T (Eq. 3),
// and the local pseudo-time step.
struct Star {
    double p, pxm, pxp, pxm2, pxp2, pym, pyp, pym2, pyp2, pzm, pzp, pzm2, pzp2;
    double u, uxm, uxp, uym, uyp, uzm, uzp;
    double v, vxm, vxp, vym, vyp, vzm, vzp;
    double w, wxm, wxp, wym, wyp, wzm, wzp;
    double t, txm, txp, tym, typ, tzm, tzp;
};

__device__ __forceinline__ double lap3(const Coef& c, double q, double xm, double xp, double ym,
                                       double yp, double zm, double zp)
{
    // (L_x + L_y + L_z) q with L_x q = ((q_{i+1} + q_{i-1}) - 2 q_i) / h_x^2
    return fma(c.ix2, fma(-2.0, q, xp + xm), fma(c.iy2, fma(-2.0, q, yp + ym), c.iz2 * fma(-2.0, q, zp + zm)));
}

__device__ __forceinline__ void cell_residual(const Coef& c, const Star& s, double R[NF], double& dt)
{
    // first differences (times 2h)
    const double dxu = s.uxp - s.uxm, dyu = s.uyp - s.uym, dzu = s.uzp - s.uzm;
    const double dxv = s.vxp - s.vxm, dyv = s.vyp - s.vym, dzv = s.vzp - s.vzm;
    const double dxw = s.wxp - s.wxm, dyw = s.wyp - s.wym, dzw = s.wzp - s.wzm;
    const double dxt = s.txp - s.txm, dyt = s.typ - s.tym, dzt = s.tzp - s.tzm;
    const double dxp = s.pxp - s.pxm, dyp = s.pyp - s.pym, dzp = s.pzp - s.pzm;

    // advecting velocity scaled by 1/(2h): V . grad q = su*dxq + sv*dyq + sw*dzq
    const double su = s.u * c.hx2, sv = s.v * c.hy2, sw = s.w * c.hz2;

    // artificial compressibility and characteristic speeds over h
    const double u2 = s.u * s.u, v2 = s.v * s.v, w2 = s.w * s.w;
    const double beta2 = fmax((u2 + v2) + w2, c.beta2_floor);
    const double b4 = 4.0 * beta2;
    const double lxn = (fabs(s.u) + sqrt(u2 + b4)) * c.hx2;   // lambda_x / h_x
    const double lyn = (fabs(s.v) + sqrt(v2 + b4)) * c.hy2;
    const double lzn = (fabs(s.w) + sqrt(w2 + b4)) * c.hz2;
    dt = c.cfl * fmin(1.0 / ((lxn + lyn) + lzn), c.dt_visc);

    // continuity (Eq. 1 times beta^2) with fourth-difference dissipation
    const double div = fma(dxu, c.hx2, fma(dyv, c.hy2, dzw * c.hz2));
    const double fx = fma(6.0, s.p, fma(-4.0, s.pxp + s.pxm, s.pxp2 + s.pxm2));
    const double fy = fma(6.0, s.p, fma(-4.0, s.pyp + s.pym, s.pyp2 + s.pym2));
    const double fz = fma(6.0, s.p, fma(-4.0, s.pzp + s.pzm, s.pzp2 + s.pzm2));
    const double diss = fma(lxn, fx, fma(lyn, fy, lzn * fz));
    R[FP] = fma(-beta2, div, -c.eps4 * diss);

    // momentum (Eq. 2) and energy (Eq. 3)
    const double adu = fma(su, dxu, fma(sv, dyu, sw * dzu));
    const double adv = fma(su, dxv, fma(sv, dyv, sw * dzv));
    const double adw = fma(su, dxw, fma(sv, dyw, sw * dzw));
    const double adt = fma(su, dxt, fma(sv, dyt, sw * dzt));
    R[FU] = fma(c.nu, lap3(c, s.u, s.uxm, s.uxp, s.uym, s.uyp, s.uzm, s.uzp), -fma(dxp, c.hx2, adu));
    R[FV] = fma(c.nu, lap3(c, s.v, s.vxm, s.vxp, s.vym, s.vyp, s.vzm, s.vzp), -fma(dyp, c.hy2, adv));
    R[FW] = fma(c.nu, lap3(c, s.w, s.wxm, s.wxp, s.wym, s.wyp, s.wzm, s.wzp),
                (s.t - c.t_inf) - fma(dzp, c.hz2, adw));
    R[FT] = fma(c.alpha, lap3(c, s.t, s.txm, s.txp, s.tym, s.typ, s.tzm, s.tzp), -adt);
}

// Gather the stars of one cell straight from global memory (used once per
// block for the centre cell).
__device__ __forceinline__ void gather_global(const Dims& d, const CState& q, int i, int j, int k, Star& s)
{
    const int o = cell_off(d, i, j, k);
    const int X = 1, Y = d.sy, Z = d.sz;
    const double* P = q.f[FP];
    s.p = P[o];
    s.pxm = P[o - X]; s.pxp = P[o + X]; s.pxm2 = P[o - 2 * X]; s.pxp2 = P[o + 2 * X];
    s.pym = P[o - Y]; s.pyp = P[o + Y]; s.pym2 = P[o - 2 * Y]; s.pyp2 = P[o + 2 * Y];
    s.pzm = P[o - Z]; s.pzp = P[o + Z]; s.pzm2 = P[o - 2 * Z]; s.pzp2 = P[o + 2 * Z];
#define STAR7(F, nm)                                                              \
    {                                                                             \
        const double* A = q.f[F];                                                 \
        s.nm = A[o];                                                              \
        s.nm##xm = A[o - X]; s.nm##xp = A[o + X];                                 \
        s.nm##ym = A[o - Y]; s.nm##yp = A[o + Y];                                 \
        s.nm##zm = A[o - Z]; s.nm##zp = A[o + Z];                                 \
    }
    STAR7(FU, u) STAR7(FV, v) STAR7(FW, w) STAR7(FT, t)
#undef STAR7
}

// Map hardware block ids (dispatched round-robin over the 8 XCDs) to tiles
// so that each XCD works on one contiguous range of tiles and neighbouring
// tiles share that XCD's L2.
__device__ __forceinline__ int xcd_block(int bid, int nb)
{
    const int per = nb >> 3, rem = nb & 7;
    const int x = bid & 7, y = bid >> 3;
    return x * per + min(x, rem) + y;
}

// ---------------------------------------------------------------------------
// The sweep.  Block = one 64 x 8 tile of (i, j) columns (one wavefront per
// j row, i along the lanes) marching over a chunk of k planes.  The current
// plane k of all five fields lives in LDS with its i/j halo (2 for p, 1 for
// the rest); the k neighbours come from per-thread register queues (p:
// k-2..k+2, others k-1..k+1).  While plane k is computed, the loads of
// plane k+1's halo strips and of the next queue entries are in flight.
template <bool NORM>
__global__ __launch_bounds__(SW_TI * SW_TJ) void sweep_kernel(Dims d, Coef c, SweepGeom g, CState q,
                                                              State qn, double* partials)
{
    constexpr int TI = SW_TI, TJ = SW_TJ;
    constexpr int PW = TI + 4;              // LDS row pitch, p
    constexpr int UW = TI + 2;              // LDS row pitch, u v w T
    constexpr int UPL = (TJ + 2) * UW;      // LDS plane, one of u v w T
    __shared__ double sP[(TJ + 4) * PW];
    __shared__ double sU[4 * UPL];

    const int b = xcd_block(blockIdx.x, g.nblocks);
    const int bi = b % g.tiles_i;
    const int bj = (b / g.tiles_i) % g.tiles_j;
    const int bk = b / (g.tiles_i * g.tiles_j);
    const int i0 = bi * TI, j0 = bj * TJ;
    const int k0 = bk * g.kc;
    const int k1 = min(k0 + g.kc, d.nk);

    const int lane = threadIdx.x, row = threadIdx.y;
    const int i = i0 + lane, j = j0 + row;
    const bool active = i < d.ni && j < d.nj;
    const bool present = i < d.ni + NG && j < d.nj + NG;   // cell exists in memory

    // New pressure at the centre cell, recomputed with the same arithmetic
    // as its owner, so that every block subtracts the identical value.
    double pc_new;
    {
        Star s;
        gather_global(d, q, d.ni / 2, d.nj / 2, d.nk / 2, s);
        double R[NF], dt;
        cell_residual(c, s, R, dt);
        pc_new = fma(dt, R[FP], s.p);
    }

    // ---- strip assignments (fixed for the whole march) ----
    // p rows j0-2, j0-1, j0+TJ, j0+TJ+1: waves 0..3, one row each.
    const int prow_lds = row < 2 ? row : TJ + row;               // LDS row (p)
    const int prow_j = j0 - 2 + prow_lds;
    const bool has_prow = row < 4 && i < d.ni + NG && prow_j < d.nj + NG;
    // u v w T rows j0-1, j0+TJ: waves 0..7, field 1 + row/2.
    const int urow_f = row >> 1;                                  // 0..3 -> u v w T
    const int urow_lds = (row & 1) ? TJ + 1 : 0;
    const int urow_j = j0 - 1 + urow_lds;
    const bool has_urow = i < d.ni + NG && urow_j < d.nj + NG;
    // column halos of this wave's row: lanes 0..3 p (i0-2, i0-1, i0+TI, i0+TI+1),
    // lanes 4..11 u v w T (i0-1, i0+TI).
    int col_i, col_f, col_lds;
    if (lane < 4) {
        col_f = FP;
        col_lds = lane < 2 ? lane : TI + lane;                   // LDS column (p)
        col_i = i0 - 2 + col_lds;
        col_lds += (row + 2) * PW;
    } else {
        const int t = lane - 4;
        col_f = min(FU + (t >> 1), (int)FT);
        const int cc = (t & 1) ? TI + 1 : 0;                     // LDS column (u v w T)
        col_i = i0 - 1 + cc;
        col_lds = (col_f - FU) * UPL + (row + 1) * UW + cc;
    }
    const bool has_col = lane < 12 && col_i < d.ni + NG && j < d.nj + NG;

    const int off_c = cell_off(d, i, j, 0);                      // this column at k = 0
    const int off_prow = cell_off(d, i, prow_j, 0);
    const int off_urow = cell_off(d, i, urow_j, 0);
    const int off_col = cell_off(d, col_i, j, 0);
    const double* Pg = q.f[FP];
    const double* Ug = q.f[FU];
    const double* Vg = q.f[FV];
    const double* Wg = q.f[FW];
    const double* Tg = q.f[FT];
    const double* URg = q.f[FU + urow_f];
    const double* COLg = q.f[col_f];
    const int Z = d.sz;

    // ---- register queues ----
    double p0 = 0, p1 = 0, p2 = 0, p3 = 0;          // p at k-2, k-1, k, k+1
    double u0 = 0, u1 = 0, v0 = 0, v1 = 0, w0 = 0, w1 = 0, t0 = 0, t1 = 0;  // k-1, k
    double np_ = 0, nu_ = 0, nv_ = 0, nw_ = 0, nt_ = 0;   // in flight: p(k+2), uvwT(k+1)
    double r_prow = 0, r_urow = 0, r_col = 0;              // in flight: strips of plane k
    if (present) {
        p0 = Pg[off_c + (k0 - 2) * Z];
        p1 = Pg[off_c + (k0 - 1) * Z];
        p2 = Pg[off_c + k0 * Z];
        p3 = Pg[off_c + (k0 + 1) * Z];
        u0 = Ug[off_c + (k0 - 1) * Z]; u1 = Ug[off_c + k0 * Z];
        v0 = Vg[off_c + (k0 - 1) * Z]; v1 = Vg[off_c + k0 * Z];
        w0 = Wg[off_c + (k0 - 1) * Z]; w1 = Wg[off_c + k0 * Z];
        t0 = Tg[off_c + (k0 - 1) * Z]; t1 = Tg[off_c + k0 * Z];
        np_ = Pg[off_c + (k0 + 2) * Z];
        nu_ = Ug[off_c + (k0 + 1) * Z];
        nv_ = Vg[off_c + (k0 + 1) * Z];
        nw_ = Wg[off_c + (k0 + 1) * Z];
        nt_ = Tg[off_c + (k0 + 1) * Z];
    }
    if (has_prow) r_prow = Pg[off_prow + k0 * Z];
    if (has_urow) r_urow = URg[off_urow + k0 * Z];
    if (has_col) r_col = COLg[off_col + k0 * Z];

    double acc[NF] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int lc_p = (row + 2) * PW + lane + 2;                 // this cell in sP
    const int lc_u = (row + 1) * UW + lane + 1;                 // this cell in sU planes

    for (int k = k0; k < k1; ++k) {
        __syncthreads();                                        // plane k-1 fully consumed
        sP[lc_p] = p2;
        sU[0 * UPL + lc_u] = u1;
        sU[1 * UPL + lc_u] = v1;
        sU[2 * UPL + lc_u] = w1;
        sU[3 * UPL + lc_u] = t1;
        if (has_prow) sP[prow_lds * PW + lane + 2] = r_prow;
        if (has_urow) sU[urow_f * UPL + urow_lds * UW + lane + 1] = r_urow;
        if (has_col) (col_f == FP ? sP : sU)[col_lds] = r_col;
        __syncthreads();

        const double p4 = np_, u2 = nu_, v2 = nv_, w2 = nw_, t2 = nt_;
        if (k + 1 < k1) {                                       // prefetch for plane k+1
            const int kz = (k + 1) * Z;
            if (present) {
                np_ = Pg[off_c + kz + 2 * Z];
                nu_ = Ug[off_c + kz + Z];
                nv_ = Vg[off_c + kz + Z];
                nw_ = Wg[off_c + kz + Z];
                nt_ = Tg[off_c + kz + Z];
            }
            if (has_prow) r_prow = Pg[off_prow + kz];
            if (has_urow) r_urow = URg[off_urow + kz];
            if (has_col) r_col = COLg[off_col + kz];
        }

        if (active) {
            Star s;
            s.p = p2;
            s.pxm = sP[lc_p - 1]; s.pxp = sP[lc_p + 1]; s.pxm2 = sP[lc_p - 2]; s.pxp2 = sP[lc_p + 2];
            s.pym = sP[lc_p - PW]; s.pyp = sP[lc_p + PW]; s.pym2 = sP[lc_p - 2 * PW]; s.pyp2 = sP[lc_p + 2 * PW];
            s.pzm = p1; s.pzp = p3; s.pzm2 = p0; s.pzp2 = p4;
#define STAR_LDS(nm, plane, c0, cm, cp)                                            \
            s.nm = c0; s.nm##zm = cm; s.nm##zp = cp;                               \
            s.nm##xm = sU[plane * UPL + lc_u - 1]; s.nm##xp = sU[plane * UPL + lc_u + 1]; \
            s.nm##ym = sU[plane * UPL + lc_u - UW]; s.nm##yp = sU[plane * UPL + lc_u + UW];
            STAR_LDS(u, 0, u1, u0, u2)
            STAR_LDS(v, 1, v1, v0, v2)
            STAR_LDS(w, 2, w1, w0, w2)
            STAR_LDS(t, 3, t1, t0, t2)
#undef STAR_LDS
            double R[NF], dt;
            cell_residual(c, s, R, dt);
            const int o = off_c + k * Z;
            qn.f[FP][o] = fma(dt, R[FP], s.p) - pc_new;
            qn.f[FU][o] = fma(dt, R[FU], s.u);
            qn.f[FV][o] = fma(dt, R[FV], s.v);
            qn.f[FW][o] = fma(dt, R[FW], s.w);
            qn.f[FT][o] = fma(dt, R[FT], s.t);
            if (NORM) {
#pragma unroll
                for (int f = 0; f < NF; ++f) acc[f] = fma(R[f], R[f], acc[f]);
            }
        }
        p0 = p1; p1 = p2; p2 = p3; p3 = p4;
        u0 = u1; u1 = u2; v0 = v1; v1 = v2; w0 = w1; w1 = w2; t0 = t1; t1 = t2;
    }

    if (NORM) {
        // fixed-order block reduction: butterfly within the wavefront, then
        // the 8 wavefront sums in order
        __shared__ double red[TJ][NF];
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
            partials[(size_t)b * NF + lane] = t;
        }
    }
}

SweepGeom sweep_geom(const Dims& d)
{
    SweepGeom g;
    g.tiles_i = (d.ni + SW_TI - 1) / SW_TI;
    g.tiles_j = (d.nj + SW_TJ - 1) / SW_TJ;
    const int tiles = g.tiles_i * g.tiles_j;
    // aim at ~512 blocks (two 8-wave blocks per CU) with at least 8 planes each
    const int target = 512;
    int nkc = (target + tiles - 1) / tiles;
    nkc = max(1, min(nkc, (d.nk + 7) / 8));
    g.kc = (d.nk + nkc - 1) / nkc;
    g.nkc = (d.nk + g.kc - 1) / g.kc;
    g.nblocks = tiles * g.nkc;
    return g;
}

hipError_t launch_sweep(const Dims& d, const Coef& c, const SweepGeom& g, CState q, State qn,
                        double* partials, bool with_norm, hipStream_t s)
{
    dim3 block(SW_TI, SW_TJ), grid(g.nblocks);
    if (with_norm)
        sweep_kernel<true><<<grid, block, 0, s>>>(d, c, g, q, qn, partials);
    else
        sweep_kernel<false><<<grid, block, 0, s>>>(d, c, g, q, qn, partials);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Wall ghost layers (Sec. 2): one thread per wall-adjacent line of cells,
// all five fields, both ghost layers.  Only face ghosts are written.
__global__ __launch_bounds__(256) void bc_kernel(Dims d, Bcs bc, State q)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nx = 2LL * d.nj * d.nk, ny = 2LL * d.ni * d.nk, nz = 2LL * d.ni * d.nj;
    int o, s, axis;
    bool high;
    if (t < nx) {                                   // x walls: (j, k, side), j fastest
        axis = 0;
        const int j = (int)(t % d.nj);
        const long long r = t / d.nj;
        const int k = (int)(r % d.nk);
        high = r >= d.nk;
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
        double* A = q.f[FP];
        const double a = A[o], b = A[o + s];
        const double g1 = 2.0 * a - b;
        A[o - s] = g1;
        A[o - 2 * s] = 2.0 * g1 - a;
    }
    // u, v, w: no-slip (odd reflection)
#pragma unroll
    for (int f = FU; f <= FW; ++f) {
        double* A = q.f[f];
        const double a = A[o], b = A[o + s];
        A[o - s] = -a;
        A[o - 2 * s] = -b;
    }
    // T: fixed value on the hot/cold walls, zero gradient elsewhere
    {
        double* A = q.f[FT];
        const double a = A[o], b = A[o + s];
        if (axis == 0) {
            const double tw = high ? bc.t_cold : bc.t_hot;
            A[o - s] = 2.0 * tw - a;
            A[o - 2 * s] = 2.0 * tw - b;
        } else {
            A[o - s] = a;
            A[o - 2 * s] = b;
        }
    }
}

hipError_t launch_bc(const Dims& d, const Bcs& b, State q, hipStream_t s)
{
    const long long n = 2LL * ((long long)d.nj * d.nk + (long long)d.ni * d.nk + (long long)d.ni * d.nj);
    bc_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(d, b, q);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Seeded initial state: SplitMix64 (Steele, Lea & Flood 2014), output number
// f*2^40 + idx of the stream seeded with `seed`.
__device__ __forceinline__ double noise(uint64_t seed, int f, uint64_t idx, double amp)
{
    uint64_t z = seed + ((((uint64_t)f) << 40) + idx + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    const double r = (double)(z >> 11) * 0x1.0p-53;
    return (2.0 * r - 1.0) * amp;
}

__global__ __launch_bounds__(256) void init_kernel(Dims d, double t_hot, double t_cold, uint64_t seed,
                                                   double amp, State q)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)d.ni * d.nj * d.nk) return;
    const int i = (int)(idx % d.ni);
    const long long r = idx / d.ni;
    const int j = (int)(r % d.nj);
    const int k = (int)(r / d.nj);
    const int o = cell_off(d, i, j, k);
    const double xc = ((double)i + 0.5) / (double)d.ni;
    q.f[FP][o] = 0.0;
    q.f[FU][o] = noise(seed, 1, (uint64_t)idx, amp);
    q.f[FV][o] = noise(seed, 2, (uint64_t)idx, amp);
    q.f[FW][o] = noise(seed, 3, (uint64_t)idx, amp);
    q.f[FT][o] = (t_hot + (t_cold - t_hot) * xc) + noise(seed, 4, (uint64_t)idx, amp);
}

hipError_t launch_init(const Dims& d, double t_hot, double t_cold, uint64_t seed, double amp, State q,
                       hipStream_t s)
{
    const long long n = (long long)d.ni * d.nj * d.nk;
    init_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(d, t_hot, t_cold, seed, amp, q);
    return hipGetLastError();
}

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
