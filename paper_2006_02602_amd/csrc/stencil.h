// Per-cell stencil code shared by the forward sweep and its adjoint: the
// coefficient struct, the stars of one cell, the residual of Eq. 1-3, the
// wall ghost rules and the generic (slow) gather of one cell's stars.
// Included by sweep.hip and adjoint.hip only; both are built with
// -ffp-contract=off.
#pragma once

#include "cavity_internal.h"

namespace cav {

// Coefficients in the arithmetic type of the sweep.
template <typename Real>
struct CoefR {
    Real hx2, hy2, hz2, ix2, iy2, iz2, eps4, beta2_floor, nu, alpha, t_inf, cfl, dt_visc, t_hot, t_cold;
    const double* t_hot_field;    // NULL or nj*nk hot-wall temperatures, j fastest
};

template <typename Real>
__device__ __forceinline__ CoefR<Real> coef_as(const Coef& c)
{
    return CoefR<Real>{(Real)c.hx2, (Real)c.hy2, (Real)c.hz2, (Real)c.ix2, (Real)c.iy2, (Real)c.iz2,
                       (Real)c.eps4, (Real)c.beta2_floor, (Real)c.nu, (Real)c.alpha, (Real)c.t_inf,
                       (Real)c.cfl, (Real)c.dt_visc, (Real)c.t_hot, (Real)c.t_cold, c.t_hot_field};
}

// Temperature of the hot wall x = 0 next to row j of plane k.
template <typename Real>
__device__ __forceinline__ Real hot_wall(const CoefR<Real>& c, const Dims& d, int j, int k)
{
    return c.t_hot_field ? (Real)c.t_hot_field[j + (long long)d.nj * k] : c.t_hot;
}

// ---------------------------------------------------------------------------
// Per-cell residual.  Inputs: the 13-point pressure star and the 7-point
// stars of u, v, w, T.  Outputs: R_p (Eq. 1 times beta^2, with the
// dissipation -eps4 * lambda_x * F_x p / h_x per axis), R_u, R_v, R_w
// (Eq. 2, advective form, buoyancy +(T - t_inf) along z) and R_T (Eq. 3),
// and the local pseudo-time step.
template <typename Real>
struct Star {
    Real p, pxm, pxp, pxm2, pxp2, pym, pyp, pym2, pyp2, pzm, pzp, pzm2, pzp2;
    Real u, uxm, uxp, uym, uyp, uzm, uzp;
    Real v, vxm, vxp, vym, vyp, vzm, vzp;
    Real w, wxm, wxp, wym, wyp, wzm, wzp;
    Real t, txm, txp, tym, typ, tzm, tzp;
};

template <typename Real>
__device__ __forceinline__ Real lap3(const CoefR<Real>& c, Real q, Real xm, Real xp, Real ym,
                                       Real yp, Real zm, Real zp)
{
    // (L_x + L_y + L_z) q with L_x q = ((q_{i+1} + q_{i-1}) - 2 q_i) / h_x^2
    return fma(c.ix2, fma(Real(-2), q, xp + xm), fma(c.iy2, fma(Real(-2), q, yp + ym), c.iz2 * fma(Real(-2), q, zp + zm)));
}

// Square root of a positive argument: hardware reciprocal-square-root
// estimate refined by Goldschmidt's iteration (one coupled step for
// sqrt(x) and 1/(2 sqrt(x)), then a final residual correction), within an
// ulp of the correctly rounded result.  Arguments below 1e-300 are clamped.
__device__ __forceinline__ double sqrt_pos(double x)
{
    x = fmax(x, 1e-300);
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(h, d, g);
}

// 1/x for x > 0: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double recip_pos(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// FP32 forms: the hardware square root (within 1 ulp; the argument is kept
// above the denormal range) and a reciprocal estimate refined by one Newton
// step.
__device__ __forceinline__ float sqrt_pos(float x) { return __builtin_amdgcn_sqrtf(fmaxf(x, 1e-30f)); }

__device__ __forceinline__ float recip_pos(float x)
{
    const float y = __builtin_amdgcn_rcpf(x);
    return fmaf(y, fmaf(-x, y, 1.0f), y);
}

template <typename Real>
__device__ __forceinline__ void cell_residual(const CoefR<Real>& c, const Star<Real>& s, Real R[NF], Real& dt)
{
    // first differences (times 2h)
    const Real dxu = s.uxp - s.uxm, dyu = s.uyp - s.uym, dzu = s.uzp - s.uzm;
    const Real dxv = s.vxp - s.vxm, dyv = s.vyp - s.vym, dzv = s.vzp - s.vzm;
    const Real dxw = s.wxp - s.wxm, dyw = s.wyp - s.wym, dzw = s.wzp - s.wzm;
    const Real dxt = s.txp - s.txm, dyt = s.typ - s.tym, dzt = s.tzp - s.tzm;
    const Real dxp = s.pxp - s.pxm, dyp = s.pyp - s.pym, dzp = s.pzp - s.pzm;

    // advecting velocity scaled by 1/(2h): V . grad q = su*dxq + sv*dyq + sw*dzq
    const Real su = s.u * c.hx2, sv = s.v * c.hy2, sw = s.w * c.hz2;

    // artificial compressibility and characteristic speeds over h
    const Real u2 = s.u * s.u, v2 = s.v * s.v, w2 = s.w * s.w;
    const Real beta2 = fmax((u2 + v2) + w2, c.beta2_floor);
    const Real b4 = Real(4) * beta2;
    const Real lxn = (fabs(s.u) + sqrt_pos(u2 + b4)) * c.hx2;   // lambda_x / h_x
    const Real lyn = (fabs(s.v) + sqrt_pos(v2 + b4)) * c.hy2;
    const Real lzn = (fabs(s.w) + sqrt_pos(w2 + b4)) * c.hz2;
    dt = c.cfl * fmin(recip_pos((lxn + lyn) + lzn), c.dt_visc);

    // continuity (Eq. 1 times beta^2) with fourth-difference dissipation
    const Real div = fma(dxu, c.hx2, fma(dyv, c.hy2, dzw * c.hz2));
    const Real fx = fma(Real(6), s.p, fma(Real(-4), s.pxp + s.pxm, s.pxp2 + s.pxm2));
    const Real fy = fma(Real(6), s.p, fma(Real(-4), s.pyp + s.pym, s.pyp2 + s.pym2));
    const Real fz = fma(Real(6), s.p, fma(Real(-4), s.pzp + s.pzm, s.pzp2 + s.pzm2));
    const Real diss = fma(lxn, fx, fma(lyn, fy, lzn * fz));
    R[FP] = fma(-beta2, div, -c.eps4 * diss);

    // momentum (Eq. 2) and energy (Eq. 3)
    const Real adu = fma(su, dxu, fma(sv, dyu, sw * dzu));
    const Real adv = fma(su, dxv, fma(sv, dyv, sw * dzv));
    const Real adw = fma(su, dxw, fma(sv, dyw, sw * dzw));
    const Real adt = fma(su, dxt, fma(sv, dyt, sw * dzt));
    R[FU] = fma(c.nu, lap3(c, s.u, s.uxm, s.uxp, s.uym, s.uyp, s.uzm, s.uzp), -fma(dxp, c.hx2, adu));
    R[FV] = fma(c.nu, lap3(c, s.v, s.vxm, s.vxp, s.vym, s.vyp, s.vzm, s.vzp), -fma(dyp, c.hy2, adv));
    R[FW] = fma(c.nu, lap3(c, s.w, s.wxm, s.wxp, s.wym, s.wyp, s.wzm, s.wzp),
                (s.t - c.t_inf) - fma(dzp, c.hz2, adw));
    R[FT] = fma(c.alpha, lap3(c, s.t, s.txm, s.txp, s.tym, s.typ, s.tzm, s.tzp), -adt);
}

// ---------------------------------------------------------------------------
// Wall ghosts on the fly (Sec. 2).  The state in HBM holds only interior
// cells that the sweep reads; a face-ghost value g = 1, 2 layers beyond a
// wall is derived from the interior cells m0 (next to the wall) and m1:
//   p:        g1 = 2 q(m0) - q(m1), g2 = 2 g1 - q(m0)  (one-sided linear
//             extrapolation, second order)
//   u, v, w:  g = -q(m_{g-1})                          (no-slip)
//   T:        g = 2 T_wall - q(m_{g-1}) on the hot (x = 0) and cold (x = 1)
//             walls, g = q(m_{g-1}) on the adiabatic walls.
enum { SIDE_X_LO = 0, SIDE_X_HI = 1, SIDE_OTHER = 2 };
constexpr int SLOT_UNUSED = 3;

// Where a thread reads one (i, j) column of every plane: the cell itself
// (code 0), or the two mirror cells of a face ghost (code = g | side << 2),
// or nothing (edge/corner column or beyond the ghosts: code 3).
struct Slot {
    int oa, ob, code;
};

__device__ __forceinline__ Slot make_slot(const Dims& d, int i, int j)
{
    Slot s{0, 0, SLOT_UNUSED};
    const bool ii = i >= 0 && i < d.ni, jj = j >= 0 && j < d.nj;
    if (ii && jj) {
        s.oa = cell_off(d, i, j, 0);
        s.code = 0;
    } else if (!ii && jj) {
        const bool lo = i < 0;
        const int g = lo ? -i : i - d.ni + 1;
        if (g <= NG) {
            s.oa = cell_off(d, lo ? 0 : d.ni - 1, j, 0);
            s.ob = cell_off(d, lo ? 1 : d.ni - 2, j, 0);
            s.code = g | ((lo ? SIDE_X_LO : SIDE_X_HI) << 2);
        }
    } else if (ii && !jj) {
        const bool lo = j < 0;
        const int g = lo ? -j : j - d.nj + 1;
        if (g <= NG) {
            s.oa = cell_off(d, i, lo ? 0 : d.nj - 1, 0);
            s.ob = cell_off(d, i, lo ? 1 : d.nj - 2, 0);
            s.code = g | (SIDE_OTHER << 2);
        }
    }
    return s;
}

// t_lo: the hot-wall temperature at this ghost's (j, k) (used on x = 0 only)
template <typename Real>
__device__ __forceinline__ Real ghost_value(int f, int code, Real a, Real b, const CoefR<Real>& c, Real t_lo)
{
    const int g = code & 3, side = code >> 2;
    if (f == FP) {
        const Real g1 = Real(2) * a - b;
        return g == 1 ? g1 : Real(2) * g1 - a;
    }
    const Real m = g == 1 ? a : b;
    if (f == FT) return side == SIDE_X_LO ? Real(2) * t_lo - m : (side == SIDE_X_HI ? Real(2) * c.t_cold - m : m);
    return -m;
}

template <typename Real>
__device__ __forceinline__ Real slot_load(const Real* G, const Slot& s, int kz, int f, const CoefR<Real>& c,
                                          Real t_lo)
{
    Real v = Real(0);
    if (s.code == 0)
        v = G[s.oa + kz];
    else if (s.code != SLOT_UNUSED)
        v = ghost_value(f, s.code, G[s.oa + kz], G[s.ob + kz], c, t_lo);
    return v;
}

// Any interior or face-ghost value, straight from global memory (used once
// per block, for the stars of the centre cell).
template <typename Real>
__device__ __forceinline__ Real value_at(const Dims& d, const CStateT<Real>& q, const CoefR<Real>& c, int f, int i, int j,
                                           int k)
{
    const Real* G = q.f[f];
    if (k < 0 || k >= d.nk) {
        const bool lo = k < 0;
        const int g = lo ? -k : k - d.nk + 1;
        const Real a = G[cell_off(d, i, j, lo ? 0 : d.nk - 1)];
        const Real b = G[cell_off(d, i, j, lo ? 1 : d.nk - 2)];
        return ghost_value(f, g | (SIDE_OTHER << 2), a, b, c, c.t_hot);
    }
    // the wall field is read only for an x = 0 ghost, whose row (j, k) is in range
    const Real t_lo = (f == FT && i < 0 && j >= 0 && j < d.nj) ? hot_wall(c, d, j, k) : c.t_hot;
    return slot_load(G, make_slot(d, i, j), k * d.sz, f, c, t_lo);
}

template <typename Real>
__device__ __forceinline__ void gather_global(const Dims& d, const CStateT<Real>& q, const CoefR<Real>& c, int i, int j, int k,
                                              Star<Real>& s)
{
    auto P = [&](int di, int dj, int dk) { return value_at(d, q, c, FP, i + di, j + dj, k + dk); };
    s.p = P(0, 0, 0);
    s.pxm = P(-1, 0, 0); s.pxp = P(1, 0, 0); s.pxm2 = P(-2, 0, 0); s.pxp2 = P(2, 0, 0);
    s.pym = P(0, -1, 0); s.pyp = P(0, 1, 0); s.pym2 = P(0, -2, 0); s.pyp2 = P(0, 2, 0);
    s.pzm = P(0, 0, -1); s.pzp = P(0, 0, 1); s.pzm2 = P(0, 0, -2); s.pzp2 = P(0, 0, 2);
#define STAR7(F, nm)                                                                  \
    {                                                                                 \
        auto A = [&](int di, int dj, int dk) { return value_at(d, q, c, F, i + di, j + dj, k + dk); }; \
        s.nm = A(0, 0, 0);                                                            \
        s.nm##xm = A(-1, 0, 0); s.nm##xp = A(1, 0, 0);                                \
        s.nm##ym = A(0, -1, 0); s.nm##yp = A(0, 1, 0);                                \
        s.nm##zm = A(0, 0, -1); s.nm##zp = A(0, 0, 1);                                \
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


}  // namespace cav
