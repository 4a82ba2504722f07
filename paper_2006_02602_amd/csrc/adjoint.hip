// Discrete adjoint (reverse mode) of one pseudo-time step and of the mean
// hot-wall Nusselt number, in FP64.
//
// One step maps the state q^n to q^{n+1} (Sec. 2, Eq. 1-3): wall ghosts G
// from the interior cells and the hot-wall temperatures Theta, per cell the
// residual R(S) and local step dt(S) of its stars S, q* = q + dt R, and the
// pressure rescale p^{n+1} = p* - p*(centre).  Given the cotangent lambda of
// q^{n+1}, the reverse step returns the cotangent of q^n and adds the
// cotangents of Theta and of Ra:
//   1. lambda*_p(centre) = lambda_p(centre) - sum over cells of lambda_p
//      (transpose of the rescale); lambda* = lambda elsewhere;
//   2. per cell: seeds dR_f = lambda*_f dt, d(dt) = sum_f lambda*_f R_f,
//      then the hand-written reverse of the residual gives the cotangents of
//      the 41 star values (stored per cell and slot) and of nu, alpha and
//      the viscous step limit (reduced per block into the Ra cotangent);
//   3. per cell and face-ghost position: the sum of the star cotangents
//      that land there, plus lambda* on interior cells (the identity part of
//      q + dt R);
//   4. transpose of the wall rules, one axis at a time: each ghost's
//      cotangent moves onto the two interior cells (and Theta) it was
//      derived from.
// Every sum runs in a fixed order, so results are run-to-run identical.
#include "cavity_internal.h"
#include "stencil.h"

#include <algorithm>

namespace cav {

namespace {

constexpr int NSLOT = 41;          // 13 pressure + 4 x 7 star values
constexpr int ADJ_THREADS = 256;

// Star slot s of field f sits at offset (di, dj, dk) from its cell.
struct SlotOff {
    signed char f, di, dj, dk;
};
__constant__ SlotOff kSlots[NSLOT] = {
    {FP, 0, 0, 0},  {FP, -1, 0, 0}, {FP, 1, 0, 0},  {FP, -2, 0, 0}, {FP, 2, 0, 0},  {FP, 0, -1, 0},
    {FP, 0, 1, 0},  {FP, 0, -2, 0}, {FP, 0, 2, 0},  {FP, 0, 0, -1}, {FP, 0, 0, 1},  {FP, 0, 0, -2},
    {FP, 0, 0, 2},
    {FU, 0, 0, 0},  {FU, -1, 0, 0}, {FU, 1, 0, 0},  {FU, 0, -1, 0}, {FU, 0, 1, 0},  {FU, 0, 0, -1},
    {FU, 0, 0, 1},
    {FV, 0, 0, 0},  {FV, -1, 0, 0}, {FV, 1, 0, 0},  {FV, 0, -1, 0}, {FV, 0, 1, 0},  {FV, 0, 0, -1},
    {FV, 0, 0, 1},
    {FW, 0, 0, 0},  {FW, -1, 0, 0}, {FW, 1, 0, 0},  {FW, 0, -1, 0}, {FW, 0, 1, 0},  {FW, 0, 0, -1},
    {FW, 0, 0, 1},
    {FT, 0, 0, 0},  {FT, -1, 0, 0}, {FT, 1, 0, 0},  {FT, 0, -1, 0}, {FT, 0, 1, 0},  {FT, 0, 0, -1},
    {FT, 0, 0, 1},
};
// first slot of each field and its count
__device__ __forceinline__ int slot_begin(int f) { return f == FP ? 0 : 13 + 7 * (f - 1); }
__device__ __forceinline__ int slot_count(int f) { return f == FP ? 13 : 7; }

// Star values in slot order (the order of kSlots).
__device__ __forceinline__ void star_to_slots(const Star<double>& s, double v[NSLOT])
{
    const double t[NSLOT] = {s.p,   s.pxm, s.pxp, s.pxm2, s.pxp2, s.pym, s.pyp, s.pym2, s.pyp2, s.pzm, s.pzp,
                             s.pzm2, s.pzp2, s.u,  s.uxm,  s.uxp,  s.uym, s.uyp, s.uzm,  s.uzp,  s.v,   s.vxm,
                             s.vxp, s.vym, s.vyp, s.vzm,  s.vzp,  s.w,   s.wxm, s.wxp,  s.wym,  s.wyp, s.wzm,
                             s.wzp, s.t,   s.txm, s.txp,  s.tym,  s.typ, s.tzm, s.tzp};
#pragma unroll
    for (int i = 0; i < NSLOT; ++i) v[i] = t[i];
}

// Stars of interior cell (i, j, k) of q: direct loads two or more cells from
// every wall, else the generic gather with the wall rules.
__device__ __forceinline__ void gather_cell(const Dims& d, const CStateT<double>& q, const CoefR<double>& c,
                                            int i, int j, int k, Star<double>& s)
{
    if (i < 2 || j < 2 || k < 2 || i >= d.ni - 2 || j >= d.nj - 2 || k >= d.nk - 2) {
        gather_global(d, q, c, i, j, k, s);
        return;
    }
    const int o = cell_off(d, i, j, k), X = 1, Y = d.sy, Z = d.sz;
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

// Reverse of cell_residual: given the cotangents a[f] of R_f and b of dt,
// return the cotangents of the 41 star values (in sb) and of nu, alpha and
// the viscous step limit.  Non-smooth points take one side: |u| has slope
// +1 at u = 0; beta^2 = max(|V|^2, floor) follows |V|^2 only where it is
// strictly larger; dt follows the convective limit only where it is
// strictly smaller than the viscous one.
__device__ __forceinline__ void residual_reverse(const CoefR<double>& c, const Star<double>& s, const double a[NF],
                                                 double b, Star<double>& sb, double& nub, double& alb,
                                                 double& dtvb)
{
    // ---- forward intermediates (same formulas as cell_residual) ----
    const double dxu = s.uxp - s.uxm, dyu = s.uyp - s.uym, dzu = s.uzp - s.uzm;
    const double dxv = s.vxp - s.vxm, dyv = s.vyp - s.vym, dzv = s.vzp - s.vzm;
    const double dxw = s.wxp - s.wxm, dyw = s.wyp - s.wym, dzw = s.wzp - s.wzm;
    const double dxt = s.txp - s.txm, dyt = s.typ - s.tym, dzt = s.tzp - s.tzm;
    const double su = s.u * c.hx2, sv = s.v * c.hy2, sw = s.w * c.hz2;
    const double u2 = s.u * s.u, v2 = s.v * s.v, w2 = s.w * s.w;
    const double vv = (u2 + v2) + w2;
    const bool beta_free = vv > c.beta2_floor;
    const double beta2 = beta_free ? vv : c.beta2_floor;
    const double b4 = 4.0 * beta2;
    const double rx = sqrt_pos(u2 + b4), ry = sqrt_pos(v2 + b4), rz = sqrt_pos(w2 + b4);
    const double lxn = (fabs(s.u) + rx) * c.hx2;
    const double lyn = (fabs(s.v) + ry) * c.hy2;
    const double lzn = (fabs(s.w) + rz) * c.hz2;
    const double inv = recip_pos((lxn + lyn) + lzn);
    const bool convective = inv < c.dt_visc;
    const double div = fma(dxu, c.hx2, fma(dyv, c.hy2, dzw * c.hz2));
    const double fx = fma(6.0, s.p, fma(-4.0, s.pxp + s.pxm, s.pxp2 + s.pxm2));
    const double fy = fma(6.0, s.p, fma(-4.0, s.pyp + s.pym, s.pyp2 + s.pym2));
    const double fz = fma(6.0, s.p, fma(-4.0, s.pzp + s.pzm, s.pzp2 + s.pzm2));
    const double lapu = lap3(c, s.u, s.uxm, s.uxp, s.uym, s.uyp, s.uzm, s.uzp);
    const double lapv = lap3(c, s.v, s.vxm, s.vxp, s.vym, s.vyp, s.vzm, s.vzp);
    const double lapw = lap3(c, s.w, s.wxm, s.wxp, s.wym, s.wyp, s.wzm, s.wzp);
    const double lapt = lap3(c, s.t, s.txm, s.txp, s.tym, s.typ, s.tzm, s.tzp);

    // ---- reverse ----
    // R_T = alpha lap T - adv T;  R_w = nu lap w + (T - t_inf) - (D_z p + adv w); ...
    const double lapub = c.nu * a[FU], lapvb = c.nu * a[FV], lapwb = c.nu * a[FW], laptb = c.alpha * a[FT];
    nub = (a[FU] * lapu + a[FV] * lapv) + a[FW] * lapw;
    alb = a[FT] * lapt;
    const double dxpb = -a[FU] * c.hx2, dypb = -a[FV] * c.hy2, dzpb = -a[FW] * c.hz2;
    const double adub = -a[FU], advb = -a[FV], adwb = -a[FW], adtb = -a[FT];
    // R_p = -beta^2 div - eps4 (lxn fx + lyn fy + lzn fz)
    double beta2b = -div * a[FP];
    const double divb = -beta2 * a[FP];
    const double dissb = -c.eps4 * a[FP];
    double lxnb = fx * dissb, lynb = fy * dissb, lznb = fz * dissb;
    const double fxb = lxn * dissb, fyb = lyn * dissb, fzb = lzn * dissb;
    // advection: adv q = su D_x q + sv D_y q + sw D_z q (differences times 2h)
    const double sub = ((adub * dxu + advb * dxv) + adwb * dxw) + adtb * dxt;
    const double svb = ((adub * dyu + advb * dyv) + adwb * dyw) + adtb * dyt;
    const double swb = ((adub * dzu + advb * dzv) + adwb * dzw) + adtb * dzt;
    const double dxub = su * adub + c.hx2 * divb, dyub = sv * adub, dzub = sw * adub;
    const double dxvb = su * advb, dyvb = sv * advb + c.hy2 * divb, dzvb = sw * advb;
    const double dxwb = su * adwb, dywb = sv * adwb, dzwb = sw * adwb + c.hz2 * divb;
    const double dxtb = su * adtb, dytb = sv * adtb, dztb = sw * adtb;
    // dt = cfl min(1 / (lxn + lyn + lzn), dt_visc)
    dtvb = 0.0;
    if (convective) {
        const double lsb = -(c.cfl * b) * inv * inv;
        lxnb += lsb;
        lynb += lsb;
        lznb += lsb;
    } else {
        dtvb = c.cfl * b;
    }
    // lambda_i / h_i = (|V_i| + sqrt(V_i^2 + 4 beta^2)) / (2 h_i)
    const double rxb = c.hx2 * lxnb, ryb = c.hy2 * lynb, rzb = c.hz2 * lznb;
    double ub = (s.u < 0.0 ? -rxb : rxb) + c.hx2 * sub;
    double vb = (s.v < 0.0 ? -ryb : ryb) + c.hy2 * svb;
    double wb = (s.w < 0.0 ? -rzb : rzb) + c.hz2 * swb;
    const double tx = rxb / (2.0 * rx), ty = ryb / (2.0 * ry), tz = rzb / (2.0 * rz);
    beta2b += 4.0 * ((tx + ty) + tz);
    double u2b = tx, v2b = ty, w2b = tz;
    if (beta_free) {
        u2b += beta2b;
        v2b += beta2b;
        w2b += beta2b;
    }
    ub += 2.0 * s.u * u2b;
    vb += 2.0 * s.v * v2b;
    wb += 2.0 * s.w * w2b;

    const double ctr = -2.0 * ((c.ix2 + c.iy2) + c.iz2);
    // pressure star: D p in the momentum equations, F p in the dissipation
    sb.p = 6.0 * ((fxb + fyb) + fzb);
    sb.pxp = dxpb - 4.0 * fxb; sb.pxm = -dxpb - 4.0 * fxb; sb.pxp2 = fxb; sb.pxm2 = fxb;
    sb.pyp = dypb - 4.0 * fyb; sb.pym = -dypb - 4.0 * fyb; sb.pyp2 = fyb; sb.pym2 = fyb;
    sb.pzp = dzpb - 4.0 * fzb; sb.pzm = -dzpb - 4.0 * fzb; sb.pzp2 = fzb; sb.pzm2 = fzb;
#define STAR7B(nm, dxb, dyb, dzb, lb, cb)                                  \
    sb.nm = (cb) + ctr * (lb);                                             \
    sb.nm##xp = (dxb) + c.ix2 * (lb); sb.nm##xm = -(dxb) + c.ix2 * (lb);   \
    sb.nm##yp = (dyb) + c.iy2 * (lb); sb.nm##ym = -(dyb) + c.iy2 * (lb);   \
    sb.nm##zp = (dzb) + c.iz2 * (lb); sb.nm##zm = -(dzb) + c.iz2 * (lb);
    STAR7B(u, dxub, dyub, dzub, lapub, ub)
    STAR7B(v, dxvb, dyvb, dzvb, lapvb, vb)
    STAR7B(w, dxwb, dywb, dzwb, lapwb, wb)
    STAR7B(t, dxtb, dytb, dztb, laptb, a[FW])        // buoyancy: dR_w/dT = 1
#undef STAR7B
}

__device__ __forceinline__ int centre_off(const Dims& d) { return cell_off(d, d.ni / 2, d.nj / 2, d.nk / 2); }

// ---- 1. sum of lambda_p over the interior, fixed order ----
// Stage 1: one thread per (j, k) row, summing along i; a fixed tree per
// block writes part[block].
__global__ __launch_bounds__(ADJ_THREADS) void row_sum_kernel(Dims d, const double* __restrict__ lp,
                                                              double* __restrict__ part)
{
    __shared__ double red[ADJ_THREADS];
    const int t = threadIdx.x;
    const long long r = (long long)blockIdx.x * ADJ_THREADS + t;
    double acc = 0.0;
    if (r < (long long)d.nj * d.nk) {
        const int j = (int)(r % d.nj), k = (int)(r / d.nj);
        const int o = cell_off(d, 0, j, k);
        for (int i = 0; i < d.ni; ++i) acc += lp[o + i];
    }
    red[t] = acc;
    __syncthreads();
    for (int w = ADJ_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = red[0];
}

// Sum of part[0..n) in a fixed order; out[0] = sum (or += when accumulate).
__global__ __launch_bounds__(ADJ_THREADS) void sum_kernel(const double* __restrict__ part, int n, double* out,
                                                          int accumulate)
{
    __shared__ double red[ADJ_THREADS];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int b = t; b < n; b += ADJ_THREADS) acc += part[b];
    red[t] = acc;
    __syncthreads();
    for (int w = ADJ_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[0] = accumulate ? out[0] + red[0] : red[0];
}

// lambda* of interior cell offset o, field f (transpose of the rescale).
__device__ __forceinline__ double lam_star(const Dims& d, const CStateT<double>& lam, int f, int o, double psum)
{
    const double v = lam.f[f][o];
    return (f == FP && o == centre_off(d)) ? v - psum : v;
}

// ---- 2. per-cell reverse of the residual and the update ----
struct RaFactors {
    double nu, alpha, dtv;        // d(nu)/dRa, d(alpha)/dRa, d(dt_visc)/dRa
};

__global__ __launch_bounds__(ADJ_THREADS) void cell_reverse_kernel(Dims d, Coef cd, RaFactors rf,
                                                                   CStateT<double> q, CStateT<double> lam,
                                                                   const double* __restrict__ psum,
                                                                   double* __restrict__ T,
                                                                   double* __restrict__ ra_part)
{
    __shared__ double red[ADJ_THREADS];
    const CoefR<double> c = coef_as<double>(cd);
    const long long n = (long long)d.ni * d.nj * d.nk;
    const long long idx = (long long)blockIdx.x * ADJ_THREADS + threadIdx.x;
    double ra = 0.0;
    if (idx < n) {
        const int i = (int)(idx % d.ni);
        const long long r = idx / d.ni;
        const int j = (int)(r % d.nj), k = (int)(r / d.nj);
        Star<double> s;
        gather_cell(d, q, c, i, j, k, s);
        double R[NF], dt;
        cell_residual(c, s, R, dt);
        const int o = cell_off(d, i, j, k);
        const double ps = psum[0];
        double a[NF], b = 0.0;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double ls = lam_star(d, lam, f, o, ps);
            a[f] = ls * dt;
            b = fma(ls, R[f], b);
        }
        Star<double> sb;
        double nub, alb, dtvb;
        residual_reverse(c, s, a, b, sb, nub, alb, dtvb);
        double v[NSLOT];
        star_to_slots(sb, v);
#pragma unroll
        for (int sl = 0; sl < NSLOT; ++sl) T[(size_t)sl * n + idx] = v[sl];
        ra = (nub * rf.nu + alb * rf.alpha) + dtvb * rf.dtv;
    }
    const int t = threadIdx.x;
    red[t] = ra;
    __syncthreads();
    for (int w = ADJ_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) ra_part[blockIdx.x] = red[0];
}

// ---- 3. gather of the star cotangents per cell and face-ghost position ----
// One thread per position (i, j, k) of the box [-2, n+2)^3 of field
// blockIdx.y; positions with two coordinates outside, or beyond the reach
// of the field's star (2 for p, 1 for u v w T), are skipped.
__global__ __launch_bounds__(ADJ_THREADS) void gather_kernel(Dims d, CStateT<double> lam,
                                                             const double* __restrict__ psum,
                                                             const double* __restrict__ T, StateT<double> out)
{
    const int f = blockIdx.y;
    const int ei = d.ni + 2 * NG, ej = d.nj + 2 * NG, ek = d.nk + 2 * NG;
    const long long e = (long long)blockIdx.x * ADJ_THREADS + threadIdx.x;
    if (e >= (long long)ei * ej * ek) return;
    const int i = (int)(e % ei) - NG;
    const long long r = e / ei;
    const int j = (int)(r % ej) - NG, k = (int)(r / ej) - NG;
    const int reach = f == FP ? 2 : 1;
    const int oi = i < 0 ? -i : (i >= d.ni ? i - d.ni + 1 : 0);
    const int oj = j < 0 ? -j : (j >= d.nj ? j - d.nj + 1 : 0);
    const int ok = k < 0 ? -k : (k >= d.nk ? k - d.nk + 1 : 0);
    if ((oi > 0) + (oj > 0) + (ok > 0) > 1 || oi > reach || oj > reach || ok > reach) return;
    const long long n = (long long)d.ni * d.nj * d.nk;
    double acc = 0.0;
    const int s0 = slot_begin(f), ns = slot_count(f);
    for (int sl = s0; sl < s0 + ns; ++sl) {
        const SlotOff so = kSlots[sl];
        const int mi = i - so.di, mj = j - so.dj, mk = k - so.dk;
        if (mi >= 0 && mi < d.ni && mj >= 0 && mj < d.nj && mk >= 0 && mk < d.nk)
            acc += T[(size_t)sl * n + mi + (long long)d.ni * (mj + (long long)d.nj * mk)];
    }
    const int o = cell_off(d, i, j, k);
    if (oi + oj + ok == 0) acc += lam_star(d, lam, f, o, psum[0]);
    out.f[f][o] = acc;
}

// ---- 4. transpose of the wall rules along one axis ----
// Ghost g = 1, 2 beyond a wall was derived from interior cells m0 (next to
// the wall) and m1:  p: g1 = 2 m0 - m1, g2 = 3 m0 - 2 m1;  u v w: g1 = -m0;
// T: g1 = 2 T_wall - m0 (hot and cold walls), g1 = m0 (adiabatic).  One
// thread per wall line handles both walls of the axis, low side first.
__global__ __launch_bounds__(ADJ_THREADS) void wall_reverse_kernel(Dims d, int axis, StateT<double> lam,
                                                                   double* __restrict__ dthot)
{
    const int n0 = axis == 0 ? d.nj : d.ni;            // tangential extents
    const int n1 = axis == 2 ? d.nj : d.nk;
    const long long t = (long long)blockIdx.x * ADJ_THREADS + threadIdx.x;
    if (t >= (long long)n0 * n1) return;
    const int a = (int)(t % n0), bq = (int)(t / n0);
    const int nn = axis == 0 ? d.ni : (axis == 1 ? d.nj : d.nk);
    const int stride = axis == 0 ? 1 : (axis == 1 ? d.sy : d.sz);
    auto at = [&](int m) {                              // cell m along the axis
        return axis == 0 ? cell_off(d, m, a, bq) : (axis == 1 ? cell_off(d, a, m, bq) : cell_off(d, a, bq, m));
    };
    for (int side = 0; side < 2; ++side) {
        const int m0 = side ? at(nn - 1) : at(0);
        const int s = side ? stride : -stride;          // towards the ghosts
        const int m1 = m0 - s;
        const int g1 = m0 + s, g2 = m0 + 2 * s;
        {
            double* L = lam.f[FP];
            const double b1 = L[g1], b2 = L[g2];
            L[m0] += 2.0 * b1 + 3.0 * b2;
            L[m1] -= b1 + 2.0 * b2;
        }
#pragma unroll
        for (int f = FU; f <= FW; ++f) lam.f[f][m0] -= lam.f[f][g1];
        {
            double* L = lam.f[FT];
            const double b1 = L[g1];
            if (axis == 0) {
                L[m0] -= b1;
                if (side == 0 && dthot) dthot[a + (long long)d.nj * bq] += 2.0 * b1;
            } else {
                L[m0] += b1;
            }
        }
    }
}

// ---- cotangent of the mean hot-wall Nusselt number ----
// Nu = sum over (j, k) of -(9 T_0 - T_1 - 8 T_wall) * ni / 3 / (nj nk dT):
// writes lambda (zero except T at i = 0, 1) and adds dNu/dT_wall.
__global__ __launch_bounds__(ADJ_THREADS) void nusselt_seed_kernel(Dims d, double scale, StateT<double> lam,
                                                                   double* __restrict__ dthot)
{
    const long long n = (long long)d.ni * d.nj * d.nk;
    const long long idx = (long long)blockIdx.x * ADJ_THREADS + threadIdx.x;
    if (idx >= n) return;
    const int i = (int)(idx % d.ni);
    const long long r = idx / d.ni;
    const int j = (int)(r % d.nj), k = (int)(r / d.nj);
    const int o = cell_off(d, i, j, k);
#pragma unroll
    for (int f = FP; f < FT; ++f) lam.f[f][o] = 0.0;
    lam.f[FT][o] = i == 0 ? -9.0 * scale : (i == 1 ? scale : 0.0);
    if (i == 0 && dthot) dthot[j + (long long)d.nj * k] += 8.0 * scale;
}

}  // namespace

// ---------------------------------------------------------------------------
size_t adjoint_ws_doubles(const Dims& d)
{
    const long long n = (long long)d.ni * d.nj * d.nk;
    const long long rows = (long long)d.nj * d.nk;
    const long long nb = std::max((n + ADJ_THREADS - 1) / ADJ_THREADS, (rows + ADJ_THREADS - 1) / ADJ_THREADS);
    const long long part = (nb + 7) / 8 * 8;
    return (size_t)(8 + part + (long long)NSLOT * n);
}

hipError_t launch_adjoint_step(const Dims& d, const Coef& c, double Ra, CStateT<double> q, CStateT<double> lam_in,
                               StateT<double> lam_out, double* ws, double* dthot, double* dra, hipStream_t s)
{
    const long long n = (long long)d.ni * d.nj * d.nk;
    const long long rows = (long long)d.nj * d.nk;
    double* psum = ws;                       // ws[0]: sum of lambda_p; ws[1]: Ra scratch
    double* part = ws + 8;
    const long long nb = std::max((n + ADJ_THREADS - 1) / ADJ_THREADS, (rows + ADJ_THREADS - 1) / ADJ_THREADS);
    double* T = part + (nb + 7) / 8 * 8;
    hipError_t e;

    const int rb = (int)((rows + ADJ_THREADS - 1) / ADJ_THREADS);
    row_sum_kernel<<<rb, ADJ_THREADS, 0, s>>>(d, lam_in.f[FP], part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    sum_kernel<<<1, ADJ_THREADS, 0, s>>>(part, rb, psum, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    RaFactors rf;
    rf.nu = -c.nu / (2.0 * Ra);
    rf.alpha = -c.alpha / (2.0 * Ra);
    rf.dtv = c.dt_visc / (2.0 * Ra);
    const int cb = (int)((n + ADJ_THREADS - 1) / ADJ_THREADS);
    cell_reverse_kernel<<<cb, ADJ_THREADS, 0, s>>>(d, c, rf, q, lam_in, psum, T, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (dra) {
        sum_kernel<<<1, ADJ_THREADS, 0, s>>>(part, cb, dra, 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }

    const long long box = (long long)(d.ni + 2 * NG) * (d.nj + 2 * NG) * (d.nk + 2 * NG);
    dim3 gg((unsigned)((box + ADJ_THREADS - 1) / ADJ_THREADS), NF);
    gather_kernel<<<gg, ADJ_THREADS, 0, s>>>(d, lam_in, psum, T, lam_out);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    const long long lines[3] = {(long long)d.nj * d.nk, (long long)d.ni * d.nk, (long long)d.ni * d.nj};
    for (int axis = 0; axis < 3; ++axis) {
        wall_reverse_kernel<<<(unsigned)((lines[axis] + ADJ_THREADS - 1) / ADJ_THREADS), ADJ_THREADS, 0, s>>>(
            d, axis, lam_out, dthot);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_nusselt_seed(const Dims& d, double scale, StateT<double> lam, double* dthot, hipStream_t s)
{
    const long long n = (long long)d.ni * d.nj * d.nk;
    nusselt_seed_kernel<<<(unsigned)((n + ADJ_THREADS - 1) / ADJ_THREADS), ADJ_THREADS, 0, s>>>(d, scale, lam,
                                                                                               dthot);
    return hipGetLastError();
}

}  // namespace cav
