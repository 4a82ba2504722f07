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
//   2. record pass, per cell m (the forward sweep's k-marching tile, so the
//      stars come from LDS and registers): seeds a_f = lambda*_f dt for R_f
//      and b = sum_f lambda*_f R_f for dt, then the hand-written reverse of
//      the residual.  The cotangents of m's 41 star values are linear in a
//      few per-cell numbers -- a_u, a_v, a_w, a_T, eps4 a_p lambda_i/h_i
//      (three), beta^2 a_p and the centre terms of u, v, w -- which are
//      stored (11 doubles per cell); nu, alpha and the viscous step limit get
//      their cotangents reduced per block into the Ra cotangent;
//   3. gather pass, per cell e: lambda*(e) plus every star cotangent that
//      lands on e, rebuilt from the records of the cells whose stars reach e
//      (13 for p, 7 for u v w T) and their velocities; cells within two of a
//      wall add the transposed wall rules of the ghosts their neighbours read
//      (and the x = 0 wall rows add to dJ/dTheta).
// Every sum runs in a fixed order, so results are run-to-run identical.
#include "cavity_internal.h"
#include "stencil.h"
#include "sweep_tile.h"

#include <algorithm>

namespace cav {

namespace {

constexpr int NREC = 11;           // record values per cell
constexpr int ADJ_THREADS = 256;
enum { R_XX, R_XY, R_XZ, R_BP, R_UB, R_VB, R_WB, R_AU, R_AV, R_AW, R_AT };

// Reverse of cell_residual for one cell, reduced to its record: given the
// cotangents a[f] of R_f and b of dt, every star cotangent of the cell is
//   p:      centre -6 (Xx + Xy + Xz); at +-1 along x: -+a_u/(2h_x) + 4 Xx;
//           at +-2 along x: -Xx (y, z alike with a_v, a_w)
//   u:      centre ub + ctr nu a_u; at +-1 along x: -+(su a_u + Bp/(2h_x))
//           + nu a_u/h_x^2; along y: -+sv a_u + nu a_u/h_y^2; z alike
//   v, w:   likewise, with the Bp term along y for v and along z for w
//   T:      centre a_w + ctr alpha a_T; along each axis -+s a_T + alpha a_T/h^2
// with Xi = eps4 a_p lambda_i/h_i, Bp = beta^2 a_p, (su, sv, sw) = V/(2h),
// ctr = -2 sum 1/h^2, "-+" meaning - at +1 and + at -1.  rec receives
// Xx, Xy, Xz, Bp, ub, vb, wb, a_u, a_v, a_w, a_T; nub, alb, dtvb are the
// cotangents of nu, alpha and the viscous step limit.  Non-smooth points
// take one side: |u| has slope +1 at u = 0; beta^2 = max(|V|^2, floor)
// follows |V|^2 only where strictly larger; dt follows the convective limit
// only where strictly smaller than the viscous one.
__device__ __forceinline__ void reverse_record(const CoefR<double>& c, const Star<double>& s, const double a[NF],
                                               double b, double rec[NREC], double& nub, double& alb, double& dtvb)
{
    // ---- forward intermediates (same formulas as cell_residual) ----
    const double dxu = s.uxp - s.uxm, dyu = s.uyp - s.uym, dzu = s.uzp - s.uzm;
    const double dxv = s.vxp - s.vxm, dyv = s.vyp - s.vym, dzv = s.vzp - s.vzm;
    const double dxw = s.wxp - s.wxm, dyw = s.wyp - s.wym, dzw = s.wzp - s.wzm;
    const double dxt = s.txp - s.txm, dyt = s.typ - s.tym, dzt = s.tzp - s.tzm;
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

    // ---- reverse ----
    nub = (a[FU] * lap3(c, s.u, s.uxm, s.uxp, s.uym, s.uyp, s.uzm, s.uzp) +
           a[FV] * lap3(c, s.v, s.vxm, s.vxp, s.vym, s.vyp, s.vzm, s.vzp)) +
          a[FW] * lap3(c, s.w, s.wxm, s.wxp, s.wym, s.wyp, s.wzm, s.wzp);
    alb = a[FT] * lap3(c, s.t, s.txm, s.txp, s.tym, s.typ, s.tzm, s.tzp);
    // R_p = -beta^2 div - eps4 (lxn fx + lyn fy + lzn fz)
    double beta2b = -div * a[FP];
    const double dissb = -c.eps4 * a[FP];
    double lxnb = fx * dissb, lynb = fy * dissb, lznb = fz * dissb;
    // advection (su D_x f + sv D_y f + sw D_z f) enters R_f with sign -
    const double sub = -(((a[FU] * dxu + a[FV] * dxv) + a[FW] * dxw) + a[FT] * dxt);
    const double svb = -(((a[FU] * dyu + a[FV] * dyv) + a[FW] * dyw) + a[FT] * dyt);
    const double swb = -(((a[FU] * dzu + a[FV] * dzv) + a[FW] * dzw) + a[FT] * dzt);
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

    rec[R_XX] = -lxn * dissb;
    rec[R_XY] = -lyn * dissb;
    rec[R_XZ] = -lzn * dissb;
    rec[R_BP] = beta2 * a[FP];
    rec[R_UB] = ub;
    rec[R_VB] = vb;
    rec[R_WB] = wb;
    rec[R_AU] = a[FU];
    rec[R_AV] = a[FV];
    rec[R_AW] = a[FW];
    rec[R_AT] = a[FT];
}

__device__ __forceinline__ int centre_off(const Dims& d) { return cell_off(d, d.ni / 2, d.nj / 2, d.nk / 2); }

// ---- 1. sum of lambda_p over the interior, fixed order ----
// Stage 1: block b sums the interior cells of rows [b*rpb, (b+1)*rpb) (row
// = (j, k)), the threads striding over the group's cells with i fastest so
// that loads are coalesced; a fixed tree per block writes part[b].
__global__ __launch_bounds__(ADJ_THREADS) void row_sum_kernel(Dims d, int rpb, const double* __restrict__ lp,
                                                              double* __restrict__ part)
{
    __shared__ double red[ADJ_THREADS];
    const int t = threadIdx.x;
    const int rows = d.nj * d.nk;
    const int r0 = blockIdx.x * rpb, r1 = min(r0 + rpb, rows);
    double acc = 0.0;
    for (int r = r0; r < r1; ++r) {                      // uniform: row offsets in scalar registers
        const int o = cell_off(d, 0, r % d.nj, r / d.nj);
        for (int i = t; i < d.ni; i += ADJ_THREADS) acc += lp[o + i];
    }
    red[t] = acc;
    __syncthreads();
    for (int w = ADJ_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = red[0];
}

// Sum of part[b * stride] for b < n in a fixed order; out[0] = sum (or +=
// when accumulate).
__global__ __launch_bounds__(ADJ_THREADS) void sum_kernel(const double* __restrict__ part, int n, int stride,
                                                          double* out, int accumulate)
{
    __shared__ double red[ADJ_THREADS];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int b = t; b < n; b += ADJ_THREADS) acc += part[(size_t)b * stride];
    red[t] = acc;
    __syncthreads();
    for (int w = ADJ_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[0] = accumulate ? out[0] + red[0] : red[0];
}

// ---- 2. record pass ----
struct RaFactors {
    double nu, alpha, dtv;        // d(nu)/dRa, d(alpha)/dRa, d(dt_visc)/dRa
};

// What the k-marching tile does with each cell: seeds from lambda*, the
// reverse of the residual, the record stored at the cell's dense index, the
// Ra term into acc[0].
struct RecordEpi {
    CStateT<double> lam;
    const double* psum;
    double* rec;
    long long n;
    RaFactors rf;
    double ps;
    int centre;
    __device__ __forceinline__ void prepare(const Dims& d, const CStateT<double>&, const CoefR<double>&)
    {
        ps = psum[0];
        centre = centre_off(d);
    }
    __device__ __forceinline__ void cell(const CoefR<double>& c, const Star<double>& s, const double R[NF], double dt,
                                         int o, int i, int j, int k, double acc[NF], const Dims& d)
    {
        double a[NF], b = 0.0;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double ls = (f == FP && o == centre) ? lam.f[f][o] - ps : lam.f[f][o];
            a[f] = ls * dt;
            b = fma(ls, R[f], b);
        }
        double v[NREC], nub, alb, dtvb;
        reverse_record(c, s, a, b, v, nub, alb, dtvb);
        const long long idx = i + (long long)d.ni * (j + (long long)d.nj * k);
#pragma unroll
        for (int m = 0; m < NREC; ++m) rec[(size_t)m * n + idx] = v[m];
        acc[0] += (nub * rf.nu + alb * rf.alpha) + dtvb * rf.dtv;
    }
};

// Binds the grid to RecordEpi::cell (the tile passes no grid to its
// epilogue).
struct RecordEpiD {
    RecordEpi e;
    Dims d;
    __device__ __forceinline__ void prepare(const Dims& dd, const CStateT<double>& q, const CoefR<double>& c)
    {
        e.prepare(dd, q, c);
    }
    __device__ __forceinline__ void cell(const CoefR<double>& c, const Star<double>& s, const double R[NF], double dt,
                                         int o, int i, int j, int k, double acc[NF])
    {
        e.cell(c, s, R, dt, o, i, j, k, acc, d);
    }
};

__global__ __launch_bounds__(SW_TI * SW_TJ) void record_kernel(Dims d, Coef cd, SweepGeom g, RaFactors rf,
                                                               CStateT<double> q, CStateT<double> lam,
                                                               const double* psum, double* rec, double* partials)
{
    __shared__ SweepLds<double> L;
    const CoefR<double> c = coef_as<double>(cd);
    const TileBox tb = tile_box(d, g.tiles_i, g.tiles_j, g.kc, xcd_block(blockIdx.x, g.nblocks));
    RecordEpiD epi{{lam, psum, rec, (long long)d.ni * d.nj * d.nk, rf, 0.0, 0}, d};
    sweep_tile<double, true, OwnAll, RecordEpiD, 2>(d, c, tb, OwnAll{}, q, epi, partials, L);
}

// What the gather needs from a neighbour m one cell away along an axis:
// the four velocity/temperature seeds, that axis's dissipation term and Bp,
// and m's velocity along the axis times 1/(2h).
struct Nb {
    double au, av, aw, at, X, Bp, s;
};

// ---- 3. gather: lambda*(e) plus every star cotangent landing on e ----
__global__ __launch_bounds__(ADJ_THREADS) void adjoint_gather_kernel(Dims d, Coef cd, CStateT<double> q,
                                                                     CStateT<double> lam,
                                                                     const double* __restrict__ psum,
                                                                     const double* __restrict__ rec,
                                                                     StateT<double> out, double* __restrict__ dthot)
{
    const CoefR<double> c = coef_as<double>(cd);
    const long long n = (long long)d.ni * d.nj * d.nk;
    // Blocks go to the 8 XCDs round-robin; XCD x walks the rows j of its
    // slab [j0, j0 + w) plane after plane, so that the records a cell reads
    // from its y neighbours (adjacent rows) and z neighbours (the same rows
    // one plane away, w rows earlier) are in that XCD's L2.
    const int x = blockIdx.x & 7;
    const int j0 = (int)((long long)x * d.nj / 8);
    const int w = (int)((long long)(x + 1) * d.nj / 8) - j0;
    const long long cl = (long long)(blockIdx.x >> 3) * ADJ_THREADS + threadIdx.x;
    if (cl >= (long long)d.ni * w * d.nk) return;
    const int i = (int)(cl % d.ni);
    const long long r = cl / d.ni;
    const int j = j0 + (int)(r % w), k = (int)(r / w);
    const long long idx = i + (long long)d.ni * (j + (long long)d.nj * k);
    const int o = cell_off(d, i, j, k);
    auto R = [&](int v, long long m) { return rec[(size_t)v * n + m]; };
    const double ctr = -2.0 * ((c.ix2 + c.iy2) + c.iz2);
    const double nu = c.nu, al = c.alpha;

    // own record, and lambda* (the identity part of q + dt R)
    const double ps = psum[0];
    const bool is_centre = o == centre_off(d);
    const double Xe[3] = {R(R_XX, idx), R(R_XY, idx), R(R_XZ, idx)};
    const double Bpe = R(R_BP, idx);
    const double au = R(R_AU, idx), av = R(R_AV, idx), aw = R(R_AW, idx), at = R(R_AT, idx);
    double Lp = (is_centre ? lam.f[FP][o] - ps : lam.f[FP][o]) - 6.0 * ((Xe[0] + Xe[1]) + Xe[2]);
    double Lu = lam.f[FU][o] + (R(R_UB, idx) + ctr * nu * au);
    double Lv = lam.f[FV][o] + (R(R_VB, idx) + ctr * nu * av);
    double Lw = lam.f[FW][o] + (R(R_WB, idx) + ctr * nu * aw);
    double Lt = lam.f[FT][o] + (aw + ctr * al * at);

    // The x neighbours are the cells of the adjacent lanes (a wavefront holds
    // consecutive cells, i fastest): their record values and u arrive by
    // cross-lane moves, loads remain only at the wavefront's edges.  Every
    // lane moves before any branch; a lane whose neighbour is no cell of
    // this launch (it returned above) never uses the moved value.
    const int wl = threadIdx.x & 63;
    const double sh_in[7] = {au, av, aw, at, Xe[0], Bpe, q.f[FU][o]};
    double sh_lo[7], sh_hi[7];
#pragma unroll
    for (int v = 0; v < 7; ++v) {
        sh_lo[v] = __shfl_up(sh_in[v], 1, 64);
        sh_hi[v] = __shfl_down(sh_in[v], 1, 64);
    }
    const int pos[3] = {i, j, k};
    const int N[3] = {d.ni, d.nj, d.nk};
    const long long dstride[3] = {1, d.ni, (long long)d.ni * d.nj};
    const int pstride[3] = {1, d.sy, d.sz};
    const double h2[3] = {c.hx2, c.hy2, c.hz2};
    const double i2[3] = {c.ix2, c.iy2, c.iz2};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int x = pos[ax], nn = N[ax];
        const double H = h2[ax], I2 = i2[ax];
        const double* V = q.f[FU + ax];
        auto nb = [&](int sgn) {
            const long long m = idx + sgn * dstride[ax];
            Nb b;
            if (ax == 0 && (sgn < 0 ? wl > 0 : wl < 63)) {
                const double* S = sgn < 0 ? sh_lo : sh_hi;
                b.au = S[0]; b.av = S[1]; b.aw = S[2]; b.at = S[3]; b.X = S[4]; b.Bp = S[5];
                b.s = S[6] * H;
                return b;
            }
            b.au = R(R_AU, m);
            b.av = R(R_AV, m);
            b.aw = R(R_AW, m);
            b.at = R(R_AT, m);
            b.X = R(R_XX + ax, m);
            b.Bp = R(R_BP, m);
            b.s = V[o + sgn * pstride[ax]] * H;
            return b;
        };
        // the cotangents cell b's star puts on the cell one step from b in
        // direction dir (+1: up the axis, slot "+"; -1: slot "-")
        auto t7 = [&](const Nb& b, int dir, double& tu, double& tv, double& tw, double& tt, double& tp) {
            const double sg = dir > 0 ? -1.0 : 1.0;
            tp = sg * ((ax == 0 ? b.au : (ax == 1 ? b.av : b.aw)) * H) + 4.0 * b.X;
            tu = sg * (b.s * b.au + (ax == 0 ? H * b.Bp : 0.0)) + I2 * nu * b.au;
            tv = sg * (b.s * b.av + (ax == 1 ? H * b.Bp : 0.0)) + I2 * nu * b.av;
            tw = sg * (b.s * b.aw + (ax == 2 ? H * b.Bp : 0.0)) + I2 * nu * b.aw;
            tt = sg * (b.s * b.at) + I2 * al * b.at;
        };
        Nb lo{0, 0, 0, 0, 0, 0, 0}, hi{0, 0, 0, 0, 0, 0, 0};
        double tu, tv, tw, tt, tp;
        if (x > 0) {                      // the cell below reaches up to e
            lo = nb(-1);
            t7(lo, +1, tu, tv, tw, tt, tp);
            Lp += tp; Lu += tu; Lv += tv; Lw += tw; Lt += tt;
        }
        if (x < nn - 1) {                 // the cell above reaches down to e
            hi = nb(+1);
            t7(hi, -1, tu, tv, tw, tt, tp);
            Lp += tp; Lu += tu; Lv += tv; Lw += tw; Lt += tt;
        }
        if (x >= 2) Lp -= R(R_XX + ax, idx - 2 * dstride[ax]);
        if (x < nn - 2) Lp -= R(R_XX + ax, idx + 2 * dstride[ax]);

        // walls: ghosts g1, g2 beyond a wall carry the cotangents of the
        // stars that read them; the wall rules move them onto m0 (next to
        // the wall) and m1:  p: m0 += 2 g1 + 3 g2, m1 -= g1 + 2 g2;
        // u v w: m0 -= g1;  T: m0 -= g1 on x walls (and Theta += 2 g1 at
        // x = 0), m0 += g1 on the others.
        if (x <= 1 || x >= nn - 2) {
            const Nb me{au, av, aw, at, Xe[ax], Bpe, V[o] * H};
            for (int side = 0; side < 2; ++side) {
                const int dir = side ? +1 : -1;          // from m0 towards the wall
                const int m0 = side ? nn - 1 : 0, m1 = side ? nn - 2 : 1;
                if (x != m0 && x != m1) continue;
                const Nb& B0 = x == m0 ? me : (side ? hi : lo);          // m0 seen from e
                const double X1 = x == m1 ? Xe[ax] : (side ? lo.X : hi.X);   // m1's X
                // g1 collects m0's one-step and m1's two-step reach past the
                // wall, g2 m0's two-step reach
                t7(B0, dir, tu, tv, tw, tt, tp);
                const double g1p = tp - X1, g2p = -B0.X;
                if (x == m0) {
                    Lp += 2.0 * g1p + 3.0 * g2p;
                    Lu -= tu;
                    Lv -= tv;
                    Lw -= tw;
                    if (ax == 0) {
                        Lt -= tt;
                        if (side == 0 && dthot) dthot[j + (long long)d.nj * k] += 2.0 * tt;
                    } else {
                        Lt += tt;
                    }
                }
                if (x == m1) Lp -= g1p + 2.0 * g2p;
            }
        }
    }
    out.f[FP][o] = Lp;
    out.f[FU][o] = Lu;
    out.f[FV][o] = Lv;
    out.f[FW][o] = Lw;
    out.f[FT][o] = Lt;
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

// Partials of the record pass: one per block of any k-chunk tiling (the
// chunking never yields more than nk/CAV_MIN_KC chunks per tile column), NF each.
long long record_partials(const Dims& d)
{
    const long long tiles = (long long)((d.ni + SW_TI - 1) / SW_TI) * ((d.nj + SW_TJ - 1) / SW_TJ);
    return tiles * std::max(1, d.nk / CAV_MIN_KC) * NF;
}

}  // namespace

// ---------------------------------------------------------------------------
size_t adjoint_ws_doubles(const Dims& d)
{
    const long long n = (long long)d.ni * d.nj * d.nk;
    const long long rows = (long long)d.nj * d.nk;
    const long long part = std::max(std::min(rows, 1024LL), record_partials(d));
    return (size_t)(8 + (part + 7) / 8 * 8 + (long long)NREC * n);
}

hipError_t launch_adjoint_step(const Dims& d, const Coef& c, const SweepGeom& g, double Ra, CStateT<double> q,
                               CStateT<double> lam_in, StateT<double> lam_out, double* ws, double* dthot,
                               double* dra, hipStream_t s)
{
    const long long n = (long long)d.ni * d.nj * d.nk;
    const long long rows = (long long)d.nj * d.nk;
    double* psum = ws;                       // ws[0]: sum of lambda_p
    double* part = ws + 8;
    const long long np = std::max(std::min(rows, 1024LL), record_partials(d));
    double* rec = part + (np + 7) / 8 * 8;
    if ((long long)g.nblocks * NF > np) return hipErrorInvalidValue;
    // about 1024 blocks of whole rows, at most one per partial slot
    const int rpb = (int)std::max(1LL, (rows + 1023) / 1024);
    const int rb = (int)((rows + rpb - 1) / rpb);
    if (rb > np) return hipErrorInvalidValue;
    hipError_t e;

    row_sum_kernel<<<rb, ADJ_THREADS, 0, s>>>(d, rpb, lam_in.f[FP], part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    sum_kernel<<<1, ADJ_THREADS, 0, s>>>(part, rb, 1, psum, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    RaFactors rf;
    rf.nu = -c.nu / (2.0 * Ra);
    rf.alpha = -c.alpha / (2.0 * Ra);
    rf.dtv = c.dt_visc / (2.0 * Ra);
    record_kernel<<<g.nblocks, dim3(SW_TI, SW_TJ), 0, s>>>(d, c, g, rf, q, lam_in, psum, rec, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (dra) {
        sum_kernel<<<1, ADJ_THREADS, 0, s>>>(part, g.nblocks, NF, dra, 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // 8 j slabs (one per XCD), as many blocks for each as the widest needs
    const long long wmax = (d.nj + 7) / 8;
    const long long per_xcd = ((long long)d.ni * wmax * d.nk + ADJ_THREADS - 1) / ADJ_THREADS;
    adjoint_gather_kernel<<<(unsigned)(8 * per_xcd), ADJ_THREADS, 0, s>>>(d, c, q, lam_in, psum, rec, lam_out,
                                                                         dthot);
    return hipGetLastError();
}

hipError_t launch_nusselt_seed(const Dims& d, double scale, StateT<double> lam, double* dthot, hipStream_t s)
{
    const long long n = (long long)d.ni * d.nj * d.nk;
    nusselt_seed_kernel<<<(unsigned)((n + ADJ_THREADS - 1) / ADJ_THREADS), ADJ_THREADS, 0, s>>>(d, scale, lam,
                                                                                               dthot);
    return hipGetLastError();
}

}  // namespace cav
