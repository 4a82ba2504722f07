// Discrete adjoint (reverse mode) of one pseudo-time step and of the mean
// hot-wall Nusselt number, in FP64.
//
// One step maps the state q^n to q^{n+1} (Sec. 2, Eq. 1-3): wall ghosts G
// from the interior cells and the hot-wall temperatures Theta, per cell the
// residual R(S) and local step dt(S) of its stars S, q* = q + dt R, and the
// pressure rescale p^{n+1} = p* - p*(centre).  Given the cotangent lambda of
// q^{n+1}, the reverse step returns the cotangent of q^n and adds the
// cotangents of Theta and of Ra:
//   1. the transpose of the rescale: lambda*_p(centre) = lambda_p(centre) -
//      S, S the sum over cells of lambda_p; lambda* = lambda elsewhere;
//   2. record pass, per cell m (the forward sweep's k-marching tile, so the
//      stars come from LDS and registers): seeds a_f = lambda_f dt for R_f
//      and b = sum_f lambda_f R_f for dt, then the hand-written reverse of
//      the residual.  The cotangents of m's 41 star values are linear in a
//      few per-cell numbers -- a_u .. a_T (lambda_f dt), eps4 a_p
//      lambda_i/h_i (three), beta^2 a_p, dt and the centre terms of u, v, w.
//      Only the last three depend on m's star; the rest follow from m's
//      velocity and lambda.  The pass stores 8 (dt, the three dissipation
//      terms, Bp and the centre terms) or, for the LDS tile gather, only
//      the 3 centre terms; nu, alpha and the viscous step limit get their
//      cotangents reduced per block into partials of the Ra cotangent, and
//      each block sums its lambda_p.  Everything is linear in the seeds, so
//      the centre cell is seeded with lambda_p like the others and also
//      stores its centre terms and Ra term for a unit p seed;
//   3. gather pass, per cell e: lambda*(e) plus every star cotangent that
//      lands on e, rebuilt from the records of the cells whose stars reach e
//      (13 for p, 7 for u v w T), their velocities and lambda; cells within
//      two of a wall add the transposed wall rules of the ghosts their
//      neighbours read (and the x = 0 wall rows add to dJ/dTheta).  The
//      cells that read the centre form S from the record blocks' partials
//      and take the centre's values for lambda*_p (the unit seed's terms
//      times S subtracted); the one holding the centre adds the Ra sum.
// Every sum runs in a fixed order, so results are run-to-run identical.
#include "cavity_internal.h"
#include "stencil.h"
#include "sweep_tile.h"

#include <algorithm>

namespace cav {

namespace {

constexpr int NREC = 8;            // record values per cell (full record)
constexpr int NREC_C = 3;          // the compact record: ub, vb, wb
constexpr int ADJ_THREADS = 256;
// Gather: rows (wavefronts) per block of the LDS tile kernel, and the
// shortest k chunk it is used for (shorter chunks take the one-cell-per-
// thread kernel, whose start-up is a single load per value).
#ifndef CAV_ADJ_GATHER_TJ
#define CAV_ADJ_GATHER_TJ 8
#endif
constexpr int ADJ_GTJ = CAV_ADJ_GATHER_TJ;
#ifndef CAV_ADJ_TILE_MIN_KC
#define CAV_ADJ_TILE_MIN_KC 8
#endif
enum { R_UB, R_VB, R_WB, R_DT, R_XX, R_XY, R_XZ, R_BP };

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
// ub, vb, wb, Xx, Xy, Xz, Bp (the caller adds dt: a_u .. a_T are lambda_f dt,
// rebuilt from lambda where they are needed; dt, the X and Bp depend only on
// the cell's velocity and lambda*_p, see cell_d); nub, alb, dtvb are the
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
}

// The part of a cell's record that depends only on its velocity and
// lambda*_p: dt, the dissipation terms Xx, Xy, Xz and Bp, by the formulas of
// cell_residual and reverse_record, so the values are the same bits as the
// record pass's.
struct CellD {
    double dt, X[3], Bp;
};
__device__ __forceinline__ CellD cell_d(const CoefR<double>& c, double u, double v, double w, double lps)
{
    const double u2 = u * u, v2 = v * v, w2 = w * w;
    const double beta2 = fmax((u2 + v2) + w2, c.beta2_floor);
    const double b4 = 4.0 * beta2;
    const double lxn = (fabs(u) + sqrt_pos(u2 + b4)) * c.hx2;
    const double lyn = (fabs(v) + sqrt_pos(v2 + b4)) * c.hy2;
    const double lzn = (fabs(w) + sqrt_pos(w2 + b4)) * c.hz2;
    CellD D;
    D.dt = c.cfl * fmin(recip_pos((lxn + lyn) + lzn), c.dt_visc);
    const double ap = lps * D.dt;
    const double dissb = -c.eps4 * ap;
    D.X[0] = -lxn * dissb;
    D.X[1] = -lyn * dissb;
    D.X[2] = -lzn * dissb;
    D.Bp = beta2 * ap;
    return D;
}

__device__ __forceinline__ int centre_off(const Dims& d) { return cell_off(d, d.ni / 2, d.nj / 2, d.nk / 2); }

// ---- 2. record pass ----
struct RaFactors {
    double nu, alpha, dtv;        // d(nu)/dRa, d(alpha)/dRa, d(dt_visc)/dRa
};

// What the k-marching tile does with each cell: seeds from lambda, the
// reverse of the residual, the record stored at the cell's dense index, the
// Ra term into acc[0] and lambda_p into acc[1] (the block's share of the
// sum S of lambda_p).  The transpose of the centre rescale seeds the centre
// cell with lambda*_p = lambda_p - S instead, and S is known only after
// the pass; the record and the Ra term are linear in the seeds, so the
// centre cell also stores ub, vb, wb and the Ra term of a unit p seed
// (a_p = dt, b = R_p) at cx[0..3], and the gather subtracts S times them.
// COMPACT: store only ub, vb, wb (the LDS tile gather forms the rest from
// the cell's velocity and lambda, cell_d); else the full record.
template <bool COMPACT>
struct RecordEpi {
    CStateT<double> lam;
    double* rec;
    long long n;
    RaFactors rf;
    double* cx;
    int centre;
    __device__ __forceinline__ void prepare(const Dims& d, const CStateT<double>&, const CoefR<double>&)
    {
        centre = centre_off(d);
    }
    __device__ __forceinline__ void cell(const CoefR<double>& c, const Star<double>& s, const double R[NF], double dt,
                                         int o, int i, int j, int k, double acc[NF], const Dims& d)
    {
        double a[NF], b = 0.0;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double l = lam.f[f][o];
            a[f] = l * dt;
            b = fma(l, R[f], b);
            if (f == FP) acc[1] += l;
        }
        double v[NREC], nub, alb, dtvb;
        reverse_record(c, s, a, b, v, nub, alb, dtvb);
        v[R_DT] = dt;
        const long long idx = i + (long long)d.ni * (j + (long long)d.nj * k);
        // streaming stores: the record (24 or 64 B per cell) is read back
        // only by the gather, after the whole pass
#pragma unroll
        for (int m = 0; m < (COMPACT ? NREC_C : NREC); ++m)
            __builtin_nontemporal_store(v[m], &rec[(size_t)m * n + idx]);
        acc[0] += (nub * rf.nu + alb * rf.alpha) + dtvb * rf.dtv;
        if (o == centre) {
            const double ae[NF] = {dt, 0.0, 0.0, 0.0, 0.0};
            double ve[NREC], nue, ale, dte;
            reverse_record(c, s, ae, R[FP], ve, nue, ale, dte);
            cx[0] = ve[R_UB];
            cx[1] = ve[R_VB];
            cx[2] = ve[R_WB];
            cx[3] = (nue * rf.nu + ale * rf.alpha) + dte * rf.dtv;
        }
    }
};

// Binds the grid to RecordEpi::cell (the tile passes no grid to its
// epilogue).
template <bool COMPACT>
struct RecordEpiD {
    RecordEpi<COMPACT> e;
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

template <bool COMPACT>
__global__ __launch_bounds__(SW_TI * SW_TJ) void record_kernel(Dims d, Coef cd, SweepGeom g, RaFactors rf,
                                                               CStateT<double> q, CStateT<double> lam, double* rec,
                                                               double* partials, double* cx)
{
    __shared__ SweepLds<double> L;
    const CoefR<double> c = coef_as<double>(cd);
    const TileBox tb = tile_box(d, g.tiles_i, g.tiles_j, g.kc, xcd_block(blockIdx.x, g.nblocks));
    RecordEpiD<COMPACT> epi{{lam, rec, (long long)d.ni * d.nj * d.nk, rf, cx, -1}, d};
    sweep_tile<double, true, OwnAll, RecordEpiD<COMPACT>, 2>(d, c, tb, OwnAll{}, q, epi, partials, L);
}

// The record pass's per-block partials (the Ra term, the sum of lambda_p)
// and the centre's unit p seed terms cx.  sums() forms, in one whole
// wavefront, the rescale sum S (every block's lambda_p partial) and the Ra
// cotangent of the step: every block's Ra partial minus S times the unit
// seed's Ra term, cx[3].  Lane l adds blocks l, l + 64, ... in order, then a
// butterfly over the lanes: IEEE addition commutes, so every lane, and every
// wavefront that calls it, gets the same bits.  All 64 lanes must be
// active.
struct CentreTerms {
    const double* part;
    int nblocks;
    const double* cx;
    __device__ __forceinline__ void sums(double& S, double& ra) const
    {
        double a = 0.0, b = 0.0;
        for (int k = threadIdx.x & 63; k < nblocks; k += 64) {
            b += part[(size_t)k * NF];
            a += part[(size_t)k * NF + 1];
        }
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) {
            a += __shfl_xor(a, m, 64);
            b += __shfl_xor(b, m, 64);
        }
        S = a;
        ra = b - a * cx[3];
    }
};

// What the gather needs from a neighbour m one cell away along an axis:
// the four velocity/temperature seeds, that axis's dissipation term and Bp,
// and m's velocity along the axis times 1/(2h).
struct Nb {
    double au, av, aw, at, X, Bp, s;
};

// ---- 3. gather: lambda*(e) plus every star cotangent landing on e ----
// The per-cell arithmetic, shared by the two gather kernels (which differ
// only in where the neighbours' records come from), so both give the same
// bits.  Accumulation order: lambda* and e's own terms, then the axes x, y,
// z, each with its -1 and +1 neighbours' stars, the fourth-difference
// terms of the cells two away, and the transposed wall rules.
struct GatherAcc {
    double Lp, Lu, Lv, Lw, Lt;
};

// lam: lambda at e (lam*, the cotangent e's record was seeded from, is
// lambda except the centre cell's p, minus the rescale sum); ub, vb, wb and
// D: e's record.  e's seeds a_u .. a_T are lambda_f dt, the product the
// record pass formed.
__device__ __forceinline__ GatherAcc gather_init(const CoefR<double>& c, const double lam[NF], bool is_centre, double ps,
                                                 double ub, double vb, double wb, const CellD& D)
{
    const double ctr = -2.0 * ((c.ix2 + c.iy2) + c.iz2);
    const double au = lam[FU] * D.dt, av = lam[FV] * D.dt, aw = lam[FW] * D.dt;
    const double at = lam[FT] * D.dt;
    GatherAcc a;
    a.Lp = (is_centre ? lam[FP] - ps : lam[FP]) - 6.0 * ((D.X[0] + D.X[1]) + D.X[2]);
    a.Lu = lam[FU] + (ub + ctr * c.nu * au);
    a.Lv = lam[FV] + (vb + ctr * c.nu * av);
    a.Lw = lam[FW] + (wb + ctr * c.nu * aw);
    a.Lt = lam[FT] + (aw + ctr * c.alpha * at);
    return a;
}

// Axis ax of cell e at coordinate x of nn: the neighbours lo (x-1) and hi
// (x+1) where they exist, the dissipation terms Xm2, Xp2 of the cells two
// away where they exist, and e itself (me) for the wall rules.  dth: the
// dJ/dTheta slot of e's wall row (x = 0 on the i axis), or NULL.
__device__ __forceinline__ void gather_axis(GatherAcc& a, const CoefR<double>& c, int ax, int x, int nn,
                                            const Nb& lo, const Nb& hi, double Xm2, double Xp2, const Nb& me,
                                            double* dth)
{
    const double H = ax == 0 ? c.hx2 : (ax == 1 ? c.hy2 : c.hz2);
    const double I2 = ax == 0 ? c.ix2 : (ax == 1 ? c.iy2 : c.iz2);
    const double nu = c.nu, al = c.alpha;
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
    double tu, tv, tw, tt, tp;
    if (x > 0) {                      // the cell below reaches up to e
        t7(lo, +1, tu, tv, tw, tt, tp);
        a.Lp += tp; a.Lu += tu; a.Lv += tv; a.Lw += tw; a.Lt += tt;
    }
    if (x < nn - 1) {                 // the cell above reaches down to e
        t7(hi, -1, tu, tv, tw, tt, tp);
        a.Lp += tp; a.Lu += tu; a.Lv += tv; a.Lw += tw; a.Lt += tt;
    }
    if (x >= 2) a.Lp -= Xm2;
    if (x < nn - 2) a.Lp -= Xp2;

    // walls: ghosts g1, g2 beyond a wall carry the cotangents of the
    // stars that read them; the wall rules move them onto m0 (next to
    // the wall) and m1:  p: m0 += 2 g1 + 3 g2, m1 -= g1 + 2 g2;
    // u v w: m0 -= g1;  T: m0 -= g1 on x walls (and Theta += 2 g1 at
    // x = 0), m0 += g1 on the others.
    if (x <= 1 || x >= nn - 2) {
        for (int side = 0; side < 2; ++side) {
            const int dir = side ? +1 : -1;          // from m0 towards the wall
            const int m0 = side ? nn - 1 : 0, m1 = side ? nn - 2 : 1;
            if (x != m0 && x != m1) continue;
            const Nb& B0 = x == m0 ? me : (side ? hi : lo);          // m0 seen from e
            const double X1 = x == m1 ? me.X : (side ? lo.X : hi.X);  // m1's X
            // g1 collects m0's one-step and m1's two-step reach past the
            // wall, g2 m0's two-step reach
            t7(B0, dir, tu, tv, tw, tt, tp);
            const double g1p = tp - X1, g2p = -B0.X;
            if (x == m0) {
                a.Lp += 2.0 * g1p + 3.0 * g2p;
                a.Lu -= tu;
                a.Lv -= tv;
                a.Lw -= tw;
                if (ax == 0) {
                    a.Lt -= tt;
                    if (side == 0 && dth) *dth += 2.0 * tt;
                } else {
                    a.Lt += tt;
                }
            }
            if (x == m1) a.Lp -= g1p + 2.0 * g2p;
        }
    }
}

// NT: non-temporal stores (the output is not read again by this pass)
template <bool NT = false>
__device__ __forceinline__ void gather_store(const GatherAcc& a, StateT<double>& out, int o)
{
    const double v[NF] = {a.Lp, a.Lu, a.Lv, a.Lw, a.Lt};
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        if (NT) __builtin_nontemporal_store(v[f], &out.f[f][o]);
        else out.f[f][o] = v[f];
    }
}

// One cell per thread.  Blocks go to the 8 XCDs round-robin; XCD x walks
// the rows j of its slab [j0, j0 + w) plane after plane, so that the
// records a cell reads from its y neighbours (adjacent rows) are in that
// XCD's L2.  (Its z neighbours' records, a slab-plane away, mostly are not:
// the blocks in flight on an XCD span more than its L2 holds.)
__global__ __launch_bounds__(ADJ_THREADS) void adjoint_gather_kernel(Dims d, Coef cd, CStateT<double> q,
                                                                     CStateT<double> lam, CentreTerms ct,
                                                                     const double* __restrict__ rec,
                                                                     StateT<double> out, double* __restrict__ dthot,
                                                                     double* __restrict__ dra)
{
    const CoefR<double> c = coef_as<double>(cd);
    const long long n = (long long)d.ni * d.nj * d.nk;
    const int x = blockIdx.x & 7;
    const int j0 = (int)((long long)x * d.nj / 8);
    const int w = (int)((long long)(x + 1) * d.nj / 8) - j0;
    const long long cl = (long long)(blockIdx.x >> 3) * ADJ_THREADS + threadIdx.x;
    const bool in = cl < (long long)d.ni * w * d.nk;
    const long long cc = in ? cl : 0;
    const int i = (int)(cc % d.ni);
    const long long r = cc / d.ni;
    const int j = j0 + (int)(r % w), k = (int)(r / w);
    const int ci = d.ni / 2, cj = d.nj / 2, ck = d.nk / 2;
    const long long idx = i + (long long)d.ni * (j + (long long)d.nj * k);
    const int o = cell_off(d, i, j, k);
    const int centre = centre_off(d);
    auto R = [&](int v, long long m) { return rec[(size_t)v * n + m]; };
    double own[NREC_C];
#pragma unroll
    for (int v = 0; v < NREC_C; ++v) own[v] = R(v, idx);
    double lm[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) lm[f] = lam.f[f][o];
    // The rescale sum S, in every wavefront holding a cell within two of the
    // centre (the cells that read the centre's seeds); the wavefront holding
    // the centre adds the Ra term.  Every lane is still active here (lanes
    // past the end loaded a real cell and return below).
    double S = 0.0;
    if (__any(in && abs(i - ci) <= 2 && abs(j - cj) <= 2 && abs(k - ck) <= 2)) {
        double ra;
        ct.sums(S, ra);
        if (dra && __any(in && i == ci && j == cj && k == ck) && (threadIdx.x & 63) == 0) dra[0] += ra;
    }
    if (!in) return;
    // dt, X and Bp of the cell at state offset om, dense index m: its record,
    // or at the centre formed from lambda*_p (its record holds lambda_p's)
    auto dxb = [&](long long m, int om) {
        if (om == centre) return cell_d(c, q.f[FU][om], q.f[FV][om], q.f[FW][om], lam.f[FP][om] - S);
        return CellD{R(R_DT, m), {R(R_XX, m), R(R_XY, m), R(R_XZ, m)}, R(R_BP, m)};
    };

    const CellD od = dxb(idx, o);
    const bool isc = o == centre;
    if (isc) {
        own[R_UB] -= S * ct.cx[0];
        own[R_VB] -= S * ct.cx[1];
        own[R_WB] -= S * ct.cx[2];
    }
    GatherAcc a = gather_init(c, lm, isc, S, own[R_UB], own[R_VB], own[R_WB], od);
    const double au = lm[FU] * od.dt, av = lm[FV] * od.dt, aw = lm[FW] * od.dt;
    const double at = lm[FT] * od.dt;

    // The x neighbours are the cells of the adjacent lanes (a wavefront holds
    // consecutive cells, i fastest): their seeds, record values and u arrive
    // by cross-lane moves, loads remain only at the wavefront's edges.  Every
    // lane moves before any branch; a lane whose neighbour is no cell of
    // this launch (it returned above) never uses the moved value.
    const int wl = threadIdx.x & 63;
    const double sh_in[7] = {au, av, aw, at, od.X[0], od.Bp, q.f[FU][o]};
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
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int xx = pos[ax], nn = N[ax];
        const double H = ax == 0 ? c.hx2 : (ax == 1 ? c.hy2 : c.hz2);
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
            const int on = o + sgn * pstride[ax];
            const CellD D = dxb(m, on);
            b.au = lam.f[FU][on] * D.dt;
            b.av = lam.f[FV][on] * D.dt;
            b.aw = lam.f[FW][on] * D.dt;
            b.at = lam.f[FT][on] * D.dt;
            b.X = D.X[ax];
            b.Bp = D.Bp;
            b.s = V[on] * H;
            return b;
        };
        Nb lo{0, 0, 0, 0, 0, 0, 0}, hi{0, 0, 0, 0, 0, 0, 0};
        if (xx > 0) lo = nb(-1);
        if (xx < nn - 1) hi = nb(+1);
        const double Xm2 = xx >= 2 ? dxb(idx - 2 * dstride[ax], o - 2 * pstride[ax]).X[ax] : 0.0;
        const double Xp2 = xx < nn - 2 ? dxb(idx + 2 * dstride[ax], o + 2 * pstride[ax]).X[ax] : 0.0;
        const Nb me{au, av, aw, at, od.X[ax], od.Bp, V[o] * H};
        gather_axis(a, c, ax, xx, nn, lo, hi, Xm2, Xp2, me,
                    (ax == 0 && dthot) ? &dthot[j + (long long)d.nj * k] : nullptr);
    }
    gather_store(a, out, o);
}

// One cell's compact record, cotangent and velocity, and the rest of its
// record formed from them, as the k queue of the tile kernel holds it.
struct Column {
    double ub, vb, wb;                 // the cell's compact record
    double l[NF - 1];                  // lambda_u .. lambda_T (the seeds a_u .. a_T are lambda_f dt)
    double lp;                         // lambda_p
    double u, v, w;                    // its velocity
    CellD D;                           // dt, the dissipation terms, Bp (cell_d)
};

// The gather as a k-marching LDS tile over the compact record: a block of
// 64 x TJ threads marches its (i, j) columns through a k chunk.  Each cell's
// dt, dissipation terms and Bp are formed once, from its velocity and
// lambda_p (cell_d), when its plane enters the k queue two planes ahead.
// Each plane, every thread puts the ten values its in-plane neighbours need
// (lambda_u .. lambda_T and dt, whose products are the seeds, Bp, the x and
// y dissipation terms, u, v) into the plane's LDS buffer, the block's
// threads together add the tile's halo (two rows above and below, two
// columns left and right; a halo thread loads a cell's velocity and
// lambda_p and forms what the halo needs of them, or loads its lambda_u ..
// lambda_T), and after one barrier every cell reads its x and y neighbours
// from LDS; its z neighbours (one and two planes away) are the k queue.  So
// every value is read from memory once per tile, plus the halo.  Two LDS
// buffers alternate between planes: the barrier of plane k+1 orders its
// writes after every read of plane k-1's buffer.  Every thread runs every
// plane (no early exit), so the barriers are uniform.
enum { L_LU, L_LV, L_LW, L_LT, L_DT, L_BP, L_XX, L_XY, L_U, L_V, NLV };

template <int TJ>
struct GatherTile {
    static constexpr int THREADS = 64 * TJ;
    static constexpr int COLS = 68, ROWS = TJ + 4;            // two halo columns / rows on each side
    static constexpr int BUF = NLV * ROWS * COLS;             // doubles per plane buffer
    static constexpr int VS = ROWS * COLS;                    // stride between the values of a cell
    // halo slots per plane, four loads each: rows -1 and TJ (velocity +
    // lambda_p, and lambda_u .. lambda_T), rows -2 and TJ+1 (velocity +
    // lambda_p, for the y dissipation term), columns -1 and 64 (both kinds),
    // columns -2 and 65 (velocity + lambda_p, for the x dissipation term)
    static constexpr int NH = 2 * 2 * 64 + 2 * 64 + 2 * 2 * TJ + 2 * TJ;
    static constexpr int SLOTS = (NH + THREADS - 1) / THREADS;
    __device__ static int at(int v, int row, int col) { return (v * ROWS + row + 2) * COLS + col + 2; }
};

template <int TJ>
__global__ __launch_bounds__(64 * TJ) void adjoint_gather_tile_kernel(Dims d, Coef cd, SweepGeom g,
                                                                      CStateT<double> q, CStateT<double> lam,
                                                                      CentreTerms ct,
                                                                      const double* __restrict__ rec,
                                                                      StateT<double> out,
                                                                      double* __restrict__ dthot,
                                                                      double* __restrict__ dra)
{
    using T = GatherTile<TJ>;
    static_assert(T::SLOTS == 1, "one halo slot per thread");
    __shared__ double L[2 * T::BUF];
    const CoefR<double> c = coef_as<double>(cd);
    const TileBox tb = tile_box<64, TJ>(d, g.tiles_i, g.tiles_j, g.kc, xcd_block(blockIdx.x, g.nblocks));
    const int lane = threadIdx.x, row = threadIdx.y, tid = lane + 64 * row;
    const int i = tb.i0 + lane, j = tb.j0 + row;
    // threads past the grid load a real cell (clamped), take part in every
    // barrier, and store nothing; no cell of the grid reads their slots
    const bool active = i < d.ni && j < d.nj;
    const int ic = min(i, d.ni - 1), jc = min(j, d.nj - 1);
    const long long n = (long long)d.ni * d.nj * d.nk;
    const long long plane = (long long)d.ni * d.nj;
    const long long col = ic + (long long)d.ni * jc;
    const int ocol = cell_off(d, ic, jc, 0);
    const int Z = d.sz;
    const int centre = centre_off(d);
    const int ci = d.ni / 2, cj = d.nj / 2, ck = d.nk / 2;
    // The rescale sum S, in blocks whose cells or halo reach the centre
    // (every wavefront forms it); the wavefront holding the centre adds the
    // Ra term.
    double ps = 0.0;
    if (ci >= tb.i0 - 2 && ci < tb.i0 + 66 && cj >= tb.j0 - 2 && cj < tb.j0 + TJ + 2 && ck >= tb.k0 - 2 &&
        ck < tb.k1 + 2) {
        double ra;
        ct.sums(ps, ra);
        if (dra && ci >= tb.i0 && ci < tb.i0 + 64 && cj == j && ck >= tb.k0 && ck < tb.k1 && lane == 0) dra[0] += ra;
    }
    // lambda*_p of the cell at state offset o
    auto lstar = [&](double lp, int o) { return o == centre ? lp - ps : lp; };

    // this thread's halo slot: kind (-1: none or outside the grid; 0:
    // velocity + lambda_p at rows/columns -1 and edge; 1: the same at -2 and
    // edge+1, for the dissipation term only; 2: lambda_u .. lambda_T), the
    // cell's state offset at k = 0, its LDS position (value 0), and whether
    // it is a row (y) or a column (x) of the halo
    int hkind = -1, hoff = 0, hpos = 0;
    bool hrow = true;
    {
        int h = tid, hr = 0, hc = 0, kind = -1;
        if (h < 2 * 2 * 64) {                       // rows -1 and TJ
            kind = h / (2 * 64) ? 2 : 0;
            const int r = h % (2 * 64);
            hc = r % 64; hr = r / 64 ? TJ : -1;
        } else if ((h -= 2 * 2 * 64) < 2 * 64) {    // rows -2 and TJ+1
            kind = 1; hc = h % 64; hr = h / 64 ? TJ + 1 : -2;
        } else if ((h -= 2 * 64) < 2 * 2 * TJ) {    // columns -1 and 64
            kind = h / (2 * TJ) ? 2 : 0;
            const int r = h % (2 * TJ);
            hr = r % TJ; hc = r / TJ ? 64 : -1;
            hrow = false;
        } else if ((h -= 2 * 2 * TJ) < 2 * TJ) {    // columns -2 and 65
            kind = 1; hr = h % TJ; hc = h / TJ ? 65 : -2;
            hrow = false;
        }
        const int hi_ = tb.i0 + hc, hj = tb.j0 + hr;
        if (kind >= 0 && hi_ >= 0 && hi_ < d.ni && hj >= 0 && hj < d.nj) {
            hkind = kind;
            hoff = cell_off(d, hi_, hj, 0);
            hpos = T::at(0, hr, hc);
        }
    }
    // the halo slot's four values of one plane
    struct Halo {
        double v[4];
    };
    auto load_halo = [&](int k, Halo& H) {
        const int o = hoff + k * Z;
        if (hkind == 2) {
#pragma unroll
            for (int f = FU; f <= FT; ++f) H.v[f - FU] = lam.f[f][o];
        } else if (hkind >= 0) {
            H.v[0] = q.f[FU][o];
            H.v[1] = q.f[FV][o];
            H.v[2] = q.f[FW][o];
            H.v[3] = lam.f[FP][o];
        }
    };
    // a velocity + lambda_p slot's values, formed in place (one plane
    // before they are stored): the dissipation term across the halo, dt,
    // Bp and the velocity component across it
    auto form_halo = [&](int k, Halo& H) {
        if (hkind == 0 || hkind == 1) {
            const CellD D = cell_d(c, H.v[0], H.v[1], H.v[2], lstar(H.v[3], hoff + k * Z));
            const double V = hrow ? H.v[1] : H.v[0];
            H.v[0] = hrow ? D.X[1] : D.X[0];
            H.v[1] = D.dt;
            H.v[2] = D.Bp;
            H.v[3] = V;
        }
    };
    // what the slot puts into the plane's buffer B
    auto store_halo = [&](const Halo& H, double* B) {
        if (hkind == 2) {
#pragma unroll
            for (int f = 0; f < 4; ++f) B[hpos + (L_LU + f) * T::VS] = H.v[f];
        } else if (hkind >= 0) {
            B[hpos + (hrow ? L_XY : L_XX) * T::VS] = H.v[0];
            if (hkind == 0) {
                B[hpos + L_DT * T::VS] = H.v[1];
                B[hpos + L_BP * T::VS] = H.v[2];
                B[hpos + (hrow ? L_V : L_U) * T::VS] = H.v[3];
            }
        }
    };

    auto R = [&](int v, long long m) { return rec[(size_t)v * n + m]; };
    // the compact record, velocity and lambda_p of plane k
    auto load = [&](int k, Column& C) {
        const long long m = col + k * plane;
        const int o = ocol + k * Z;
        C.ub = R(R_UB, m);
        C.vb = R(R_VB, m);
        C.wb = R(R_WB, m);
        C.u = q.f[FU][o];
        C.v = q.f[FV][o];
        C.w = q.f[FW][o];
        C.lp = lam.f[FP][o];
    };
    auto load_l = [&](int k, Column& C) {
#pragma unroll
        for (int f = FU; f <= FT; ++f) C.l[f - FU] = lam.f[f][ocol + k * Z];
    };
    auto derive = [&](int k, Column& C) { C.D = cell_d(c, C.u, C.v, C.w, lstar(C.lp, ocol + k * Z)); };
    const int k0 = tb.k0, k1 = tb.k1, nk = d.nk;
    const double Hx = c.hx2, Hy = c.hy2, Hz = c.hz2;
    Nb prv{0, 0, 0, 0, 0, 0, 0};
    double xm2 = 0.0;
    if (k0 >= 2) {
        const int om = ocol + (k0 - 2) * Z;
        xm2 = cell_d(c, q.f[FU][om], q.f[FV][om], q.f[FW][om], lstar(lam.f[FP][om], om)).X[2];
    }
    if (k0 >= 1) {
        const int om = ocol + (k0 - 1) * Z;
        const CellD D = cell_d(c, q.f[FU][om], q.f[FV][om], q.f[FW][om], lstar(lam.f[FP][om], om));
        prv = Nb{lam.f[FU][om] * D.dt, lam.f[FV][om] * D.dt, lam.f[FW][om] * D.dt, lam.f[FT][om] * D.dt, D.X[2],
                 D.Bp, q.f[FW][om] * Hz};
    }
    // Three register sets of planes (records and halo) rotate through the
    // roles k, k+1, k+2, so that no set is copied while its loads are in
    // flight: each set's compact record, velocity and lambda_p are loaded
    // three planes before it is the current one, at the same time as the
    // neighbouring tiles load that plane's cells, and formed into its dt, X
    // and Bp two planes before; its lambda_u .. lambda_T are loaded two
    // planes before (a value in flight holds its register; they are issued
    // before the further plane's record, so waiting for them does not wait
    // for it).
    Column C0, C1, C2;
    Halo H0, H1, H2;
    load(k0, C0);
    load_l(k0, C0);
    load_halo(k0, H0);
    if (k0 + 1 < nk) {
        load(k0 + 1, C1);
        load_l(k0 + 1, C1);
    }
    if (k0 + 1 < k1) load_halo(k0 + 1, H1);
    if (k0 + 2 < nk) load(k0 + 2, C2);
    if (k0 + 2 < k1) load_halo(k0 + 2, H2);
    derive(k0, C0);
    if (k0 + 1 < nk) derive(k0 + 1, C1);
    form_halo(k0, H0);

    // plane k: cur = plane k, nxt = k+1, nn2 = k+2 (its dt, X and Bp are
    // formed here; only its z dissipation term is read); H = plane k's
    // halo, Hn = plane k+1's (formed here); cur and H are reloaded with
    // plane k+3 once used
    auto body = [&](int k, Column& cur, Column& nxt, Column& nn2, Halo& H, Halo& Hn) __attribute__((always_inline)) {
        double* B = L + ((k - k0) & 1) * T::BUF;
        {
            const double own[NLV] = {cur.l[0], cur.l[1], cur.l[2], cur.l[3], cur.D.dt,
                                     cur.D.Bp, cur.D.X[0], cur.D.X[1], cur.u, cur.v};
#pragma unroll
            for (int v = 0; v < NLV; ++v) B[T::at(v, row, lane)] = own[v];
        }
        store_halo(H, B);
        if (k + 3 < k1) load_halo(k + 3, H);
        __syncthreads();

        const int o = ocol + k * Z;
        const double lm[NF] = {cur.lp, cur.l[0], cur.l[1], cur.l[2], cur.l[3]};
        const bool isc = o == centre;
        // the centre's record holds lambda_p's terms; lambda*_p's differ by
        // S times the unit p seed's
        const double ub = isc ? cur.ub - ps * ct.cx[0] : cur.ub;
        const double vb = isc ? cur.vb - ps * ct.cx[1] : cur.vb;
        const double wb = isc ? cur.wb - ps * ct.cx[2] : cur.wb;
        GatherAcc a = gather_init(c, lm, isc, ps, ub, vb, wb, cur.D);
        const double dt = cur.D.dt;
        const double au = cur.l[0] * dt, av = cur.l[1] * dt, aw = cur.l[2] * dt, at = cur.l[3] * dt;
        // the neighbour at (row, col) of the plane's buffer, with its x (or y)
        // dissipation term X and velocity V
        auto nbl = [&](int r, int cl, int X, int V, double H) {
            const double dm = B[T::at(L_DT, r, cl)];
            return Nb{B[T::at(L_LU, r, cl)] * dm, B[T::at(L_LV, r, cl)] * dm, B[T::at(L_LW, r, cl)] * dm,
                      B[T::at(L_LT, r, cl)] * dm, B[T::at(X, r, cl)], B[T::at(L_BP, r, cl)], B[T::at(V, r, cl)] * H};
        };
        auto nbx = [&](int dc) { return nbl(row, lane + dc, L_XX, L_U, Hx); };
        auto nby = [&](int dr) { return nbl(row + dr, lane, L_XY, L_V, Hy); };
        {
            const Nb lo = i > 0 ? nbx(-1) : Nb{0, 0, 0, 0, 0, 0, 0};
            const Nb hi = i < d.ni - 1 ? nbx(+1) : Nb{0, 0, 0, 0, 0, 0, 0};
            const double Xm2 = i >= 2 ? B[T::at(L_XX, row, lane - 2)] : 0.0;
            const double Xp2 = i < d.ni - 2 ? B[T::at(L_XX, row, lane + 2)] : 0.0;
            const Nb me{au, av, aw, at, cur.D.X[0], cur.D.Bp, cur.u * Hx};
            gather_axis(a, c, 0, i, d.ni, lo, hi, Xm2, Xp2, me,
                        (dthot && active) ? &dthot[j + (long long)d.nj * k] : nullptr);
        }
        {
            const Nb lo = j > 0 ? nby(-1) : Nb{0, 0, 0, 0, 0, 0, 0};
            const Nb hi = j < d.nj - 1 ? nby(+1) : Nb{0, 0, 0, 0, 0, 0, 0};
            const double Xm2 = j >= 2 ? B[T::at(L_XY, row - 2, lane)] : 0.0;
            const double Xp2 = j < d.nj - 2 ? B[T::at(L_XY, row + 2, lane)] : 0.0;
            const Nb me{au, av, aw, at, cur.D.X[1], cur.D.Bp, cur.v * Hy};
            gather_axis(a, c, 1, j, d.nj, lo, hi, Xm2, Xp2, me, nullptr);
        }
        if (k + 2 < nk) derive(k + 2, nn2);
        {
            const double dn = nxt.D.dt;
            const Nb hi = k < nk - 1 ? Nb{nxt.l[0] * dn, nxt.l[1] * dn, nxt.l[2] * dn, nxt.l[3] * dn,
                                          nxt.D.X[2], nxt.D.Bp, nxt.w * Hz}
                                     : Nb{0, 0, 0, 0, 0, 0, 0};
            const double Xp2 = k < nk - 2 ? nn2.D.X[2] : 0.0;
            const Nb me{au, av, aw, at, cur.D.X[2], cur.D.Bp, cur.w * Hz};
            gather_axis(a, c, 2, k, nk, k > 0 ? prv : Nb{0, 0, 0, 0, 0, 0, 0}, hi, k >= 2 ? xm2 : 0.0, Xp2, me,
                        nullptr);
        }
        if (active) gather_store<true>(a, out, o);
        if (k + 1 < k1) form_halo(k + 1, Hn);

        xm2 = prv.X;
        prv = Nb{au, av, aw, at, cur.D.X[2], cur.D.Bp, cur.w * Hz};
        // plane k+2's lambda_u .. lambda_T (from iteration k+1 on, as its
        // k+1), plane k+3's record (from iteration k+1 on, as its k+2)
        if (k + 2 < nk && k + 1 < k1) load_l(k + 2, nn2);
        if (k + 3 < nk && k + 1 < k1) load(k + 3, cur);
    };
    for (int k = k0; k < k1; k += 3) {
        body(k, C0, C1, C2, H0, H1);
        if (k + 1 < k1) body(k + 1, C1, C2, C0, H1, H2);
        if (k + 2 < k1) body(k + 2, C2, C0, C1, H2, H0);
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

// Partials of the record pass: one per block of any k-chunk tiling (the
// chunking never yields more than nk/CAV_MIN_KC chunks per tile column),
// NF each.
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
    return (size_t)(8 + (record_partials(d) + 7) / 8 * 8 + (long long)NREC * n);
}

hipError_t launch_adjoint_step(const Dims& d, const Coef& c, const SweepGeom& g, const SweepGeom& gg, double Ra,
                               CStateT<double> q, CStateT<double> lam_in, StateT<double> lam_out, double* ws,
                               double* dthot, double* dra, hipStream_t s)
{
    double* cx = ws;                         // ws[0..3]: the centre's unit p seed terms
    double* part = ws + 8;
    const long long np = record_partials(d);
    double* rec = part + (np + 7) / 8 * 8;
    if ((long long)g.nblocks * NF > np) return hipErrorInvalidValue;
    hipError_t e;

    RaFactors rf;
    rf.nu = -c.nu / (2.0 * Ra);
    rf.alpha = -c.alpha / (2.0 * Ra);
    rf.dtv = c.dt_visc / (2.0 * Ra);
    // the LDS tile gather reads the compact record, the one-cell gather the
    // full one
    const bool tile = gg.kc >= CAV_ADJ_TILE_MIN_KC;
    // every cell's record (the centre's seeded with lambda_p, plus its unit
    // p seed terms in cx); each block's Ra term and sum of lambda_p
    if (tile) record_kernel<true><<<g.nblocks, dim3(SW_TI, SW_TJ), 0, s>>>(d, c, g, rf, q, lam_in, rec, part, cx);
    else record_kernel<false><<<g.nblocks, dim3(SW_TI, SW_TJ), 0, s>>>(d, c, g, rf, q, lam_in, rec, part, cx);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the gather, with the rescale sum and the Ra cotangent's sum
    const CentreTerms ct{part, g.nblocks, cx};
    if (tile) {
        adjoint_gather_tile_kernel<ADJ_GTJ><<<gg.nblocks, dim3(64, ADJ_GTJ), 0, s>>>(d, c, gg, q, lam_in, ct, rec,
                                                                                 lam_out, dthot, dra);
    } else {
        // 8 j slabs (one per XCD), as many blocks for each as the widest needs
        const long long wmax = (d.nj + 7) / 8;
        const long long per_xcd = ((long long)d.ni * wmax * d.nk + ADJ_THREADS - 1) / ADJ_THREADS;
        adjoint_gather_kernel<<<(unsigned)(8 * per_xcd), ADJ_THREADS, 0, s>>>(d, c, q, lam_in, ct, rec, lam_out,
                                                                             dthot, dra);
    }
    return hipGetLastError();
}

SweepGeom gather_geom(const Dims& d, int cus)
{
    static int per_cu = 0;
    if (per_cu == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, adjoint_gather_tile_kernel<ADJ_GTJ>, 64 * ADJ_GTJ, 0) !=
                hipSuccess ||
            n < 1)
            n = 1;
        per_cu = n;
    }
    return sweep_geom(d, cus * per_cu, 64, ADJ_GTJ);
}

hipError_t launch_nusselt_seed(const Dims& d, double scale, StateT<double> lam, double* dthot, hipStream_t s)
{
    const long long n = (long long)d.ni * d.nj * d.nk;
    nusselt_seed_kernel<<<(unsigned)((n + ADJ_THREADS - 1) / ADJ_THREADS), ADJ_THREADS, 0, s>>>(d, scale, lam,
                                                                                               dthot);
    return hipGetLastError();
}

}  // namespace cav
