// Residual + Euler-update sweep kernels (single cavity, interior/exterior
// split, batched), wall boundary conditions, seeded init, the hot-wall
// Nusselt integral and the residual-norm finalize for gfx950, in FP64 and
// FP32 (the per-cell code is in stencil.h, the k-marching tile in
// sweep_tile.h).
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
#include "sweep_tile.h"

namespace cav {

// Tile of the step sweep: FP64 64 x 8 (eight wavefronts; at its register
// count one block per compute unit), FP32 32 x 8 (four wavefronts; three
// resident blocks per compute unit, whose barriers interleave).
template <typename Real>
struct StepTile {
    static constexpr int TI = sizeof(Real) == 4 ? F32_TI : F64_TI;
    static constexpr int TJ = sizeof(Real) == 4 ? F32_TJ : F64_TJ;
    static constexpr int THREADS = TI * TJ;
    // minimum waves per SIMD the compiler must fit (0: its own choice)
    static constexpr int MINW = sizeof(Real) == 4 ? 0 : CAV_F64_STEP_WAVES;
    // planes of loads in flight ahead of the computed plane
    static constexpr int DEPTH = sizeof(Real) == 4 ? 3 : CAV_F64_STEP_DEPTH;
};

// The step's epilogue with the i-face part of the next exchange's pack
// (Sec. 4.5: the noncontiguous faces that "Optimized V1" packs), for splits
// along i only: a lane whose column lies within a face width of a cut also
// stores the new values of its cell at their places in the halo buffer (the
// layout of halo_pack), so the next step needs no pack kernel.  The values
// stored are the very ones written to the new state.  Needs every subdomain
// extent along i >= 2 x the largest width, so that a column lies in at most
// one face box.
struct XPackGeom {
    int ex, pi;          // subdomain extent along i, subdomains along i
    int nj;              // face rows per plane (the split is along i only)
    int area;            // face area nj * nk
    int wsum;
    int w[NF], wpre[NF];
};

template <typename Real>
struct StepXPackEpi : StepEpi<Real> {
    Real* buf;
    int dd;          // distance of the column to its cut (< the largest width), or -1: no face
    int face;        // 0: the -i face of the column's subdomain, 1: its +i face
    int seg;         // element offset of that face's segment in the buffer
    XPackGeom x;

    __device__ __forceinline__ void init(const Dims& d, int i)
    {
        dd = -1;
        if (i >= d.ni) return;
        int wmax = 0;
#pragma unroll
        for (int f = 0; f < NF; ++f) wmax = max(wmax, x.w[f]);
        const int a = i / x.ex;
        const int lo = i - a * x.ex, hi = x.ex - 1 - lo;
        if (a > 0 && lo < wmax) { face = 0; dd = lo; }
        else if (a < x.pi - 1 && hi < wmax) { face = 1; dd = hi; }
        // segments in subdomain order, -i before +i face (buffer layout):
        // subdomain 0 has only its +i face, the others both (the last one
        // only its -i face)
        seg = (a > 0 ? 2 * a - 1 + face : 0) * x.area * x.wsum;
    }
    __device__ __forceinline__ void cell(const CoefR<Real>&, const Star<Real>& s, const Real R[NF], Real dt, int o,
                                         int, int j, int k, double acc[NF])
    {
        const Real nv[NF] = {fma(dt, R[FP], s.p) - this->pc_new, fma(dt, R[FU], s.u), fma(dt, R[FV], s.v),
                             fma(dt, R[FW], s.w), fma(dt, R[FT], s.t)};
#pragma unroll
        for (int f = 0; f < NF; ++f) __builtin_nontemporal_store(nv[f], &this->qn.f[f][o]);
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] = fma((double)R[f], (double)R[f], acc[f]);
        if (dd < 0) return;
        const int row = k * x.nj + j;              // (k, j) index on the face
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int w = x.w[f];
            if (dd < w) buf[seg + x.wpre[f] * x.area + row * w + (face ? w - 1 - dd : dd)] = nv[f];
        }
    }
};

// FIELD = false: the hot wall is the scalar t_hot, known at compile time to
// need no field loads (the kernel the uniform-wall problem runs).  XP: the
// epilogue also packs the i faces of the new state into xbuf (geometry xh).
template <typename Real, bool NORM, bool FIELD, bool XP>
__global__ __launch_bounds__(StepTile<Real>::THREADS, StepTile<Real>::MINW) void sweep_kernel(
    Dims d, Coef cd, SweepGeom g, CStateT<Real> q, StateT<Real> qn, double* partials, XPackGeom xg, Real* xbuf)
{
    constexpr int TI = StepTile<Real>::TI, TJ = StepTile<Real>::TJ;
    __shared__ SweepLds<Real, TI, TJ> L;
    CoefR<Real> c = coef_as<Real>(cd);
    if constexpr (!FIELD) c.t_hot_field = nullptr;
    const TileBox tb = tile_box<TI, TJ>(d, g.tiles_i, g.tiles_j, g.kc, xcd_block(blockIdx.x, g.nblocks));
    if constexpr (XP) {
        StepXPackEpi<Real> epi;
        epi.qn = qn;
        epi.pc_new = Real(0);
        epi.x = xg;
        epi.buf = xbuf;
        const int tid = threadIdx.x + SW_TI * threadIdx.y;
        epi.init(d, tb.i0 + tid % TI);
        sweep_tile<Real, NORM, OwnAll, StepXPackEpi<Real>, StepTile<Real>::DEPTH, TI, TJ>(d, c, tb, OwnAll{}, q, epi,
                                                                                         partials, L);
    } else {
        StepEpi<Real> epi{qn, Real(0)};
        sweep_tile<Real, NORM, OwnAll, StepEpi<Real>, StepTile<Real>::DEPTH, TI, TJ>(d, c, tb, OwnAll{}, q, epi,
                                                                                    partials, L);
    }
}

// The step sweep's memory streams without its work: the same tiles, block
// order, k chunks and prefetch depth, and per interior cell the five fields
// read once and written once (non-temporal) -- no halo loads, no LDS, no
// arithmetic.  Its rate is the ceiling of the sweep's access pattern on the
// device it runs on.
template <typename Real>
__global__ __launch_bounds__(StepTile<Real>::THREADS) void stream_copy_kernel(Dims d, SweepGeom g, CStateT<Real> q,
                                                                              StateT<Real> qn)
{
    constexpr int TI = StepTile<Real>::TI, TJ = StepTile<Real>::TJ, DEPTH = StepTile<Real>::DEPTH;
    const TileBox tb = tile_box<TI, TJ>(d, g.tiles_i, g.tiles_j, g.kc, xcd_block(blockIdx.x, g.nblocks));
    const int tid = threadIdx.x + SW_TI * threadIdx.y;
    const int i = tb.i0 + tid % TI, j = tb.j0 + tid / TI;
    if (i >= d.ni || j >= d.nj) return;
    const int o0 = cell_off(d, i, j, 0), Z = d.sz;
    Real v[DEPTH][NF];
#pragma unroll
    for (int s = 0; s < DEPTH; ++s)
        if (tb.k0 + s < tb.k1)
#pragma unroll
            for (int f = 0; f < NF; ++f) v[s][f] = q.f[f][o0 + (tb.k0 + s) * Z];
    for (int k = tb.k0; k < tb.k1; k += DEPTH) {
#pragma unroll
        for (int s = 0; s < DEPTH; ++s) {
            if (k + s < tb.k1) {
                const int o = o0 + (k + s) * Z;
#pragma unroll
                for (int f = 0; f < NF; ++f) __builtin_nontemporal_store(v[s][f], &qn.f[f][o]);
                if (k + s + DEPTH < tb.k1)
#pragma unroll
                    for (int f = 0; f < NF; ++f) v[s][f] = q.f[f][o + DEPTH * Z];
            }
        }
    }
}

template <typename Real>
hipError_t launch_stream_copy(const Dims& d, const SweepGeom& g, CStateT<Real> q, StateT<Real> qn, hipStream_t s)
{
    dim3 block(SW_TI, StepTile<Real>::THREADS / SW_TI), grid(g.nblocks);
    stream_copy_kernel<Real><<<grid, block, 0, s>>>(d, g, q, qn);
    return hipGetLastError();
}
template hipError_t launch_stream_copy<double>(const Dims&, const SweepGeom&, CStateT<double>, StateT<double>,
                                               hipStream_t);
template hipError_t launch_stream_copy<float>(const Dims&, const SweepGeom&, CStateT<float>, StateT<float>,
                                              hipStream_t);

// The sweep's square root and reciprocal (stencil.h) on an array: out[2m] =
// sqrt_pos(x[m]), out[2m+1] = recip_pos(x[m]).
__global__ __launch_bounds__(256) void math_kernel(const double* __restrict__ x, double* __restrict__ out, int n)
{
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= n) return;
    out[2 * m] = sqrt_pos(x[m]);
    out[2 * m + 1] = recip_pos(x[m]);
}

hipError_t launch_math(const double* x, double* out, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    math_kernel<<<(n + 255) / 256, 256, 0, s>>>(x, out, n);
    return hipGetLastError();
}

SweepGeom sweep_geom(const Dims& d, int slots, int ti, int tj)
{
    SweepGeom g;
    g.tiles_i = (d.ni + ti - 1) / ti;
    g.tiles_j = (d.nj + tj - 1) / tj;
    const int tiles = g.tiles_i * g.tiles_j;
    // Split the k columns into nkc chunks so that the launch finishes
    // earliest: blocks run in rounds of `slots` (the blocks resident at
    // once), a block costs its planes plus ~3 planes of start-up
    // (the queue and halo planes it loads before its first plane).
    const int overhead = 3;
    long long best_cost = -1;
    int best = 1;
    const int max_nkc = max(1, d.nk / CAV_MIN_KC);
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
SweepGeom step_geom(const Dims& d, int cus)
{
    // resident blocks per compute unit of the step kernel (registers and LDS
    // decide it); the same for every launch on this device
    static int per_cu = 0;
    if (per_cu == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_kernel<Real, false, false, false>,
                                                         StepTile<Real>::THREADS, 0) != hipSuccess ||
            n < 1)
            n = 1;
        per_cu = n;
    }
    return sweep_geom(d, cus * per_cu, StepTile<Real>::TI, StepTile<Real>::TJ);
}
template SweepGeom step_geom<double>(const Dims&, int);
template SweepGeom step_geom<float>(const Dims&, int);

// g comes from step_geom<Real>.  xh, xbuf: the i-face pack in the epilogue
// (both NULL: none; never with the norm pass).
template <typename Real>
hipError_t launch_sweep(const Dims& d, const Coef& c, const SweepGeom& g, CStateT<Real> q, StateT<Real> qn,
                        double* partials, bool with_norm, hipStream_t s, const HaloGeom* xh, Real* xbuf)
{
    dim3 block(SW_TI, StepTile<Real>::THREADS / SW_TI), grid(g.nblocks);
    XPackGeom xg{};
    const bool xp = xh && xbuf && !with_norm;
    if (xp) {
        xg.ex = xh->e[0];
        xg.pi = xh->P[0];
        xg.nj = d.nj;
        xg.area = (int)xh->area[0];
        xg.wsum = xh->wsum;
        for (int f = 0; f < NF; ++f) {
            xg.w[f] = xh->w[f];
            xg.wpre[f] = xh->wpre[f];
        }
    }
    if (c.t_hot_field) {
        if (with_norm)
            sweep_kernel<Real, true, true, false><<<grid, block, 0, s>>>(d, c, g, q, qn, partials, xg, nullptr);
        else if (xp)
            sweep_kernel<Real, false, true, true><<<grid, block, 0, s>>>(d, c, g, q, qn, partials, xg, xbuf);
        else
            sweep_kernel<Real, false, true, false><<<grid, block, 0, s>>>(d, c, g, q, qn, partials, xg, nullptr);
    } else {
        if (with_norm)
            sweep_kernel<Real, true, false, false><<<grid, block, 0, s>>>(d, c, g, q, qn, partials, xg, nullptr);
        else if (xp)
            sweep_kernel<Real, false, false, true><<<grid, block, 0, s>>>(d, c, g, q, qn, partials, xg, xbuf);
        else
            sweep_kernel<Real, false, false, false><<<grid, block, 0, s>>>(d, c, g, q, qn, partials, xg, nullptr);
    }
    return hipGetLastError();
}
template hipError_t launch_sweep<double>(const Dims&, const Coef&, const SweepGeom&, CStateT<double>,
                                         StateT<double>, double*, bool, hipStream_t, const HaloGeom*, double*);
template hipError_t launch_sweep<float>(const Dims&, const Coef&, const SweepGeom&, CStateT<float>,
                                        StateT<float>, double*, bool, hipStream_t, const HaloGeom*, float*);

// ---------------------------------------------------------------------------
// Interior/exterior split (Sec. 4.7): with a halo exchange in the step, the
// cells whose stars reach no cell the unpack writes (the interior) are
// updated by one launch that may run while the exchange is in flight; the
// rest (the exterior: cells within `m` of a cut) by a second launch after
// it.  Each cell is computed by exactly one launch with the same per-cell
// code as the unsplit sweep, so the new state is bit-identical to it.

// Tile shape of the exterior x slabs (2m <= 8 owned columns).
constexpr int XS_TI = 16, XS_TJ = 32;

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

// The interior launch runs the step sweep's tile of its type (g from
// step_geom<Real>).
template <typename Real, bool NORM, bool FIELD>
__global__ __launch_bounds__(StepTile<Real>::THREADS) void interior_kernel(Dims d, Coef cd, SweepGeom g, SplitGeom sg,
                                                                           CStateT<Real> q, StateT<Real> qn,
                                                                           double* partials, int)
{
    constexpr int TI = StepTile<Real>::TI, TJ = StepTile<Real>::TJ;
    __shared__ SweepLds<Real, TI, TJ> L;
    CoefR<Real> c = coef_as<Real>(cd);
    if constexpr (!FIELD) c.t_hot_field = nullptr;
    const TileBox tb = tile_box<TI, TJ>(d, g.tiles_i, g.tiles_j, g.kc, xcd_block(blockIdx.x, g.nblocks));
    StepEpi<Real> epi{qn, Real(0)};
    sweep_tile<Real, NORM, OwnInterior, StepEpi<Real>, StepTile<Real>::DEPTH, TI, TJ>(d, c, tb, OwnInterior{sg}, q,
                                                                                     epi, partials, L);
}

// Exterior work items, block b: first the x slabs (per cut: 16 x 32 tiles,
// j tiles x k chunks of kce planes), then the y slabs (per cut: i tiles x k
// chunks), then the z slabs (per cut: i x j tiles, the 2m planes around the
// cut).
// Norm partials follow the interior launch's, at pidx = pidx0 + b (pidx0:
// the interior launch's block count).  g: the 64 x 8 tiling (sweep_geom).
template <typename Real, bool NORM, bool FIELD>
__global__ __launch_bounds__(SW_TI * SW_TJ) void exterior_kernel(Dims d, Coef cd, SweepGeom g, SplitGeom sg,
                                                                 CStateT<Real> q, StateT<Real> qn,
                                                                 double* partials, int pidx0)
{
    __shared__ union {
        SweepLds<Real> yz;                       // 64 x 8 tiles for the y and z slabs
        SweepLds<Real, XS_TI, XS_TJ> x;          // 16 x 32 tiles for the x slabs
    } L;
    CoefR<Real> c = coef_as<Real>(cd);
    if constexpr (!FIELD) c.t_hot_field = nullptr;
    const int b = blockIdx.x;
    const int nkce = (d.nk + sg.kce - 1) / sg.kce;
    const int tjx = (d.nj + XS_TJ - 1) / XS_TJ;
    const int per0 = tjx * nkce, per1 = g.tiles_i * nkce, per2 = g.tiles_i * g.tiles_j;
    const int n0 = (sg.P[0] - 1) * per0, n1 = (sg.P[1] - 1) * per1;
    TileBox tb;
    int axis, cut;
    if (b < n0) {
        axis = 0;
        const int r = b % per0;
        cut = (b / per0 + 1) * sg.e[0];
        tb.i0 = cut - sg.m;
        tb.j0 = (r % tjx) * XS_TJ;
        tb.k0 = (r / tjx) * sg.kce;
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
    tb.pidx = pidx0 + b;
    StepEpi<Real> epi{qn, Real(0)};
    if (axis == 0)          // 2m <= 8 owned columns: a narrow tile wastes fewer lanes
        sweep_tile<Real, NORM, OwnSlab, StepEpi<Real>, 3, XS_TI, XS_TJ>(d, c, tb, OwnSlab{sg, axis, cut}, q, epi,
                                                                      partials, L.x);
    else
        sweep_tile<Real, NORM>(d, c, tb, OwnSlab{sg, axis, cut}, q, epi, partials, L.yz);
}

int exterior_blocks(const Dims& d, const SweepGeom& g, const SplitGeom& sg)
{
    const int nkce = (d.nk + sg.kce - 1) / sg.kce;
    return (sg.P[0] - 1) * ((d.nj + XS_TJ - 1) / XS_TJ) * nkce + (sg.P[1] - 1) * g.tiles_i * nkce +
           (sg.P[2] - 1) * g.tiles_i * g.tiles_j;
}

// gi: the interior launch's geometry (step_geom<Real>); g: the 64 x 8 tiling
// the exterior slabs are decoded from (sweep_geom).
template <typename Real>
hipError_t launch_split(const Dims& d, const Coef& c, const SweepGeom& gi, const SweepGeom& g, const SplitGeom& sg,
                        bool exterior, CStateT<Real> q, StateT<Real> qn, double* partials, bool with_norm,
                        hipStream_t s)
{
    const dim3 block = exterior ? dim3(SW_TI, SW_TJ) : dim3(SW_TI, StepTile<Real>::THREADS / SW_TI);
    const SweepGeom& gl = exterior ? g : gi;
    const int nb = exterior ? exterior_blocks(d, g, sg) : gi.nblocks;
    const int pidx0 = gi.nblocks;
    if (nb == 0) return hipSuccess;
    const bool fld = c.t_hot_field != nullptr;
#define SPLIT_LAUNCH(K)                                                                                       \
    do {                                                                                                      \
        if (fld) {                                                                                            \
            if (with_norm) K<Real, true, true><<<nb, block, 0, s>>>(d, c, gl, sg, q, qn, partials, pidx0);     \
            else K<Real, false, true><<<nb, block, 0, s>>>(d, c, gl, sg, q, qn, partials, pidx0);              \
        } else {                                                                                              \
            if (with_norm) K<Real, true, false><<<nb, block, 0, s>>>(d, c, gl, sg, q, qn, partials, pidx0);    \
            else K<Real, false, false><<<nb, block, 0, s>>>(d, c, gl, sg, q, qn, partials, pidx0);             \
        }                                                                                                     \
    } while (0)
    if (exterior)
        SPLIT_LAUNCH(exterior_kernel);
    else
        SPLIT_LAUNCH(interior_kernel);
#undef SPLIT_LAUNCH
    return hipGetLastError();
}
template hipError_t launch_split<double>(const Dims&, const Coef&, const SweepGeom&, const SweepGeom&,
                                         const SplitGeom&, bool, CStateT<double>, StateT<double>, double*, bool,
                                         hipStream_t);
template hipError_t launch_split<float>(const Dims&, const Coef&, const SweepGeom&, const SweepGeom&,
                                        const SplitGeom&, bool, CStateT<float>, StateT<float>, double*, bool,
                                        hipStream_t);

// ---------------------------------------------------------------------------
// Batched form: a persistent grid walks the work list of all members; each
// item is one tile column's k chunk of one member, computed by the same
// sweep_tile as the single-cavity sweep.  `parity` selects which of q and
// q_tmp holds the current state of every member.
template <typename Real>
struct BatchTiles {
    static constexpr bool F32 = sizeof(Real) == 4;
    static constexpr int THREADS = batch_threads(F32);
    static constexpr int WTI = batch_wide_ti(F32), WTJ = batch_tj(F32, WTI);
    static constexpr int NTI = batch_narrow_ti(F32), NTJ = batch_tj(F32, NTI);
    // prefetch depth: the FP64 kernel would spill a third register set
    static constexpr int DEPTH = F32 ? 3 : 2;
    // waves per SIMD the one-shape FP32 kernels must fit (three 256-thread
    // blocks per CU, as the FP32 step sweep; 0: the compiler's choice)
    static constexpr int MINW1 = F32 ? 3 : 0;
};

// The item walk of one block: with at least BATCH_SEGS blocks, block b
// (on XCD b % 8) takes every (blocks on its XCD)-th item of segment b % 8;
// with fewer blocks, block b walks whole segments b, b + gridDim.x, ...
template <typename F>
__device__ __forceinline__ void for_each_item(const int* __restrict__ segs, F&& body)
{
    const int G = gridDim.x, b = blockIdx.x;
    if (G >= BATCH_SEGS) {
        const int s = b % BATCH_SEGS, lb = b / BATCH_SEGS;
        const int nbs = (G - s + BATCH_SEGS - 1) / BATCH_SEGS;      // blocks on segment s
        for (int it = segs[s] + lb; it < segs[s + 1]; it += nbs) body(it);
    } else {
        for (int s = b; s < BATCH_SEGS; s += G)
            for (int it = segs[s]; it < segs[s + 1]; ++it) body(it);
    }
}

// SHAPES: 3 = each member's tile shape (both compiled in: the registers of
// the larger, two blocks per CU in FP32), 1 = the wide shape only, 2 = the
// narrow one only (one shape: three blocks per CU in FP32).
template <typename Real, bool NORM, int SHAPES>
__global__ __launch_bounds__(BatchTiles<Real>::THREADS, SHAPES == 3 ? 0 : BatchTiles<Real>::MINW1) void batch_kernel(
    const BatchCav* __restrict__ cavs, const int* __restrict__ segs, const BatchItem* __restrict__ items, int parity)
{
    using BT = BatchTiles<Real>;
    using Wide = SweepLds<Real, BT::WTI, BT::WTJ>;
    using Narrow = SweepLds<Real, BT::NTI, BT::NTJ>;
    __shared__ union {
        Wide wide;
        Narrow narrow;
    } L;
    for_each_item(segs, [&](int it) {
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
        StepEpi<Real> epi{qn, Real(0)};
        if (SHAPES == 2 || (SHAPES == 3 && cv.ti == BT::NTI)) {
            const TileBox tb = tile_box<BT::NTI, BT::NTJ>(d, cv.tiles_i, cv.tiles_j, cv.kc, w.tile);
            sweep_tile<Real, NORM, OwnAll, StepEpi<Real>, BT::DEPTH, BT::NTI, BT::NTJ>(
                d, c, tb, OwnAll{}, qs, epi, cv.ws + WS_HEAD_DOUBLES, L.narrow);
        } else {
            const TileBox tb = tile_box<BT::WTI, BT::WTJ>(d, cv.tiles_i, cv.tiles_j, cv.kc, w.tile);
            sweep_tile<Real, NORM, OwnAll, StepEpi<Real>, BT::DEPTH, BT::WTI, BT::WTJ>(
                d, c, tb, OwnAll{}, qs, epi, cv.ws + WS_HEAD_DOUBLES, L.wide);
        }
        __syncthreads();                  // LDS is reused by the next item
    });
}

template <typename Real>
hipError_t launch_batch(const BatchCav* cavs, const int* segs, const BatchItem* items, int parity, bool with_norm,
                        int nblocks, int shapes, hipStream_t s)
{
    dim3 block(SW_TI, BatchTiles<Real>::THREADS / SW_TI), grid(nblocks);
#define BATCH_LAUNCH(SH)                                                                      \
    do {                                                                                      \
        if (with_norm) batch_kernel<Real, true, SH><<<grid, block, 0, s>>>(cavs, segs, items, parity);  \
        else batch_kernel<Real, false, SH><<<grid, block, 0, s>>>(cavs, segs, items, parity);           \
    } while (0)
    if (shapes == 1) BATCH_LAUNCH(1);
    else if (shapes == 2) BATCH_LAUNCH(2);
    else BATCH_LAUNCH(3);
#undef BATCH_LAUNCH
    return hipGetLastError();
}
template hipError_t launch_batch<double>(const BatchCav*, const int*, const BatchItem*, int, bool, int, int,
                                         hipStream_t);
template hipError_t launch_batch<float>(const BatchCav*, const int*, const BatchItem*, int, bool, int, int,
                                        hipStream_t);

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
