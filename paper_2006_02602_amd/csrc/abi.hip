// Host side of the C ABI declared in include/cavity.h: argument checks (pure
// host code, run before anything is enqueued), launch geometry, the step
// loop, error reporting and the optional per-kernel event timing.
#include "cavity.h"
#include "cavity_internal.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace cav;

// Scratch of cavity_step_noalloc: 5 FP64 norm partials per sweep block, for
// up to CAV_NOALLOC_MAX_SWEEP_BLOCKS blocks (1.25 MiB).  One copy per device,
// held until the process ends; every call on a device shares it.
constexpr int NOALLOC_MAX_BLOCKS = CAV_NOALLOC_MAX_SWEEP_BLOCKS;
static __device__ __align__(256) double scratch[(size_t)NOALLOC_MAX_BLOCKS * NF];

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

// ---- per-kernel event timing ---------------------------------------------
struct TimeRec {
    const char* name;
    hipEvent_t a, b;
};
std::atomic<bool> g_timing{false};
std::mutex g_tm;
std::vector<TimeRec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event()
{
    std::lock_guard<std::mutex> lk(g_tm);
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <class F>
hipError_t run(const char* name, hipStream_t s, F&& launch)
{
    if (!g_timing.load(std::memory_order_relaxed)) return launch();
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_tm);
    g_recs.push_back({name, a, b});
    return e;
}

int hip_fail(const char* what, hipError_t e)
{
    return fail(CAV_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---- argument checks ------------------------------------------------------
int elem_size(int dtype) { return dtype == CAV_F32 ? 4 : 8; }

int check_grid(const cav_grid* g)
{
    if (!g) return fail(CAV_EINVAL, "grid is NULL");
    if (g->ng != NG) return fail(CAV_EINVAL, "ng must be %d (got %d)", NG, g->ng);
    if (g->dtype != CAV_F64 && g->dtype != CAV_F32) return fail(CAV_EINVAL, "unknown dtype %d", g->dtype);
    if (g->ni < 2 || g->nj < 2 || g->nk < 2)
        return fail(CAV_EINVAL, "every grid extent must be >= 2 (got %d x %d x %d)", g->ni, g->nj, g->nk);
    const long long align = ROW_ALIGN_BYTES / elem_size(g->dtype);
    const long long row = (align + (long long)g->ni + NG + align - 1) / align * align;
    const long long per = row * (g->nj + 2 * NG) * (g->nk + 2 * NG);
    if (per >= (1LL << 31))
        return fail(CAV_EINVAL, "grid %d x %d x %d too large (one field must stay below 2^31 elements)",
                    g->ni, g->nj, g->nk);
    return CAV_OK;
}

Dims dims_of(const cav_grid* g)
{
    Dims d;
    d.ni = g->ni;
    d.nj = g->nj;
    d.nk = g->nk;
    const int align = ROW_ALIGN_BYTES / elem_size(g->dtype);
    d.lead = align;
    d.sy = (d.lead + g->ni + NG + align - 1) / align * align;
    d.sz = (g->nj + 2 * NG) * d.sy;
    return d;
}

size_t field_elems(const Dims& d) { return (size_t)(d.nk + 2 * NG) * (size_t)d.sz; }

template <typename Real>
StateT<Real> state_of(void* q, const Dims& d)
{
    StateT<Real> s;
    Real* base = static_cast<Real*>(q);
    for (int f = 0; f < NF; ++f) s.f[f] = base + (size_t)f * field_elems(d);
    return s;
}

template <typename Real>
CStateT<Real> cstate_of(const void* q, const Dims& d)
{
    CStateT<Real> s;
    const Real* base = static_cast<const Real*>(q);
    for (int f = 0; f < NF; ++f) s.f[f] = base + (size_t)f * field_elems(d);
    return s;
}

int check_params(const cav_params* p)
{
    if (!p) return fail(CAV_EINVAL, "params is NULL");
    const double v[9] = {p->Ra, p->Pr, p->cfl, p->eps4, p->kappa, p->u_ref, p->t_hot, p->t_cold, p->t_inf};
    for (double x : v)
        if (!std::isfinite(x)) return fail(CAV_EINVAL, "params must be finite");
    if (!(p->Ra > 0) || !(p->Pr > 0)) return fail(CAV_EINVAL, "Ra and Pr must be > 0");
    if (!(p->cfl > 0)) return fail(CAV_EINVAL, "cfl must be > 0");
    if (p->eps4 < 0 || p->kappa < 0 || p->u_ref < 0)
        return fail(CAV_EINVAL, "eps4, kappa and u_ref must be >= 0");
    return CAV_OK;
}

Coef coef_of(const cav_grid* g, const cav_params* p)
{
    Coef c;
    const double nx = g->ni, ny = g->nj, nz = g->nk;
    c.hx2 = 0.5 * nx; c.hy2 = 0.5 * ny; c.hz2 = 0.5 * nz;
    c.ix2 = nx * nx; c.iy2 = ny * ny; c.iz2 = nz * nz;
    c.nx = nx; c.ny = ny; c.nz = nz;
    c.eps4 = p->eps4;
    c.beta2_floor = p->kappa * p->u_ref * p->u_ref;
    c.nu = std::sqrt(p->Pr / p->Ra);
    c.alpha = 1.0 / std::sqrt(p->Ra * p->Pr);
    c.t_inf = p->t_inf;
    c.cfl = p->cfl;
    const double dmax = c.nu > c.alpha ? c.nu : c.alpha;
    c.dt_visc = 1.0 / (2.0 * dmax * (nx * nx + ny * ny + nz * nz));
    c.t_hot = p->t_hot;
    c.t_cold = p->t_cold;
    c.t_hot_field = static_cast<const double*>(p->t_hot_field);
    return c;
}

int check_halo(const cav_grid* g, const cav_halo* h, HaloGeom* out)
{
    if (!h) return fail(CAV_EINVAL, "halo is NULL");
    const int n[3] = {g->ni, g->nj, g->nk};
    HaloGeom hg;
    long long nsub = 1;
    for (int a = 0; a < 3; ++a) {
        if (h->split[a] < 1) return fail(CAV_EINVAL, "split[%d] = %d must be >= 1", a, h->split[a]);
        if (n[a] % h->split[a])
            return fail(CAV_EINVAL, "split[%d] = %d does not divide the grid extent %d", a, h->split[a], n[a]);
        hg.P[a] = h->split[a];
        hg.e[a] = n[a] / h->split[a];
        nsub *= h->split[a];
    }
    if (nsub * 6 > 65535) return fail(CAV_EINVAL, "too many subdomains (%lld)", nsub);
    int wmax = 0;
    hg.wsum = 0;
    for (int f = 0; f < NF; ++f) {
        const int w = h->width[f];
        if (w < 0 || w > g->ng) return fail(CAV_EINVAL, "width[%d] = %d outside [0, ng=%d]", f, w, g->ng);
        hg.w[f] = w;
        hg.wpre[f] = hg.wsum;
        hg.wsum += w;
        wmax = w > wmax ? w : wmax;
    }
    for (int a = 0; a < 3; ++a)
        if (hg.P[a] > 1 && hg.e[a] < wmax)
            return fail(CAV_EINVAL, "subdomain extent %d along axis %d is thinner than width %d", hg.e[a], a, wmax);
    hg.area[0] = (long long)hg.e[1] * hg.e[2];
    hg.area[1] = (long long)hg.e[0] * hg.e[2];
    hg.area[2] = (long long)hg.e[0] * hg.e[1];
    // the launch: for each axis, its cut faces (2 per cut and transverse
    // subdomain pair) times the blocks one face needs
    long long end = 0;
    for (int a = 0; a < 3; ++a) {
        hg.nface[a] = (int)(2LL * (hg.P[a] - 1) * (nsub / hg.P[a]));
        const long long per_block = (long long)HALO_THREADS * HALO_ROWS;
        hg.bpf[a] = hg.nface[a] > 0 ? (int)((hg.area[a] + per_block - 1) / per_block) : 0;
        end += (long long)hg.nface[a] * hg.bpf[a];
        if (end >= (1LL << 31)) return fail(CAV_EINVAL, "halo launch of %lld blocks is too large", end);
        hg.blk_end[a] = (int)end;
    }
    if (out) *out = hg;
    return CAV_OK;
}

size_t halo_elems(const HaloGeom& h)
{
    const long long nsub = (long long)h.P[0] * h.P[1] * h.P[2];
    long long faces_area = 0;
    for (int a = 0; a < 3; ++a) faces_area += h.area[a] * 2LL * (h.P[a] - 1) * (nsub / h.P[a]);
    return (size_t)(faces_area * h.wsum);
}

// Whether the sweep's epilogue packs the exchange: a split along i only
// (every face is an i face, the noncontiguous kind), every column in at most
// one face box (subdomain extent along i >= 2 x the largest width), buffer
// offsets within 32 bits.  Other splits keep the pack kernel: there the
// epilogue's extra stores cost the sweep more than the i faces' pack costs
// (2x2x2 at 256^3: sweep +33 us for pack -20 us, unpack +10 us).
bool xpack_fusable(const HaloGeom& hg)
{
    int wmax = 0;
    for (int f = 0; f < NF; ++f) wmax = std::max(wmax, hg.w[f]);
    return hg.P[0] > 1 && hg.P[1] == 1 && hg.P[2] == 1 && wmax > 0 && hg.e[0] >= 2 * wmax &&
           halo_elems(hg) < (size_t)INT32_MAX;
}

constexpr size_t WS_HEAD = 64;   // 5 final norms, padded

// Sweep blocks resident at once: one per compute unit (the sweep needs
// more than 128 VGPRs per lane, so one 8-wave block fills a CU).  Queried
// once; 256 (MI355X) when no device is visible.
int device_slots()
{
    static int slots = 0;
    if (slots == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        slots = cus;
    }
    return slots;
}

// Large enough for any k-chunk length and any tile shape the type's
// kernels use (one partial per tile and plane).
size_t ws_bytes_of(const Dims& d, bool f32)
{
    auto tiles = [&](int ti, int tj) { return (size_t)((d.ni + ti - 1) / ti) * ((d.nj + tj - 1) / tj); };
    size_t t = std::max(tiles(SW_TI, SW_TJ), tiles(batch_wide_ti(f32), batch_tj(f32, batch_wide_ti(f32))));
    t = std::max(t, tiles(batch_narrow_ti(f32), batch_tj(f32, batch_narrow_ti(f32))));
    t = std::max(t, f32 ? tiles(F32_TI, F32_TJ) : tiles(F64_TI, F64_TJ));
    return WS_HEAD + t * d.nk * NF * sizeof(double);
}
size_t ws_bytes_of(const cav_grid* g) { return ws_bytes_of(dims_of(g), g->dtype == CAV_F32); }

// Work items of a batch member for k-chunk length kc (0 = whole columns)
// and tile width ti (batch_wide_ti or batch_narrow_ti of the type).
SweepGeom member_geom(const Dims& d, int kc, int ti, bool f32)
{
    SweepGeom g;
    const int tj = batch_tj(f32, ti);
    g.tiles_i = (d.ni + ti - 1) / ti;
    g.tiles_j = (d.nj + tj - 1) / tj;
    g.kc = (kc > 0 && kc < d.nk) ? kc : d.nk;
    g.nkc = (d.nk + g.kc - 1) / g.kc;
    g.nblocks = g.tiles_i * g.tiles_j * g.nkc;
    return g;
}

bool ti_valid(const cav_batch_member& m)
{
    const bool f32 = m.grid.dtype == CAV_F32;
    return m.ti == 0 || m.ti == batch_wide_ti(f32) || m.ti == batch_narrow_ti(f32);
}

int check_member(const cav_batch_member& m, int idx, int dtype)
{
    int rc;
    if ((rc = check_grid(&m.grid)) || (rc = check_params(&m.params)))
        return fail(rc, "batch member %d: %s", idx, std::string(g_err).c_str());
    if (m.grid.dtype != dtype) return fail(CAV_EINVAL, "batch member %d: dtype differs from member 0", idx);
    if (!m.q || !m.q_tmp || !m.ws) return fail(CAV_EINVAL, "batch member %d: q, q_tmp and ws must not be NULL", idx);
    if (m.q == m.q_tmp) return fail(CAV_EINVAL, "batch member %d: q and q_tmp must be distinct", idx);
    if (m.kc < 0) return fail(CAV_EINVAL, "batch member %d: kc = %d must be >= 0", idx, m.kc);
    const bool f32 = dtype == CAV_F32;
    if (!ti_valid(m))
        return fail(CAV_EINVAL, "batch member %d: ti = %d must be 0, %d or %d", idx, m.ti, batch_wide_ti(f32),
                    batch_narrow_ti(f32));
    const size_t need = ws_bytes_of(&m.grid);
    if (m.ws_bytes < need) return fail(CAV_ESIZE, "batch member %d: ws_bytes %zu < required %zu", idx, m.ws_bytes, need);
    return CAV_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int member_ti(const cav_batch_member& m)
{
    const bool f32 = m.grid.dtype == CAV_F32;
    return m.ti == batch_narrow_ti(f32) ? batch_narrow_ti(f32) : batch_wide_ti(f32);
}

template <typename Real>
hipError_t batch_launches(const cav_batch& b, int32_t nsteps, int nblocks, int parity, hipStream_t stream, bool timed)
{
    const BatchCav* cavs = static_cast<const BatchCav*>(b.table);
    const char* region = static_cast<const char*>(b.table) + align256(sizeof(BatchCav) * b.members);
    const int* segs = reinterpret_cast<const int*>(region);
    const BatchItem* items = reinterpret_cast<const BatchItem*>(region + BATCH_HEAD_BYTES);
    hipError_t e = hipSuccess;
    for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
        const bool last = n == nsteps - 1;
        auto go = [&] { return launch_batch<Real>(cavs, segs, items, parity, last, nblocks, b.shapes, stream); };
        e = timed ? run(last ? "batch_norm" : "batch", stream, go) : go();
        parity ^= 1;
    }
    if (e == hipSuccess && nsteps > 0) {
        auto fin = [&] { return launch_batch_norms(cavs, b.members, stream); };
        e = timed ? run("batch_norm_finalize", stream, fin) : fin();
    }
    return e;
}

int check_batch(const cav_batch* b)
{
    if (!b || !b->table) return fail(CAV_EINVAL, "batch (or its table) is NULL");
    if (b->members < 1 || b->items < 1) return fail(CAV_EINVAL, "empty batch");
    if (b->dtype != CAV_F64 && b->dtype != CAV_F32) return fail(CAV_EINVAL, "unknown batch dtype %d", b->dtype);
    if (b->parity != 0 && b->parity != 1) return fail(CAV_EINVAL, "batch parity must be 0 or 1");
    return CAV_OK;
}

// Host object behind a batch graph handle: the executable graph and what it
// was captured from (its launches read the current states from q or q_tmp
// as the batch's parity was at capture, so a replay is valid only while the
// parity and the table are unchanged).
struct BatchGraph {
    hipGraphExec_t exec;
    const void* table;
    int32_t items;
    int32_t parity;
};

int do_halo(const cav_grid* grid, const HaloGeom& hg, void* q, void* buf, bool pack, hipStream_t s,
            bool timed = true, int first_axis = 0)
{
    if (hg.blk_end[2] == 0 || hg.wsum == 0) return CAV_OK;       // nothing to exchange
    const Dims d = dims_of(grid);
    auto launch = [&] {
        return grid->dtype == CAV_F32
                   ? launch_halo<float>(d, hg, state_of<float>(q, d), static_cast<float*>(buf), pack, s, first_axis)
                   : launch_halo<double>(d, hg, state_of<double>(q, d), static_cast<double*>(buf), pack, s,
                                         first_axis);
    };
    hipError_t e = timed ? run(pack ? "halo_pack" : "halo_unpack", s, launch) : launch();
    return e == hipSuccess ? CAV_OK : hip_fail(pack ? "halo_pack launch" : "halo_unpack launch", e);
}

// The pseudo-time steps of cavity_step in element type Real.  The last
// sweep writes 5 norm partials per block into `partials` and the finalize
// reduces them into norms[0..4]; with norms == NULL the norm pass is
// skipped.  `timed` allows the event timing (which creates events); the
// allocation-free entry point passes false.
template <typename Real>
int step_impl(const cav_grid* grid, const cav_params* prm, const cav_halo* halo, const HaloGeom& hg, void* q,
              void* q_tmp, double* partials, double* norms, void* halo_buf, int32_t nsteps, hipStream_t stream,
              bool timed = true)
{
    int rc;
    const Dims d = dims_of(grid);
    const Coef c = coef_of(grid, prm);
    const SweepGeom g = step_geom<Real>(d, device_slots());
    auto go = [&](const char* name, auto&& launch) { return timed ? run(name, stream, launch) : launch(); };
    // the sweep of step n packs the i faces of step n+1's exchange when the
    // split allows (xfuse); that step's pack then moves the j and k faces
    const bool xfuse = halo && xpack_fusable(hg);
    void* cur = q;
    void* nxt = q_tmp;
    hipError_t e;
    for (int n = 0; n < nsteps; ++n) {
        // the wall ghosts are derived inside the sweep; no separate pass
        if (halo) {
            const int first_axis = xfuse && n > 0 ? 1 : 0;
            if ((rc = do_halo(grid, hg, cur, halo_buf, true, stream, timed, first_axis))) return rc;
            if ((rc = do_halo(grid, hg, cur, halo_buf, false, stream, timed))) return rc;
        }
        const bool last = n == nsteps - 1 && norms;
        const bool xp = xfuse && n < nsteps - 1;
        e = go(last ? "sweep_norm" : (xp ? "sweep_xpack" : "sweep"), [&] {
            return launch_sweep<Real>(d, c, g, cstate_of<Real>(cur, d), state_of<Real>(nxt, d), partials, last,
                                      stream, xp ? &hg : nullptr, xp ? static_cast<Real*>(halo_buf) : nullptr);
        });
        if (e != hipSuccess) return hip_fail("sweep launch", e);
        void* t = cur;
        cur = nxt;
        nxt = t;
    }
    if (norms) {
        const double ncell = (double)d.ni * d.nj * d.nk;
        e = go("norm_finalize", [&] { return launch_norm_finalize(partials, g.nblocks, ncell, norms, stream); });
        if (e != hipSuccess) return hip_fail("norm finalize launch", e);
    }
    if (cur != q) {
        const size_t bytes = (size_t)NF * field_elems(d) * sizeof(Real);
        e = go("copy", [&] { return hipMemcpyAsync(q, cur, bytes, hipMemcpyDeviceToDevice, stream); });
        if (e != hipSuccess) return hip_fail("state copy", e);
    }
    return CAV_OK;
}

// Argument checks shared by cavity_step and cavity_step_noalloc (everything
// but the workspace).
int check_step(const cav_grid* grid, const cav_params* prm, const cav_halo* halo, const void* q, const void* q_tmp,
               const void* halo_buf, size_t halo_bytes, int32_t nsteps, HaloGeom* hg)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_params(prm))) return rc;
    if (nsteps < 0) return fail(CAV_EINVAL, "nsteps = %d must be >= 0", nsteps);
    if (!q || !q_tmp) return fail(CAV_EINVAL, "q and q_tmp must not be NULL");
    if (q == q_tmp) return fail(CAV_EINVAL, "q and q_tmp must be distinct buffers");
    if (halo) {
        if ((rc = check_halo(grid, halo, hg))) return rc;
        const size_t need = halo_elems(*hg) * (size_t)elem_size(grid->dtype);
        if (need && !halo_buf) return fail(CAV_EINVAL, "halo_buf is NULL");
        if (halo_bytes < need) return fail(CAV_ESIZE, "halo_bytes %zu < required %zu", halo_bytes, need);
    }
    return CAV_OK;
}

// ---- the scratch of cavity_step_noalloc -------------------------------------
// Its sweeps' per-block norm partials live in the file-scope array `scratch`
// (declared above this namespace).  Host code never uses the array's name as
// an address: on the host it is a stand-in, not device memory.  Each
// device's address is looked up once with hipGetSymbolAddress, with that
// device current, and kept in g_scratch_dev.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
int scratch_of_current_device(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail("hipGetDevice", e);
    if (dev < 0 || dev >= MAX_DEVICES) return fail(CAV_EINVAL, "device %d beyond the %d supported", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail("hipGetSymbolAddress(scratch)", e);
        if (!p) return fail(CAV_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return CAV_OK;
}

// Interior/exterior split: margin m = the widest reach of an unpacked
// layer into the stars (width + 2 for p, width + 1 for u v w T); exterior x
// and y slabs in k chunks of 16 planes, longer if the norm partials would
// not fit the workspace.
int split_geom(const cav_grid* grid, const HaloGeom& hg, const SweepGeom& gi, const SweepGeom& g, size_t ws_bytes,
               SplitGeom* out)
{
    const Dims d = dims_of(grid);
    SplitGeom sg;
    sg.m = 0;
    for (int f = 0; f < NF; ++f)
        if (hg.w[f] > 0) sg.m = std::max(sg.m, hg.w[f] + (f == FP ? 2 : 1));
    const int n[3] = {grid->ni, grid->nj, grid->nk};
    for (int a = 0; a < 3; ++a) {
        sg.P[a] = sg.m > 0 ? hg.P[a] : 1;
        sg.e[a] = n[a] / hg.P[a];
        if (sg.P[a] > 1 && sg.e[a] < 2 * sg.m)
            return fail(CAV_EINVAL, "subdomain extent %d along axis %d is below 2 x the exterior margin %d", sg.e[a], a,
                        sg.m);
    }
    const size_t cap = (ws_bytes - WS_HEAD) / (NF * sizeof(double));
    for (sg.kce = std::min(16, d.nk);; sg.kce = std::min(2 * sg.kce, d.nk)) {
        if ((size_t)gi.nblocks + exterior_blocks(d, g, sg) <= cap) break;
        if (sg.kce == d.nk)
            return fail(CAV_ESIZE, "workspace too small for the norm partials of the split sweep");
    }
    *out = sg;
    return CAV_OK;
}

template <typename Real>
int overlap_impl(const cav_grid* grid, const cav_params* prm, const HaloGeom& hg, void* q, void* q_tmp, void* ws,
                 size_t ws_bytes, void* halo_buf, int32_t nsteps, hipStream_t stream, hipStream_t comm)
{
    int rc;
    const Dims d = dims_of(grid);
    const Coef c = coef_of(grid, prm);
    const SweepGeom gi = step_geom<Real>(d, device_slots());   // interior: the step sweep's tile
    const SweepGeom g = sweep_geom(d, device_slots());          // exterior slabs: the 64 x 8 tiling
    SplitGeom sg;
    if ((rc = split_geom(grid, hg, gi, g, ws_bytes, &sg))) return rc;
    const int nb_ext = exterior_blocks(d, g, sg);
    double* wsd = static_cast<double*>(ws);
    double* partials = reinterpret_cast<double*>(static_cast<char*>(ws) + WS_HEAD);
    hipEvent_t ready = nullptr, exchanged = nullptr;
    hipError_t e;
    if ((e = hipEventCreateWithFlags(&ready, hipEventDisableTiming)) != hipSuccess) return hip_fail("event create", e);
    if ((e = hipEventCreateWithFlags(&exchanged, hipEventDisableTiming)) != hipSuccess) {
        (void)hipEventDestroy(ready);
        return hip_fail("event create", e);
    }
    auto done = [&](int r) {                             // destroyed once their work completes
        (void)hipEventDestroy(ready);
        (void)hipEventDestroy(exchanged);
        return r;
    };
    void* cur = q;
    void* nxt = q_tmp;
    for (int n = 0; n < nsteps; ++n) {
        const bool last = n == nsteps - 1;
        // the exchange on `comm` once the state is complete
        if ((e = hipEventRecord(ready, stream)) != hipSuccess) return done(hip_fail("event record", e));
        if ((e = hipStreamWaitEvent(comm, ready, 0)) != hipSuccess) return done(hip_fail("stream wait", e));
        if ((rc = do_halo(grid, hg, cur, halo_buf, true, comm))) return done(rc);
        if ((rc = do_halo(grid, hg, cur, halo_buf, false, comm))) return done(rc);
        if ((e = hipEventRecord(exchanged, comm)) != hipSuccess) return done(hip_fail("event record", e));
        // interior meanwhile on `stream`, exterior after the exchange
        e = run(last ? "interior_norm" : "interior", stream, [&] {
            return launch_split<Real>(d, c, gi, g, sg, false, cstate_of<Real>(cur, d), state_of<Real>(nxt, d),
                                      partials, last, stream);
        });
        if (e != hipSuccess) return done(hip_fail("interior launch", e));
        if ((e = hipStreamWaitEvent(stream, exchanged, 0)) != hipSuccess) return done(hip_fail("stream wait", e));
        e = run(last ? "exterior_norm" : "exterior", stream, [&] {
            return launch_split<Real>(d, c, gi, g, sg, true, cstate_of<Real>(cur, d), state_of<Real>(nxt, d),
                                      partials, last, stream);
        });
        if (e != hipSuccess) return done(hip_fail("exterior launch", e));
        std::swap(cur, nxt);
    }
    const double ncell = (double)d.ni * d.nj * d.nk;
    e = run("norm_finalize", stream,
            [&] { return launch_norm_finalize(partials, gi.nblocks + nb_ext, ncell, wsd, stream); });
    if (e != hipSuccess) return done(hip_fail("norm finalize launch", e));
    if (cur != q) {
        const size_t bytes = (size_t)NF * field_elems(d) * sizeof(Real);
        e = run("copy", stream, [&] { return hipMemcpyAsync(q, cur, bytes, hipMemcpyDeviceToDevice, stream); });
        if (e != hipSuccess) return done(hip_fail("state copy", e));
    }
    return done(CAV_OK);
}

}  // namespace

extern "C" {

size_t cavity_state_elems(const cav_grid* grid)
{
    if (check_grid(grid) != CAV_OK) return 0;
    return (size_t)NF * field_elems(dims_of(grid));
}

int cavity_layout(const cav_grid* grid, cav_layout* out)
{
    int rc;
    if ((rc = check_grid(grid))) return rc;
    if (!out) return fail(CAV_EINVAL, "out is NULL");
    const Dims d = dims_of(grid);
    out->lead = d.lead;
    out->sj = d.sy;
    out->sk = d.sz;
    out->sf = (int64_t)field_elems(d);
    out->origin = (int64_t)NG * d.sz + (int64_t)NG * d.sy + d.lead;
    return CAV_OK;
}

size_t cavity_workspace_bytes(const cav_grid* grid)
{
    if (check_grid(grid) != CAV_OK) return 0;
    return ws_bytes_of(grid);
}

size_t halo_buffer_bytes(const cav_grid* grid, const cav_halo* halo)
{
    HaloGeom hg;
    if (check_grid(grid) != CAV_OK || check_halo(grid, halo, &hg) != CAV_OK) return 0;
    return halo_elems(hg) * (size_t)elem_size(grid->dtype);
}

int cavity_init(const cav_grid* grid, const cav_params* prm, uint64_t seed, double noise_amp, void* q,
                hipStream_t stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_params(prm))) return rc;
    if (!q) return fail(CAV_EINVAL, "q is NULL");
    if (!std::isfinite(noise_amp)) return fail(CAV_EINVAL, "noise_amp must be finite");
    const Dims d = dims_of(grid);
    const Bcs bc{prm->t_hot, prm->t_cold, static_cast<const double*>(prm->t_hot_field)};
    const bool f32 = grid->dtype == CAV_F32;
    hipError_t e = run("init", stream, [&] {
        return f32 ? launch_init<float>(d, prm->t_hot, prm->t_cold, seed, noise_amp, state_of<float>(q, d), stream)
                   : launch_init<double>(d, prm->t_hot, prm->t_cold, seed, noise_amp, state_of<double>(q, d), stream);
    });
    if (e != hipSuccess) return hip_fail("init launch", e);
    e = run("bc", stream, [&] {
        return f32 ? launch_bc<float>(d, bc, state_of<float>(q, d), stream)
                   : launch_bc<double>(d, bc, state_of<double>(q, d), stream);
    });
    if (e != hipSuccess) return hip_fail("bc launch", e);
    return CAV_OK;
}

int cavity_step(const cav_grid* grid, const cav_params* prm, const cav_halo* halo, void* q, void* q_tmp,
                void* ws, size_t ws_bytes, void* halo_buf, size_t halo_bytes, int32_t nsteps,
                hipStream_t stream)
{
    int rc;
    HaloGeom hg;
    if ((rc = check_step(grid, prm, halo, q, q_tmp, halo_buf, halo_bytes, nsteps, &hg))) return rc;
    if (!ws) return fail(CAV_EINVAL, "ws must not be NULL");
    const size_t need_ws = ws_bytes_of(grid);
    if (ws_bytes < need_ws) return fail(CAV_ESIZE, "ws_bytes %zu < required %zu", ws_bytes, need_ws);
    if (nsteps == 0) return CAV_OK;
    double* norms = static_cast<double*>(ws);
    double* partials = reinterpret_cast<double*>(static_cast<char*>(ws) + WS_HEAD);
    return grid->dtype == CAV_F32
               ? step_impl<float>(grid, prm, halo, hg, q, q_tmp, partials, norms, halo_buf, nsteps, stream)
               : step_impl<double>(grid, prm, halo, hg, q, q_tmp, partials, norms, halo_buf, nsteps, stream);
}

int cavity_step_from(const cav_grid* grid, const cav_params* prm, const void* q_in, void* q_out, void* ws,
                     size_t ws_bytes, hipStream_t stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_params(prm))) return rc;
    if (!q_in || !q_out) return fail(CAV_EINVAL, "q_in and q_out must not be NULL");
    if (q_in == q_out) return fail(CAV_EINVAL, "q_in and q_out must be distinct buffers");
    if (ws && ws_bytes < ws_bytes_of(grid))
        return fail(CAV_ESIZE, "ws_bytes %zu < required %zu", ws_bytes, ws_bytes_of(grid));
    const Dims d = dims_of(grid);
    const Coef c = coef_of(grid, prm);
    double* norms = static_cast<double*>(ws);
    double* partials = ws ? reinterpret_cast<double*>(static_cast<char*>(ws) + WS_HEAD) : nullptr;
    auto one = [&](auto tag) {
        using Real = decltype(tag);
        const SweepGeom g = step_geom<Real>(d, device_slots());
        hipError_t e = run(ws ? "sweep_norm" : "sweep", stream, [&] {
            return launch_sweep<Real>(d, c, g, cstate_of<Real>(q_in, d), state_of<Real>(q_out, d), partials,
                                      ws != nullptr, stream);
        });
        if (e != hipSuccess) return hip_fail("sweep launch", e);
        if (ws) {
            const double ncell = (double)d.ni * d.nj * d.nk;
            e = run("norm_finalize", stream,
                    [&] { return launch_norm_finalize(partials, g.nblocks, ncell, norms, stream); });
            if (e != hipSuccess) return hip_fail("norm finalize launch", e);
        }
        return (int)CAV_OK;
    };
    return grid->dtype == CAV_F32 ? one(float{}) : one(double{});
}

int cavity_step_noalloc(const cav_grid* grid, const cav_params* prm, const cav_halo* halo, void* q, void* q_tmp,
                        void* halo_buf, size_t halo_bytes, double* norms, int32_t nsteps, hipStream_t stream)
{
    int rc;
    HaloGeom hg;
    if ((rc = check_step(grid, prm, halo, q, q_tmp, halo_buf, halo_bytes, nsteps, &hg))) return rc;
    const SweepGeom g = grid->dtype == CAV_F32 ? step_geom<float>(dims_of(grid), device_slots())
                                               : step_geom<double>(dims_of(grid), device_slots());
    if (norms && g.nblocks > NOALLOC_MAX_BLOCKS)
        return fail(CAV_ESIZE,
                    "grid %d x %d x %d: its sweep runs %d blocks, whose norm partials exceed the static scratch "
                    "of %d blocks (pass norms = NULL, or use cavity_step with a workspace)",
                    grid->ni, grid->nj, grid->nk, g.nblocks, NOALLOC_MAX_BLOCKS);
    double* partials = nullptr;
    if ((rc = scratch_of_current_device(&partials))) return rc;
    if (nsteps == 0) return CAV_OK;
    return grid->dtype == CAV_F32
               ? step_impl<float>(grid, prm, halo, hg, q, q_tmp, partials, norms, halo_buf, nsteps, stream, false)
               : step_impl<double>(grid, prm, halo, hg, q, q_tmp, partials, norms, halo_buf, nsteps, stream, false);
}

int cavity_step_overlap(const cav_grid* grid, const cav_params* prm, const cav_halo* halo, void* q, void* q_tmp,
                        void* ws, size_t ws_bytes, void* halo_buf, size_t halo_bytes, int32_t nsteps,
                        hipStream_t stream, hipStream_t comm_stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_params(prm))) return rc;
    if (nsteps < 0) return fail(CAV_EINVAL, "nsteps = %d must be >= 0", nsteps);
    if (!halo) return fail(CAV_EINVAL, "halo is NULL (the split needs the exchange it overlaps)");
    if (!q || !q_tmp || !ws) return fail(CAV_EINVAL, "q, q_tmp and ws must not be NULL");
    if (q == q_tmp) return fail(CAV_EINVAL, "q and q_tmp must be distinct buffers");
    const size_t need_ws = ws_bytes_of(grid);
    if (ws_bytes < need_ws) return fail(CAV_ESIZE, "ws_bytes %zu < required %zu", ws_bytes, need_ws);
    HaloGeom hg;
    if ((rc = check_halo(grid, halo, &hg))) return rc;
    const size_t need = halo_elems(hg) * (size_t)elem_size(grid->dtype);
    if (need && !halo_buf) return fail(CAV_EINVAL, "halo_buf is NULL");
    if (halo_bytes < need) return fail(CAV_ESIZE, "halo_bytes %zu < required %zu", halo_bytes, need);
    if (nsteps == 0) return CAV_OK;
    return grid->dtype == CAV_F32
               ? overlap_impl<float>(grid, prm, hg, q, q_tmp, ws, ws_bytes, halo_buf, nsteps, stream, comm_stream)
               : overlap_impl<double>(grid, prm, hg, q, q_tmp, ws, ws_bytes, halo_buf, nsteps, stream, comm_stream);
}

int halo_pack(const cav_grid* grid, const cav_halo* halo, const void* q, void* buf, size_t buf_bytes,
              hipStream_t stream)
{
    int rc;
    HaloGeom hg;
    if ((rc = check_grid(grid)) || (rc = check_halo(grid, halo, &hg))) return rc;
    const size_t need = halo_elems(hg) * (size_t)elem_size(grid->dtype);
    if (!q || (need && !buf)) return fail(CAV_EINVAL, "q and buf must not be NULL");
    if (buf_bytes < need) return fail(CAV_ESIZE, "buf_bytes %zu < required %zu", buf_bytes, need);
    return do_halo(grid, hg, const_cast<void*>(q), buf, true, stream);
}

int halo_unpack(const cav_grid* grid, const cav_halo* halo, const void* buf, size_t buf_bytes, void* q,
                hipStream_t stream)
{
    int rc;
    HaloGeom hg;
    if ((rc = check_grid(grid)) || (rc = check_halo(grid, halo, &hg))) return rc;
    const size_t need = halo_elems(hg) * (size_t)elem_size(grid->dtype);
    if (!q || (need && !buf)) return fail(CAV_EINVAL, "q and buf must not be NULL");
    if (buf_bytes < need) return fail(CAV_ESIZE, "buf_bytes %zu < required %zu", buf_bytes, need);
    return do_halo(grid, hg, q, const_cast<void*>(buf), false, stream);
}

int cavity_residual_norm(const cav_grid* grid, const void* ws, size_t ws_bytes, double* out5, hipStream_t stream)
{
    int rc;
    if ((rc = check_grid(grid))) return rc;
    if (!ws || !out5) return fail(CAV_EINVAL, "ws and out5 must not be NULL");
    const size_t need = ws_bytes_of(grid);
    if (ws_bytes < need) return fail(CAV_ESIZE, "ws_bytes %zu < required %zu", ws_bytes, need);
    hipError_t e = hipMemcpyAsync(out5, ws, NF * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return hip_fail("norm copy", e);
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail("stream synchronize", e);
    for (int f = 0; f < NF; ++f)
        if (!std::isfinite(out5[f])) return fail(CAV_ENONFINITE, "residual norm of field %d is not finite", f);
    return CAV_OK;
}

int cavity_nusselt(const cav_grid* grid, const cav_params* prm, const void* q, void* ws, size_t ws_bytes,
                   double* out, hipStream_t stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_params(prm))) return rc;
    if (!q || !ws || !out) return fail(CAV_EINVAL, "q, ws and out must not be NULL");
    if (prm->t_hot == prm->t_cold) return fail(CAV_EINVAL, "t_hot == t_cold: the Nusselt number is undefined");
    const Dims d = dims_of(grid);
    const size_t need = ws_bytes_of(grid);
    if (ws_bytes < need) return fail(CAV_ESIZE, "ws_bytes %zu < required %zu", ws_bytes, need);
    double* slot = static_cast<double*>(ws) + 6;
    const Bcs bc{prm->t_hot, prm->t_cold, static_cast<const double*>(prm->t_hot_field)};
    hipError_t e = run("nusselt", stream, [&] {
        return grid->dtype == CAV_F32 ? launch_nusselt<float>(d, bc, cstate_of<float>(q, d), slot, stream)
                                      : launch_nusselt<double>(d, bc, cstate_of<double>(q, d), slot, stream);
    });
    if (e != hipSuccess) return hip_fail("nusselt launch", e);
    e = hipMemcpyAsync(out, slot, sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return hip_fail("nusselt copy", e);
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail("stream synchronize", e);
    return CAV_OK;
}

size_t cavity_adjoint_workspace_bytes(const cav_grid* grid)
{
    if (check_grid(grid) != CAV_OK || grid->dtype != CAV_F64) return 0;
    return adjoint_ws_doubles(dims_of(grid)) * sizeof(double);
}

int cavity_nusselt_adjoint(const cav_grid* grid, const cav_params* prm, void* lam, double* dj_dthot,
                           hipStream_t stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_params(prm))) return rc;
    if (grid->dtype != CAV_F64) return fail(CAV_EINVAL, "the adjoint is available for CAV_F64 only");
    if (!lam) return fail(CAV_EINVAL, "lam is NULL");
    if (prm->t_hot == prm->t_cold) return fail(CAV_EINVAL, "t_hot == t_cold: the Nusselt number is undefined");
    const Dims d = dims_of(grid);
    const double scale = ((double)grid->ni / 3.0) / ((double)grid->nj * (double)grid->nk) / (prm->t_hot - prm->t_cold);
    hipError_t e = run("nusselt_seed", stream, [&] {
        return launch_nusselt_seed(d, scale, state_of<double>(lam, d), dj_dthot, stream);
    });
    if (e != hipSuccess) return hip_fail("nusselt seed launch", e);
    return CAV_OK;
}

int cavity_adjoint_step(const cav_grid* grid, const cav_params* prm, const void* q_n, const void* lam_in,
                        void* lam_out, void* ws, size_t ws_bytes, double* dj_dthot, double* dj_dra,
                        hipStream_t stream)
{
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_params(prm))) return rc;
    if (grid->dtype != CAV_F64) return fail(CAV_EINVAL, "the adjoint is available for CAV_F64 only");
    if (!q_n || !lam_in || !lam_out || !ws) return fail(CAV_EINVAL, "q_n, lam_in, lam_out and ws must not be NULL");
    if (lam_out == q_n || lam_in == q_n) return fail(CAV_EINVAL, "the cotangents must not alias q_n");
    if (lam_out == lam_in)
        return fail(CAV_EINVAL, "lam_out must not alias lam_in (the gather reads lam_in at every cell's neighbours)");
    const Dims d = dims_of(grid);
    const size_t need = adjoint_ws_doubles(d) * sizeof(double);
    if (ws_bytes < need) return fail(CAV_ESIZE, "ws_bytes %zu < required %zu", ws_bytes, need);
    const Coef c = coef_of(grid, prm);
    const SweepGeom g = sweep_geom(d, device_slots());
    const SweepGeom gg = gather_geom(d, device_slots());
    hipError_t e = run("adjoint_step", stream, [&] {
        return launch_adjoint_step(d, c, g, gg, prm->Ra, cstate_of<double>(q_n, d), cstate_of<double>(lam_in, d),
                                   state_of<double>(lam_out, d), static_cast<double*>(ws), dj_dthot, dj_dra,
                                   stream);
    });
    if (e != hipSuccess) return hip_fail("adjoint launch", e);
    return CAV_OK;
}

size_t cavity_batch_table_bytes(int32_t n, const cav_batch_member* members)
{
    if (n < 1 || !members) return 0;
    size_t items = 0;
    for (int m = 0; m < n; ++m) {
        if (check_grid(&members[m].grid) != CAV_OK || members[m].kc < 0) return 0;
        if (!ti_valid(members[m])) return 0;
        items += (size_t)member_geom(dims_of(&members[m].grid), members[m].kc, member_ti(members[m]),
                                     members[m].grid.dtype == CAV_F32).nblocks;
    }
    return align256(sizeof(BatchCav) * n) + BATCH_HEAD_BYTES + sizeof(BatchItem) * items;
}

int cavity_batch_build(int32_t n, const cav_batch_member* members, void* table, size_t table_bytes, cav_batch* out,
                       hipStream_t stream)
{
    int rc;
    if (n < 1 || !members || !table || !out) return fail(CAV_EINVAL, "n >= 1, members, table and out are required");
    const int dtype = members[0].grid.dtype;
    for (int m = 0; m < n; ++m)
        if ((rc = check_member(members[m], m, dtype))) return rc;
    const size_t need = cavity_batch_table_bytes(n, members);
    if (table_bytes < need) return fail(CAV_ESIZE, "table_bytes %zu < required %zu", table_bytes, need);

    std::vector<BatchCav> cavs(n);
    struct Work { BatchItem it; long long cost; };
    std::vector<Work> work;
    uint64_t cells = 0;
    for (int m = 0; m < n; ++m) {
        const cav_batch_member& mb = members[m];
        const Dims d = dims_of(&mb.grid);
        const bool f32 = dtype == CAV_F32;
        const int ti = member_ti(mb), tj = batch_tj(f32, ti);
        const SweepGeom g = member_geom(d, mb.kc, ti, f32);
        BatchCav& cv = cavs[m];
        cv.d = d;
        cv.ti = ti;
        cv.tiles_i = g.tiles_i;
        cv.tiles_j = g.tiles_j;
        cv.kc = g.kc;
        cv.ntiles = g.nblocks;
        cv.c = coef_of(&mb.grid, &mb.params);
        cv.q = mb.q;
        cv.q_tmp = mb.q_tmp;
        cv.ws = static_cast<double*>(mb.ws);
        cv.fstride = (long long)field_elems(d);
        cells += (uint64_t)d.ni * d.nj * d.nk;
        for (int t = 0; t < g.nblocks; ++t) {
            const int bi = t % g.tiles_i, bj = (t / g.tiles_i) % g.tiles_j, bk = t / (g.tiles_i * g.tiles_j);
            const long long ci = std::min(ti, d.ni - bi * ti), cj = std::min(tj, d.nj - bj * tj);
            const long long ck = std::min(g.kc, d.nk - bk * g.kc);
            work.push_back({{m, t}, ci * cj * ck});
        }
    }
    // Members with the longest items first (so the persistent blocks finish
    // together), each member's tiles in tiling order; then the list is cut
    // into BATCH_SEGS contiguous segments of about equal cost, one per XCD.
    std::vector<long long> mcost(n, 0);
    for (const Work& w : work) mcost[w.it.cav] = std::max(mcost[w.it.cav], w.cost);
    std::stable_sort(work.begin(), work.end(), [&](const Work& a, const Work& b) {
        return mcost[a.it.cav] > mcost[b.it.cav] || (mcost[a.it.cav] == mcost[b.it.cav] && a.it.cav < b.it.cav);
    });
    long long total = 0;
    for (const Work& w : work) total += w.cost;
    std::vector<char> host(need, 0);
    std::memcpy(host.data(), cavs.data(), sizeof(BatchCav) * n);
    char* region = host.data() + align256(sizeof(BatchCav) * n);
    int* segs = reinterpret_cast<int*>(region);
    BatchItem* items = reinterpret_cast<BatchItem*>(region + BATCH_HEAD_BYTES);
    static_assert((BATCH_SEGS + 1) * sizeof(int) <= BATCH_HEAD_BYTES, "segment bounds fit the head");
    long long run = 0;
    int seg = 1;
    segs[0] = 0;
    for (size_t w = 0; w < work.size(); ++w) {
        items[w] = work[w].it;
        run += work[w].cost;
        // close segment `seg` once its share of the cost is reached
        while (seg < BATCH_SEGS && run * BATCH_SEGS >= total * seg) segs[seg++] = (int)(w + 1);
    }
    while (seg <= BATCH_SEGS) segs[seg++] = (int)work.size();
    hipError_t e = hipMemcpyAsync(table, host.data(), need, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail("batch table upload", e);
    out->table = table;
    out->members = n;
    out->items = (int32_t)work.size();
    out->dtype = dtype;
    out->parity = 0;
    out->cells = cells;
    out->shapes = 0;
    for (int m = 0; m < n; ++m) out->shapes |= member_ti(members[m]) == batch_wide_ti(dtype == CAV_F32) ? 1 : 2;
    out->reserved = 0;
    return CAV_OK;
}

int cavity_batch_step(cav_batch* batch, int32_t nsteps, int32_t nblocks, hipStream_t stream)
{
    int rc;
    if ((rc = check_batch(batch))) return rc;
    if (nsteps < 0) return fail(CAV_EINVAL, "nsteps = %d must be >= 0", nsteps);
    if (nblocks < 0) return fail(CAV_EINVAL, "nblocks = %d must be >= 0", nblocks);
    if (nsteps == 0) return CAV_OK;
    const int nb = nblocks ? nblocks : device_slots();
    const hipError_t e = batch->dtype == CAV_F32 ? batch_launches<float>(*batch, nsteps, nb, batch->parity, stream, true)
                                                 : batch_launches<double>(*batch, nsteps, nb, batch->parity, stream, true);
    if (e != hipSuccess) return hip_fail("batch launch", e);
    batch->parity ^= (nsteps & 1);
    return CAV_OK;
}

int cavity_batch_graph_create(const cav_batch* batch, int32_t nsteps, int32_t nblocks, hipStream_t stream,
                              void** graph_exec)
{
    int rc;
    if ((rc = check_batch(batch))) return rc;
    if (nsteps < 2 || (nsteps & 1)) return fail(CAV_EINVAL, "nsteps = %d must be even and >= 2", nsteps);
    if (nblocks < 0) return fail(CAV_EINVAL, "nblocks = %d must be >= 0", nblocks);
    if (!graph_exec) return fail(CAV_EINVAL, "graph_exec is NULL");
    if (!stream) return fail(CAV_EINVAL, "graph capture needs a created stream, not the null stream");
    const int nb = nblocks ? nblocks : device_slots();
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail("begin capture", e);
    hipError_t el = batch->dtype == CAV_F32 ? batch_launches<float>(*batch, nsteps, nb, batch->parity, stream, false)
                                            : batch_launches<double>(*batch, nsteps, nb, batch->parity, stream, false);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(stream, &graph);
    if (el != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail("batch capture", el != hipSuccess ? el : e);
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail("graph instantiate", e);
    *graph_exec = new BatchGraph{exec, batch->table, batch->items, batch->parity};
    return CAV_OK;
}

int cavity_batch_graph_launch(const cav_batch* batch, void* graph_exec, hipStream_t stream)
{
    int rc;
    if ((rc = check_batch(batch))) return rc;
    if (!graph_exec) return fail(CAV_EINVAL, "graph_exec is NULL");
    const BatchGraph* g = static_cast<const BatchGraph*>(graph_exec);
    if (g->table != batch->table || g->items != batch->items)
        return fail(CAV_EINVAL, "the graph was captured from another batch table");
    if (g->parity != batch->parity)
        return fail(CAV_EINVAL,
                    "the batch's newest states moved (parity %d, captured at %d): an odd number of eager steps "
                    "ran since the capture; step once more or capture a new graph",
                    batch->parity, g->parity);
    const hipError_t e = run("batch_graph", stream, [&] { return hipGraphLaunch(g->exec, stream); });
    return e == hipSuccess ? CAV_OK : hip_fail("graph launch", e);
}

int cavity_batch_graph_destroy(void* graph_exec)
{
    if (!graph_exec) return CAV_OK;
    BatchGraph* g = static_cast<BatchGraph*>(graph_exec);
    const hipError_t e = hipGraphExecDestroy(g->exec);
    delete g;
    return e == hipSuccess ? CAV_OK : hip_fail("graph destroy", e);
}

int cavity_stream_copy(const cav_grid* grid, const void* q, void* q_tmp, hipStream_t stream)
{
    int rc;
    if ((rc = check_grid(grid))) return rc;
    if (!q || !q_tmp) return fail(CAV_EINVAL, "q and q_tmp must not be NULL");
    if (q == q_tmp) return fail(CAV_EINVAL, "q and q_tmp must be distinct buffers");
    const Dims d = dims_of(grid);
    hipError_t e = run("stream_copy", stream, [&] {
        return grid->dtype == CAV_F32
                   ? launch_stream_copy<float>(d, step_geom<float>(d, device_slots()), cstate_of<float>(q, d),
                                               state_of<float>(q_tmp, d), stream)
                   : launch_stream_copy<double>(d, step_geom<double>(d, device_slots()), cstate_of<double>(q, d),
                                                state_of<double>(q_tmp, d), stream);
    });
    return e == hipSuccess ? CAV_OK : hip_fail("stream copy launch", e);
}

int cavity_selftest_math(const double* x, double* out, int32_t n, hipStream_t stream)
{
    if (n < 0) return fail(CAV_EINVAL, "n = %d must be >= 0", n);
    if (n > 0 && (!x || !out)) return fail(CAV_EINVAL, "x and out must not be NULL");
    hipError_t e = launch_math(x, out, n, stream);
    return e == hipSuccess ? CAV_OK : hip_fail("math launch", e);
}

const char* cavity_last_error(void) { return g_err; }

int cavity_timing_enable(int32_t on)
{
    g_timing.store(on != 0);
    return CAV_OK;
}

int cavity_timing_read(cav_kernel_time* out, int32_t max_entries, int32_t* n_out)
{
    if (max_entries < 0 || (max_entries > 0 && !out)) return fail(CAV_EINVAL, "bad output array");
    std::lock_guard<std::mutex> lk(g_tm);
    std::vector<cav_kernel_time> acc;
    int rc = CAV_OK;
    for (const TimeRec& r : g_recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) rc = hip_fail("event timing", e);
        size_t k = 0;
        while (k < acc.size() && std::strcmp(acc[k].name, r.name)) ++k;
        if (k == acc.size()) {
            cav_kernel_time t;
            std::memset(&t, 0, sizeof t);
            std::snprintf(t.name, sizeof t.name, "%s", r.name);
            acc.push_back(t);
        }
        acc[k].launches += 1;
        acc[k].total_ms += ms;
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    const int n = (int)acc.size() < max_entries ? (int)acc.size() : max_entries;
    for (int k = 0; k < n; ++k) out[k] = acc[k];
    if (n_out) *n_out = (int32_t)acc.size();
    return rc;
}

}  // extern "C"
