// Internal declarations shared by the library's own sources (host ABI and
// kernels).  Not installed; the public interface is include/cavity.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cav {

constexpr int NG = 2;       // ghost layers per side
constexpr int NF = 5;       // fields p, u, v, w, T
enum Field { FP = 0, FU = 1, FV = 2, FW = 3, FT = 4 };

// Field base pointers of one state array (element type Real: double for the
// FP64 form, float for the FP32 form).  Cell offsets inside one field fit in
// 32 bits for every grid this library accepts (checked by the host).
template <typename Real>
struct StateT {
    Real* f[NF];
};
template <typename Real>
struct CStateT {
    const Real* f[NF];
};

// Padded state layout: every interior row starts on a 128-byte boundary
// (lead = 128 bytes of elements into its row), rows and planes are
// multiples of 128 bytes.  Cell (i, j, k) of a field sits at
// (k+NG)*sz + (j+NG)*sy + lead + i.
constexpr int ROW_ALIGN_BYTES = 128;

struct Dims {
    int ni, nj, nk;
    int sy;     // row pitch: lead + ni + NG rounded up to 128 bytes
    int sz;     // plane pitch: (nj + 2*NG) * sy
    int lead;   // elements before interior cell i = 0 in a row (NG of them ghosts)
};

__host__ __device__ inline int cell_off(const Dims& d, int i, int j, int k)
{
    return (k + NG) * d.sz + (j + NG) * d.sy + (i + d.lead);
}

// Per-cell coefficients of the residual (all derived on the host).
struct Coef {
    double hx2, hy2, hz2;     // 1/(2h) = n/2 per axis
    double ix2, iy2, iz2;     // 1/h^2 = n^2 per axis
    double nx, ny, nz;        // 1/h = n per axis
    double eps4;              // fourth-difference dissipation coefficient
    double beta2_floor;       // kappa * u_ref^2
    double nu, alpha;         // momentum and thermal diffusivities
    double t_inf;             // buoyancy reference temperature
    double cfl;
    double dt_visc;           // 1 / (2 max(nu, alpha) (nx^2 + ny^2 + nz^2))
    double t_hot, t_cold;     // hot (x = 0) and cold (x = 1) wall temperatures
    const double* t_hot_field;   // NULL, or nj*nk hot-wall temperatures (device, j fastest)
};

// Sweep launch geometry.
constexpr int SW_TI = 64;     // tile width along i (one wavefront)
constexpr int SW_TJ = 8;      // tile rows along j (one wavefront each)

// Shortest k chunk the launch geometry considers (planes per block).
#ifndef CAV_MIN_KC
#define CAV_MIN_KC 2
#endif

struct SweepGeom {
    int tiles_i, tiles_j;     // tiles per plane
    int kc;                   // k planes per block
    int nkc;                  // k chunks
    int nblocks;              // tiles_i * tiles_j * nkc
};
// slots: blocks resident at once; ti x tj: the tile of the launch
SweepGeom sweep_geom(const Dims& d, int slots, int ti = SW_TI, int tj = SW_TJ);
// Tile of the single-cavity step sweep in FP32: 32 x 8 threads, four
// wavefronts, so that three blocks stay resident per compute unit at that
// kernel's register count (FP64 keeps SW_TI x SW_TJ, one block of eight).
constexpr int F32_TI = 32, F32_TJ = 8;
#ifndef CAV_F64_STEP_TJ
#define CAV_F64_STEP_TJ 8
#endif
#ifndef CAV_F64_STEP_DEPTH
#define CAV_F64_STEP_DEPTH 3
#endif
#ifndef CAV_F64_STEP_WAVES
#define CAV_F64_STEP_WAVES 0
#endif
constexpr int F64_TI = 64, F64_TJ = CAV_F64_STEP_TJ;
// Geometry of the step sweep for element type Real on `cus` compute units
// (its tile, and the resident blocks per compute unit the occupancy query
// reports).
template <typename Real>
SweepGeom step_geom(const Dims& d, int cus);

struct Bcs {
    double t_hot, t_cold;
    const double* t_hot_field;   // NULL, or nj*nk hot-wall temperatures (device, j fastest)
};

// Halo geometry (virtual split, widths) shared by pack and unpack.
struct HaloGeom {
    int P[3];                 // subdomains along i, j, k
    int e[3];                 // subdomain extents
    int w[NF];                // widths
    int wsum;                 // sum of widths
    int wpre[NF];             // exclusive prefix sums of widths
    long long area[3];        // face area of an i, j, k face
    int nface[3];             // cut faces normal to i, j, k (both sides of every cut)
    int bpf[3];               // blocks per face normal to i, j, k
    int blk_end[3];           // end of each axis' block range in the launch (cumulative)
};
// Tangential cells one halo thread moves (all fields and layers of each),
// HALO_ROWS of them 256 apart (2: twice the blocks of 4 rows, so that the
// 2x2x2 exchange fills the chip: its pack 28.5 -> 24 us at 256^3).
constexpr int HALO_THREADS = 256;
constexpr int HALO_ROWS = 2;

// Tile shapes of the batched kernel, a wide and a narrow one per element
// type, both of the type's block size: FP64 64 x 8 and 32 x 16 (512
// threads); FP32 32 x 8 and 16 x 16 (256 threads, so that two blocks stay
// resident per compute unit).  The narrow shape wastes fewer lanes on
// narrow cavities.
constexpr int batch_threads(bool f32) { return f32 ? 256 : 512; }
constexpr int batch_wide_ti(bool f32) { return f32 ? 32 : 64; }
constexpr int batch_narrow_ti(bool f32) { return f32 ? 16 : 32; }
constexpr int batch_tj(bool f32, int ti) { return batch_threads(f32) / ti; }

// One member of a batch and one work item (a tile column's k chunk).
struct BatchCav {
    Dims d;
    int ti;                               // tile width: batch_wide_ti or batch_narrow_ti of the type
    int tiles_i, tiles_j, kc, ntiles;     // ntiles = tiles_i * tiles_j * (k chunks)
    Coef c;
    void* q;                              // state, q_tmp the scratch state
    void* q_tmp;
    double* ws;                           // workspace (norms, then partials)
    long long fstride;                    // elements per field
};
struct BatchItem {
    int cav, tile;
};
// The work list is cut into BATCH_SEGS contiguous segments of about equal
// cost, one per XCD: the items region of the table starts with the
// BATCH_SEGS + 1 segment bounds (padded to BATCH_HEAD_BYTES), then the
// items.  Blocks on XCD x (hardware ids dispatched round-robin over the 8
// XCDs) walk only segment x, so neighbouring tiles of a member run on one
// XCD and share its L2.
constexpr int BATCH_SEGS = 8;
constexpr int BATCH_HEAD_BYTES = 64;
constexpr int WS_HEAD_DOUBLES = 8;        // norms (5), Nusselt, padding

// Launchers (return hipGetLastError() of the launch); Real = double or float.
template <typename Real>
hipError_t launch_bc(const Dims& d, const Bcs& b, StateT<Real> q, hipStream_t s);
template <typename Real>
hipError_t launch_init(const Dims& d, double t_hot, double t_cold, uint64_t seed, double amp,
                       StateT<Real> q, hipStream_t s);
template <typename Real>
hipError_t launch_sweep(const Dims& d, const Coef& c, const SweepGeom& g, CStateT<Real> q, StateT<Real> qn,
                        double* partials, bool with_norm, hipStream_t s, const HaloGeom* xh = nullptr,
                        Real* xbuf = nullptr);
hipError_t launch_norm_finalize(const double* partials, int nblocks, double ncell, double* out,
                                hipStream_t s);
hipError_t launch_math(const double* x, double* out, int n, hipStream_t s);
// g comes from step_geom<Real>
template <typename Real>
hipError_t launch_stream_copy(const Dims& d, const SweepGeom& g, CStateT<Real> q, StateT<Real> qn, hipStream_t s);
// first_axis 1: only the j and k faces (their block ranges)
template <typename Real>
hipError_t launch_halo(const Dims& d, const HaloGeom& h, StateT<Real> q, Real* buf, bool pack,
                       hipStream_t s, int first_axis = 0);
template <typename Real>
// shapes: the tile shapes among the members (1 wide, 2 narrow, 3 both)
hipError_t launch_batch(const BatchCav* cavs, const int* segs, const BatchItem* items, int parity, bool with_norm,
                        int nblocks, int shapes, hipStream_t s);
hipError_t launch_batch_norms(const BatchCav* cavs, int members, hipStream_t s);
template <typename Real>
hipError_t launch_nusselt(const Dims& d, const Bcs& b, CStateT<Real> q, double* out,
                          hipStream_t s);

// Interior/exterior split of the sweep around the cuts of a virtual split:
// P subdomains of extent e per axis; a cell within m of a cut is exterior;
// exterior x and y slabs are cut into k chunks of kce planes.
struct SplitGeom {
    int P[3], e[3], m, kce;
};
int exterior_blocks(const Dims& d, const SweepGeom& g, const SplitGeom& sg);
template <typename Real>
hipError_t launch_split(const Dims& d, const Coef& c, const SweepGeom& gi, const SweepGeom& g, const SplitGeom& sg,
                        bool exterior, CStateT<Real> q, StateT<Real> qn, double* partials, bool with_norm,
                        hipStream_t s);

// Discrete adjoint (FP64): workspace size in doubles, one reverse step, and
// the cotangent of the mean hot-wall Nusselt number (scale = ni/3/(nj nk dT)).
// g: the record pass (sweep_geom); gg: the gather (gather_geom).
size_t adjoint_ws_doubles(const Dims& d);
SweepGeom gather_geom(const Dims& d, int cus);
hipError_t launch_adjoint_step(const Dims& d, const Coef& c, const SweepGeom& g, const SweepGeom& gg, double Ra,
                               CStateT<double> q, CStateT<double> lam_in, StateT<double> lam_out, double* ws,
                               double* dthot, double* dra, hipStream_t s);
hipError_t launch_nusselt_seed(const Dims& d, double scale, StateT<double> lam, double* dthot, hipStream_t s);

}  // namespace cav
