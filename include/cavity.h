/*
 * cavity.h -- C ABI of the MI355X cavity library (libcavity.so).
 *
 * One GPU's share of an explicit pseudo-time solver for the 3D buoyancy-driven
 * cavity (Xue & Roy, "Multi-GPU Performance Optimization of a CFD Code using
 * OpenACC on Different Platforms", arXiv:2006.02602):
 *   - the residual + first-order Euler update sweep of the artificial-
 *     compressibility Boussinesq equations (Sec. 2, Eq. 1-3; Sec. 3.1),
 *     with the wall boundary conditions and the per-iteration pressure
 *     rescale at the cavity centre (Sec. 2),
 *   - in-device packing / unpacking of noncontiguous halo faces into one
 *     contiguous buffer with a ghost width per variable (Sec. 4.5,
 *     "Optimized V1/V2/V3", Listings 1-2),
 * and around them: an FP32 precision form, a batched form (many cavities,
 * one launch per step, graph replay), the interior/exterior split step of
 * Sec. 4.7 (the exchange on a second stream), and the discrete adjoint of
 * the step and of the hot-wall Nusselt number.
 *
 * Conventions shared by every call
 *   - State layout.  q is ONE allocation of 5 fields in the order
 *     p, u, v, w, T (Listing 2: var 1 is pressure, vars 2..5 the velocities
 *     and temperature), i fastest and k slowest (Sec. 3.1), (i,j,k) = (x,y,z),
 *     with g = ng = 2 ghost layers per side (Sec. 4.5, Listing 1, whose
 *     1-based arrays keep two ghost layers before the first interior cell).  Rows are padded so that every interior row starts on
 *     a 128-byte boundary (when q is 128-byte aligned): field f, cell
 *     (i, j, k) with -2 <= i < ni+2 etc. lives at element
 *         f*sf + (k+2)*sk + (j+2)*sj + lead + i
 *     with lead = 128 bytes of elements (16 doubles or 32 floats),
 *     sj = (lead + ni + 2) rounded up to a multiple of lead,
 *     sk = (nj+4)*sj, sf = (nk+4)*sk (cavity_layout returns them).  Interior
 *     cells are 0 <= i < ni etc.  cavity_init also fills the face ghost
 *     layers; no step reads a ghost cell (their contents after a step are
 *     unspecified).  Element type: double for CAV_F64, float for
 *     CAV_F32 (the halo buffer uses the same element type).
 *   - Pointers are DEVICE pointers unless the comment says (host).  The
 *     caller owns every buffer; the library allocates no device memory and
 *     keeps no pointer after a call returns.
 *   - Every call enqueues its work on `stream` (0 = the null stream) and
 *     returns without waiting, except cavity_residual_norm, cavity_nusselt,
 *     cavity_batch_build and cavity_timing_read, which wait (each says so).
 *   - Arguments are validated on the host BEFORE anything is enqueued; on
 *     any error nothing is enqueued and a negative CAV_E* code is returned.
 *     cavity_last_error() then describes the failure (thread-local text).
 *   - The library keeps no per-problem state: calls are reentrant, but two
 *     calls that write the same buffers must be ordered by the caller.
 */
#ifndef CAVITY_H_
#define CAVITY_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define CAV_OK          0
#define CAV_EINVAL    (-1)  /* bad argument: null pointer, sizes, split, widths */
#define CAV_ESIZE     (-2)  /* a caller buffer is smaller than required        */
#define CAV_EHIP      (-3)  /* a HIP launch or runtime call failed             */
#define CAV_ENONFINITE (-4) /* a residual norm is NaN or infinite              */
#define CAV_ENOSYS    (-5)  /* operation not available (reserved)              */

/* ---- element types ---------------------------------------------------- */
#define CAV_F64 0   /* state and stencil arithmetic in FP64                  */
#define CAV_F32 1   /* state and stencil arithmetic in FP32; residual norms and
                       the Nusselt integral still accumulate in FP64       */

/* Grid of one cavity (or one GPU's block of it).  ni, nj, nk >= 2 interior
 * cells; ng must be 2 (the pressure stencil reaches two cells, Sec. 3.1). */
typedef struct {
    int32_t ni, nj, nk;
    int32_t ng;
    int32_t dtype;          /* CAV_F64 or CAV_F32 */
} cav_grid;

/* Physical and numerical parameters (Sec. 2).  Nondimensional, free-fall
 * scaling on the unit cube: nu = sqrt(Pr/Ra), alpha = 1/sqrt(Ra*Pr),
 * buoyancy +(T - t_inf) along +z.  The hot wall is x = 0, the cold wall
 * x = 1, the other four walls adiabatic.
 *   cfl    pseudo-time CFL number of the local time step
 *   eps4   coefficient of the fourth-difference pressure dissipation (Eq. 1)
 *   kappa, u_ref   artificial compressibility: beta^2 = max(|V|^2, kappa*u_ref^2)
 *   t_hot_field    NULL (the hot wall is at t_hot), or a DEVICE array of
 *                  nj*nk doubles, j fastest: the hot-wall temperature next
 *                  to each (j, k) row.  Borrowed; it must stay valid until
 *                  the work of every call given it has completed.  Its
 *                  values enter the wall ghosts and the Nusselt integral;
 *                  cavity_init still starts T linear between t_hot and
 *                  t_cold.  The normalisation of the Nusselt number keeps
 *                  the scalar t_hot - t_cold. */
typedef struct {
    double Ra, Pr, cfl, eps4, kappa, u_ref, t_hot, t_cold, t_inf;
    const void* t_hot_field;
} cav_params;

/* Virtual domain decomposition for the halo exchange (Sec. 3.2; Sec. 4.5).
 * split = (Pi, Pj, Pk) subdomains along i, j, k; each must divide the grid
 * extent.  width[f] = ghost layers exchanged for field f (order p,u,v,w,T),
 * 0 <= width[f] <= ng and width[f] <= every subdomain extent.  The paper's
 * stencil-based widths (Optimized V2) are {2,1,1,1,1}. */
typedef struct {
    int32_t split[3];
    int32_t width[5];
} cav_halo;

/* Element strides of the state layout (see "State layout" above):
 * cell (f, i, j, k) is at origin + f*sf + k*sk + j*sj + i, where
 * origin = 2*sk + 2*sj + lead is the element of interior cell (0, 0, 0). */
typedef struct {
    int64_t lead, sj, sk, sf, origin;
} cav_layout;

int cavity_layout(const cav_grid* grid, cav_layout* out);

/* Number of elements of one state array (all 5 fields, ghosts and row
 * padding included): 5*sf.  Returns 0 for an invalid grid. */
size_t cavity_state_elems(const cav_grid* grid);

/* Bytes of the workspace `ws` that cavity_step and cavity_residual_norm
 * need (per-block residual partials and the final norms).  0 if invalid. */
size_t cavity_workspace_bytes(const cav_grid* grid);

/* Bytes of the contiguous halo buffer for `halo` on `grid` (Sec. 4.5):
 * sum over subdomains s = a + Pi*(b + Pj*c), over the cut faces of s in
 * the order -x,+x,-y,+y,-z,+z (faces on a cavity wall are skipped), over
 * the fields p,u,v,w,T with width > 0, of width * (face area of s) *
 * sizeof(element).  Within a segment, elements run over the sender's box
 * of `width` layers next to the face in (k, j, i) order, i fastest
 * (Listing 1's index order).  Returns 0 for invalid arguments. */
size_t halo_buffer_bytes(const cav_grid* grid, const cav_halo* halo);

/* Seeded initial state (not part of the timed path).  Interior:
 *   u, v, w = noise(seed, 1..3, idx), p = 0,
 *   T = t_hot + (t_cold - t_hot) * (i + 1/2)/ni + noise(seed, 4, idx),
 * where idx = i + ni*(j + nj*k) and noise(seed, f, idx) = (2r - 1)*noise_amp
 * with r = (z >> 11) * 2^-53, z the output number f*2^40 + idx (0-based) of
 * the SplitMix64 generator seeded with `seed` (Steele, Lea & Flood, 2014).
 * Then the face ghost layers are filled with the wall rules of cavity_step.
 * q: device, cavity_state_elems(grid) elements, written. */
int cavity_init(const cav_grid* grid, const cav_params* prm, uint64_t seed,
                double noise_amp, void* q, hipStream_t stream);

/* Advance the state `nsteps` >= 0 pseudo-time steps (Sec. 2; Sec. 3.1).
 * Each step, in this order:
 *   1. if halo != NULL: halo_pack into halo_buf, then halo_unpack from it
 *      (all virtual subdomains live in q, so the exchange is a round trip),
 *   2. for every interior cell: residuals R_p, R_u, R_v, R_w, R_T of
 *      Eq. 1-3 (second-order central differences; fourth-difference
 *      pressure dissipation), local time step, q' = q + dt*R written to
 *      q_tmp (Jacobi: every residual uses the old state).  The wall ghost
 *      values the stencils reach (Sec. 2: no-slip velocity; T fixed on the
 *      hot/cold walls and zero-gradient on the adiabatic walls, second
 *      order; p extrapolated linearly, one-sided second order) are derived
 *      from interior cells as they are loaded: no ghost cell of q or q_tmp
 *      is read,
 *   3. p' -= p'(ni/2, nj/2, nk/2) over the interior (Sec. 2, rescale at the
 *      centre point every iteration),
 *   4. swap q and q_tmp.
 * On return the newest state is in q (for odd nsteps the library copies it
 * back from q_tmp); q_tmp holds scratch.  The residual L2 norms of the last
 * step are left in ws for cavity_residual_norm.
 * q, q_tmp: device, cavity_state_elems(grid) elements each, distinct.
 * ws: device, >= cavity_workspace_bytes(grid) = ws_bytes.
 * halo_buf: device, >= halo_buffer_bytes(grid, halo) = halo_bytes; ignored
 * (may be NULL) when halo == NULL. */
int cavity_step(const cav_grid* grid, const cav_params* prm, const cav_halo* halo,
                void* q, void* q_tmp, void* ws, size_t ws_bytes,
                void* halo_buf, size_t halo_bytes, int32_t nsteps,
                hipStream_t stream);

/* One pseudo-time step out of place (Sec. 2; Sec. 3.1): the state after one
 * step of cavity_step without a halo, read from q_in and written to q_out
 * (q_in is left unchanged), as a recomputation from a checkpoint needs it.
 * q_in, q_out: device, cavity_state_elems(grid) elements each, distinct; only
 * the interior cells of q_out are written.  ws: device workspace as for
 * cavity_step (the step's residual norms are left there for
 * cavity_residual_norm), or NULL to skip the norm pass. */
int cavity_step_from(const cav_grid* grid, const cav_params* prm, const void* q_in,
                     void* q_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* Largest number of sweep blocks whose norm partials cavity_step_noalloc's
 * static scratch holds (5 doubles each: 1.25 MiB per device). */
#define CAV_NOALLOC_MAX_SWEEP_BLOCKS 32768

/* cavity_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same kernels, launches and results as cavity_step, with no workspace
 * argument.  The per-block norm partials live in a static device array of
 * the library (CAV_NOALLOC_MAX_SWEEP_BLOCKS blocks), one per device, held
 * until the process ends; the call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine; it never records timing events),
 * and looks the array's address up on its first call on each device.
 * norms: device, 5 doubles (p, u, v, w, T), written with the residual L2
 * norms of the last step; or NULL, which skips the norm pass.
 * Every call on one device shares that device's array, and every sweep
 * that computes norms overwrites its own partials first, so nothing needs
 * clearing between calls; two calls that overlap in time on one device
 * (on different streams, or from several threads) race on it and must
 * not be issued.  CAV_ESIZE when norms != NULL and the grid's sweep needs
 * more blocks than the array holds (every cube up to the largest accepted
 * grid fits; only very flat grids exceed it).  Other arguments and errors
 * as for cavity_step. */
int cavity_step_noalloc(const cav_grid* grid, const cav_params* prm, const cav_halo* halo,
                        void* q, void* q_tmp, void* halo_buf, size_t halo_bytes,
                        double* norms, int32_t nsteps, hipStream_t stream);

/* cavity_step with the interior/exterior split of Sec. 4.7: per step the
 * exchange (halo_pack, halo_unpack) runs on comm_stream while the cells
 * whose stars reach no unpacked cell (the interior) are updated on
 * `stream`; the cells within m of a cut (the exterior; m = the largest
 * width[f] + reach of field f's star, reach 2 for p and 1 for u v w T) are
 * updated on `stream` after the exchange.  Each cell goes through the same
 * per-cell arithmetic as in cavity_step, so q after the call is bit-identical
 * to cavity_step's; the residual norms agree to rounding (their partial sums
 * are grouped by launch).  Every subdomain extent along a split axis must
 * be >= 2m (CAV_EINVAL otherwise).  halo must not be NULL.  comm_stream
 * may equal `stream` (no overlap, same results).  Ordering between the two
 * streams uses two events created and destroyed by the call; when `stream`
 * has completed, so has all work of the call.  Other arguments as for
 * cavity_step; CAV_ESIZE when the norm partials of the split do not fit
 * ws (only for grids with very few planes). */
int cavity_step_overlap(const cav_grid* grid, const cav_params* prm, const cav_halo* halo,
                        void* q, void* q_tmp, void* ws, size_t ws_bytes,
                        void* halo_buf, size_t halo_bytes, int32_t nsteps,
                        hipStream_t stream, hipStream_t comm_stream);

/* Gather every halo segment of `halo` (layout: halo_buffer_bytes) from q
 * into the contiguous buffer buf (Sec. 4.5, Listings 1-2: the parallel
 * in-device pack of the "Optimized" versions; V3 covers i, j and k faces).
 * One kernel launch.  q: device, read.  buf: device, buf_bytes >=
 * halo_buffer_bytes(grid, halo), written. */
int halo_pack(const cav_grid* grid, const cav_halo* halo, const void* q,
              void* buf, size_t buf_bytes, hipStream_t stream);

/* Scatter buf back into the ghost boxes of the receiving subdomains (the
 * unpack of Sec. 4.5).  With all subdomains in one array the receiver's
 * ghost box beyond a face is the sender's box, so
 * halo_unpack(halo_pack(q)) leaves q bit-identical.  One kernel launch.
 * buf: device, read.  q: device, written on the segment cells only. */
int halo_unpack(const cav_grid* grid, const cav_halo* halo, const void* buf,
                size_t buf_bytes, void* q, hipStream_t stream);

/* Residual L2 norms of the last step run by cavity_step on this ws:
 * out5[f] = sqrt(sum over interior cells of R_f^2 / (ni*nj*nk)), f in
 * p,u,v,w,T order (Sec. 4.2 mentions residual norms, printed outside the
 * timed runs).  Reduced in FP64 in a fixed order (run-to-run identical).
 * out5: HOST, 5 doubles.  Waits for `stream`.  Returns CAV_ENONFINITE if
 * any norm is NaN or infinite (the values are still written). */
int cavity_residual_norm(const cav_grid* grid, const void* ws, size_t ws_bytes,
                         double* out5, hipStream_t stream);

/* Mean Nusselt number of the hot wall x = 0 of state q, accumulated in
 * FP64 (either dtype): the wall heat flux -dT/dx from the second-order
 * one-sided difference (9 T_0 - T_1 - 8 t_hot) / (3h), h = 1/ni, through the
 * wall value and the first two cell centres, averaged over the wall and
 * divided by t_hot - t_cold (Sec. 2: the cavity carries heat between its
 * hot and cold vertical walls).  q: device, read.  ws: device workspace
 * (>= cavity_workspace_bytes).  out: HOST, 1 double.  Waits for `stream`. */
int cavity_nusselt(const cav_grid* grid, const cav_params* prm, const void* q,
                   void* ws, size_t ws_bytes, double* out, hipStream_t stream);

/* ---- discrete adjoint (reverse mode), FP64 only ------------------------
 * Objective: the mean hot-wall Nusselt number J = Nu(q^N) of the state
 * after N steps (cavity_nusselt).  Parameters: the hot-wall temperatures
 * Theta (t_hot_field, or t_hot on every row) and Ra.  The adjoint of one
 * step is the transpose of the exact derivative of the step that
 * cavity_step computes (Sec. 2, Eq. 1-3: wall ghosts, residual, local time
 * step, explicit update, centre rescale of p), written by hand; at the
 * non-smooth points it takes one side: |u| has slope +1 at u = 0,
 * beta^2 = max(|V|^2, kappa u_ref^2) follows |V|^2 only where strictly
 * larger, dt follows the convective limit only where strictly smaller.
 * The halo exchange of the virtual split is the identity on the state, so
 * it has no adjoint term.
 * A gradient is formed as: lam = cavity_nusselt_adjoint; for n = N-1 .. 0:
 * cavity_adjoint_step(q^n, lam -> lam); then lam is dJ/dq^0 on the interior
 * cells, dj_dthot dJ/dTheta and dj_dra dJ/dRa (both zeroed by the caller
 * first).  q^n must be the states of the forward run (kept, or recomputed
 * from checkpoints); every call must get the same params as the forward. */

/* Bytes of the workspace cavity_adjoint_step needs (in doubles: 8, the
 * per-block partial sums, and 8 values per cell); 0 for an invalid grid or
 * a CAV_F32 grid. */
size_t cavity_adjoint_workspace_bytes(const cav_grid* grid);

/* Cotangent of J = Nu(q): writes lam (device, state layout, interior cells;
 * zero except T in the first two cells off the hot wall) and ADDS dNu/dTheta
 * (8 ni / (3 nj nk (t_hot - t_cold)) per row) into dj_dthot (device, nj*nk
 * doubles, j fastest; NULL to skip).  Asynchronous on `stream`.
 * CAV_EINVAL for a CAV_F32 grid or t_hot == t_cold. */
int cavity_nusselt_adjoint(const cav_grid* grid, const cav_params* prm, void* lam,
                           double* dj_dthot, hipStream_t stream);

/* One reverse step: given lam_in = dJ/dq^{n+1} (device, state layout,
 * interior cells read) and q_n (device, the state the forward step started
 * from, interior cells read), writes lam_out = dJ/dq^n on the interior cells
 * (its ghost cells are used as scratch and left unspecified) and ADDS this
 * step's terms into dj_dthot (device, nj*nk doubles, j fastest) and dj_dra
 * (device, 1 double); either may be NULL to skip it.  lam_out must not
 * overlap lam_in (the gather reads lam_in at every cell's neighbours while
 * it writes lam_out) or q_n; CAV_EINVAL when it equals either.  ws: device, >=
 * cavity_adjoint_workspace_bytes.  Two launches on `stream` (the record
 * pass; the gather, which also forms the rescale sum and the Ra sum), no
 * allocation, no synchronisation.  CAV_EINVAL for a CAV_F32 grid. */
int cavity_adjoint_step(const cav_grid* grid, const cav_params* prm,
                        const void* q_n, const void* lam_in, void* lam_out,
                        void* ws, size_t ws_bytes, double* dj_dthot,
                        double* dj_dra, hipStream_t stream);

/* ---- batched form: many independent cavities, one launch per step -------
 * A batch advances n cavities of arbitrary sizes and parameters (all of one
 * dtype) together: every step is ONE launch of a persistent kernel whose
 * blocks walk a device work list of (cavity, tile column, k chunk) items,
 * each computed with the per-cell code of cavity_step, so every member's
 * state is bit-identical to advancing it alone, whatever its tile shape and
 * k-chunk length (only the grouping of the norm sums differs).  There is no halo exchange in the batched form. */
typedef struct {
    cav_grid grid;          /* member grid; dtype must match the batch      */
    cav_params params;      /* member parameters                             */
    void* q;                /* device state, cavity_state_elems(grid) elems */
    void* q_tmp;            /* device scratch state, same size, distinct    */
    void* ws;               /* device workspace                              */
    size_t ws_bytes;        /* >= cavity_workspace_bytes(grid)               */
    int32_t kc;             /* k planes per work item, 0 = whole columns    */
    int32_t ti;             /* tile width: 0 = the wide shape; CAV_F64:
                               64 = 64 x 8 or 32 = 32 x 16 columns (512
                               threads); CAV_F32: 32 = 32 x 8 or 16 = 16 x
                               16 (256 threads).  The narrow shape wastes
                               fewer lanes on narrow cavities; the result
                               does not depend on it; other values are
                               CAV_EINVAL                                   */
} cav_batch_member;

/* Host handle of a built batch (plain data; owns nothing). */
typedef struct {
    const void* table;      /* device table written by cavity_batch_build   */
    int32_t members, items, dtype;
    int32_t parity;         /* 0: newest states in q, 1: in q_tmp            */
    uint64_t cells;         /* interior cells over all members               */
    int32_t shapes;         /* tile shapes among the members: 1 the wide one
                               only, 2 the narrow one only, 3 both (a batch
                               of one shape runs a kernel compiled for it)   */
    int32_t reserved;
} cav_batch;

/* Bytes of the device table for these members (host array of n). */
size_t cavity_batch_table_bytes(int32_t n, const cav_batch_member* members);

/* Validate the members, write the work list and per-member descriptors into
 * `table` (device, >= cavity_batch_table_bytes) and fill *out.  Waits for
 * `stream` (the table is staged from host memory). */
int cavity_batch_build(int32_t n, const cav_batch_member* members, void* table,
                       size_t table_bytes, cav_batch* out, hipStream_t stream);

/* Advance every member nsteps pseudo-time steps (same step as cavity_step
 * without a halo): one persistent launch of `nblocks` blocks per step
 * (0 = one per compute unit), then one norm-finalize launch for all
 * members; each member's last-step residual norms land in its ws.  The
 * q/q_tmp roles alternate: batch->parity tells where the newest states are
 * (it is updated). */
int cavity_batch_step(cav_batch* batch, int32_t nsteps, int32_t nblocks, hipStream_t stream);

/* Capture nsteps (even, >= 2) batch steps on `stream` into a HIP graph and
 * instantiate it; *graph_exec receives a handle (host memory owned by the
 * library until cavity_batch_graph_destroy releases it).  The captured
 * launches read the newest states from where batch->parity says they were
 * at capture, and hold the table's address and item count.
 * cavity_batch_graph_launch(batch, ...) replays the nsteps steps (the
 * parity stays the same, nsteps being even); it returns CAV_EINVAL and
 * enqueues nothing when batch->parity differs from the captured one (an odd
 * number of eager cavity_batch_step steps ran since) or when batch->table /
 * batch->items are not the captured ones (the table was rebuilt).  A
 * rebuild into the same memory (cavity_batch_build) is not detectable by
 * address: destroy the graph before rebuilding. */
int cavity_batch_graph_create(const cav_batch* batch, int32_t nsteps, int32_t nblocks,
                              hipStream_t stream, void** graph_exec);
int cavity_batch_graph_launch(const cav_batch* batch, void* graph_exec, hipStream_t stream);
int cavity_batch_graph_destroy(void* graph_exec);

/* Measurement support: the memory streams of cavity_step's sweep without its
 * work.  Copies the interior cells of all five fields of q into q_tmp with
 * the sweep's tiles, block order, k chunks and prefetch depth, each value
 * read once and written once (non-temporal stores); no halo loads, no LDS,
 * no arithmetic.  Its rate bounds what the sweep's access pattern can reach
 * on the device.  q: device, read; q_tmp: device, interior cells written
 * (ghost cells untouched); both cavity_state_elems(grid) elements. */
int cavity_stream_copy(const cav_grid* grid, const void* q, void* q_tmp, hipStream_t stream);

/* Test support: the FP64 square root and reciprocal the step's residual uses
 * (the hardware estimates refined to within an ulp), on n arguments.
 * x: device, n doubles > 0 (read); out: device, 2n doubles, written with
 * out[2m] = sqrt(x[m]) and out[2m+1] = 1/x[m] as the kernels compute them. */
int cavity_selftest_math(const double* x, double* out, int32_t n, hipStream_t stream);

/* Thread-local description of the last error returned on this thread. */
const char* cavity_last_error(void);

/* ---- per-kernel timing (measurement support) ---------------------------
 * While enabled, every kernel the library launches is bracketed by a pair
 * of HIP events recorded on the stream the kernel is launched on.
 * cavity_timing_read waits for those events, returns per-kernel totals
 * (at most max_entries, names as in the rocprofv3 kernel trace prefix)
 * and clears them. */
typedef struct {
    char    name[32];
    int64_t launches;
    double  total_ms;
} cav_kernel_time;

int cavity_timing_enable(int32_t on);
int cavity_timing_read(cav_kernel_time* out, int32_t max_entries, int32_t* n_out);

#ifdef __cplusplus
}
#endif
#endif /* CAVITY_H_ */
