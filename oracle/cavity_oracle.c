/*
 * cavity_oracle.c -- TEST INFRASTRUCTURE ONLY (see cavity_oracle.h).
 *
 * The explicit pseudo-time solver of the 3D buoyancy-driven cavity of
 * Xue & Roy (arXiv:2006.02602), written as plain loops in FP64, in the order
 * the method states it.  Built with -O2 -ffp-contract=off (no fused
 * multiply-add, no fast-math), optionally with OpenMP over k-planes; every
 * reduction is summed in a fixed order so results do not depend on the
 * thread count.
 *
 * The paper gives the equations (Sec. 2, Eq. 1-3), the stencil widths
 * (Sec. 3.1), the boundary-condition wording and the centre rescale (Sec. 2)
 * and the pack/unpack loops (Sec. 4.5, Listings 1-2), but no numerical
 * constants.  Every reading of a point the paper leaves open is marked
 * "Reading:" below.
 */
#include "cavity_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 2                      /* ghost layers per side */
enum { FP = 0, FU = 1, FV = 2, FW = 3, FT = 4, NF = 5 };

/* Index of field f, cell (i, j, k) with interior cells at 0..n-1 and
 * ghosts at -2, -1, n, n+1 (two ghost layers per side, Sec. 4.5, Listing 1). */
static inline size_t at(const orc_problem* P, int f, int i, int j, int k)
{
    size_t sx = (size_t)P->ni + 2 * NG, sy = (size_t)P->nj + 2 * NG, sz = (size_t)P->nk + 2 * NG;
    return (((size_t)f * sz + (size_t)(k + NG)) * sy + (size_t)(j + NG)) * sx + (size_t)(i + NG);
}

size_t orc_state_elems(const orc_problem* P)
{
    return (size_t)NF * (P->ni + 2 * NG) * (P->nj + 2 * NG) * (P->nk + 2 * NG);
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Seeded initial state.  SplitMix64 (Steele, Lea & Flood, OOPSLA 2014):
 * state advances by the golden-ratio increment, output = mix(state).
 * orc_splitmix64(seed, n) is output number n (0-based) of the stream
 * seeded with `seed`. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Uniform in [-amp, amp): r = top 53 bits / 2^53 in [0,1), 2r-1 is exact. */
static double noise(uint64_t seed, int f, size_t idx, double amp)
{
    uint64_t z = orc_splitmix64(seed, ((uint64_t)f << 40) + (uint64_t)idx);
    double r = (double)(z >> 11) * 0x1.0p-53;
    return (2.0 * r - 1.0) * amp;
}

/* Initial field: fluid at rest up to noise, p = 0, T linear between the
 * hot (x = 0) and cold (x = 1) walls plus noise; then the wall ghosts. */
void orc_init(const orc_problem* P, uint64_t seed, double amp, double* q)
{
    memset(q, 0, orc_state_elems(P) * sizeof(double));
    for (int k = 0; k < P->nk; ++k)
        for (int j = 0; j < P->nj; ++j)
            for (int i = 0; i < P->ni; ++i) {
                size_t idx = (size_t)i + (size_t)P->ni * ((size_t)j + (size_t)P->nj * (size_t)k);
                double xc = ((double)i + 0.5) / (double)P->ni;
                q[at(P, FP, i, j, k)] = 0.0;
                q[at(P, FU, i, j, k)] = noise(seed, 1, idx, amp);
                q[at(P, FV, i, j, k)] = noise(seed, 2, idx, amp);
                q[at(P, FW, i, j, k)] = noise(seed, 3, idx, amp);
                q[at(P, FT, i, j, k)] = (P->t_hot + (P->t_cold - P->t_hot) * xc) + noise(seed, 4, idx, amp);
            }
    orc_apply_bc(P, q);
}

/* ------------------------------------------------------------------ */
/* Wall boundary conditions (Sec. 2).  Cell-centred grid, walls on the cell
 * faces at 0 and 1; ghost g = 1, 2 is the g-th cell outside the wall and
 * mirrors interior cell g-1.
 *  - u, v, w: no-slip, odd reflection (wall value 0).
 *  - T: Dirichlet on the hot (x = 0) and cold (x = 1) walls by odd
 *    reflection about the wall value; zero normal gradient (even mirror,
 *    second order at the face) on the four adiabatic walls.
 *  - p: one-sided linear extrapolation on all six walls (second order):
 *    p_{-1} = 2 p_0 - p_1, then p_{-2} = 2 p_{-1} - p_0.
 * Reading: the paper names the p and T extrapolations only for the
 * adiabatic walls; the same p rule is used on the hot/cold walls.
 * Only face ghosts are written; edge and corner ghosts are never read. */
static void bc_line(double* q, size_t i0, ptrdiff_t s, int kind, double wall)
{
    /* q[i0 + s*m] is interior cell m (m = 0, 1); ghost g sits at -g. */
    double a = q[i0], b = q[i0 + s];
    switch (kind) {
    case 0: /* odd about 0 */
        q[i0 - s] = -a;
        q[i0 - 2 * s] = -b;
        break;
    case 1: /* odd about `wall` (Dirichlet) */
        q[i0 - s] = 2.0 * wall - a;
        q[i0 - 2 * s] = 2.0 * wall - b;
        break;
    case 2: /* even (zero gradient) */
        q[i0 - s] = a;
        q[i0 - 2 * s] = b;
        break;
    default: { /* linear extrapolation */
        double g1 = 2.0 * a - b;
        q[i0 - s] = g1;
        q[i0 - 2 * s] = 2.0 * g1 - a;
    }
    }
}

void orc_apply_bc(const orc_problem* P, double* q)
{
    const ptrdiff_t sx = 1, sy = P->ni + 2 * NG, sz = (ptrdiff_t)(P->ni + 2 * NG) * (P->nj + 2 * NG);
    const int kind[NF] = {3, 0, 0, 0, 2};   /* p, u, v, w, T (adiabatic) */
    for (int f = 0; f < NF; ++f) {
        /* x walls */
        for (int k = 0; k < P->nk; ++k)
            for (int j = 0; j < P->nj; ++j) {
                int kx = kind[f];
                double wlo = 0.0, whi = 0.0;
                if (f == FT) {
                    kx = 1;
                    wlo = P->t_hot_field ? P->t_hot_field[j + (size_t)P->nj * k] : P->t_hot;
                    whi = P->t_cold;
                }
                bc_line(q, at(P, f, 0, j, k), sx, kx, wlo);
                bc_line(q, at(P, f, P->ni - 1, j, k), -sx, kx, whi);
            }
        /* y walls */
        for (int k = 0; k < P->nk; ++k)
            for (int i = 0; i < P->ni; ++i) {
                bc_line(q, at(P, f, i, 0, k), sy, kind[f], 0.0);
                bc_line(q, at(P, f, i, P->nj - 1, k), -sy, kind[f], 0.0);
            }
        /* z walls */
        for (int j = 0; j < P->nj; ++j)
            for (int i = 0; i < P->ni; ++i) {
                bc_line(q, at(P, f, i, j, 0), sz, kind[f], 0.0);
                bc_line(q, at(P, f, i, j, P->nk - 1), -sz, kind[f], 0.0);
            }
    }
}

/* ------------------------------------------------------------------ */
/* Residual of one interior cell (Sec. 2, Eq. 1-3; Sec. 3.1).
 *
 * Nondimensional form (Reading: free-fall scaling on the unit cube, since
 * the paper's dimensional constants are not given): rho = 1,
 * nu = sqrt(Pr/Ra), alpha = 1/sqrt(Ra*Pr), gravity along -z, so the
 * buoyancy term sigma*(T - T_inf)*g_j of Eq. 2 is +(T - t_inf) in the
 * w equation (hot fluid rises).
 *
 * Artificial compressibility (Eq. 1; Reading of "local velocity magnitude
 * along with a reference velocity"): beta^2 = max(|V|^2, kappa*u_ref^2).
 *
 * Second-order central differences (Sec. 3.1), with h_x = 1/ni etc.:
 *   D_x q = (q_{i+1} - q_{i-1}) / (2 h_x)
 *   L_x q = ((q_{i+1} + q_{i-1}) - 2 q_i) / h_x^2
 * Fourth-difference pressure dissipation on the continuity equation only
 * (Sec. 2: alleviates odd-even decoupling; 5-point stencil, Sec. 3.1):
 *   F_x p = ((p_{i+2} + p_{i-2}) - 4 (p_{i+1} + p_{i-1})) + 6 p_i
 * Reading of Eq. 1's right-hand side: its coefficient is the spectral-
 * radius-scaled, damping-signed -eps4 * lambda_x * h_x^3 / beta^2, so after
 * multiplying Eq. 1 by beta^2 the term is -eps4 * lambda_x * F_x p / h_x,
 * with lambda_x = (|u| + sqrt(u^2 + 4 beta^2)) / 2 the largest eigenvalue
 * modulus of the 1D artificial-compressibility system along x.
 *
 * Pseudo-time residuals (the right-hand sides of Eq. 1 times beta^2, and
 * of Eq. 2-3 in advective form):
 *   R_p = -beta^2 rho (D_x u + D_y v + D_z w)
 *         - eps4 (lambda_x F_x p / h_x + lambda_y F_y p / h_y + lambda_z F_z p / h_z)
 *   R_u = -(u D_x u + v D_y u + w D_z u) - D_x p / rho + nu (L_x + L_y + L_z) u
 *   R_v, R_w likewise, R_w adds (T - t_inf)
 *   R_T = -(u D_x T + v D_y T + w D_z T) + alpha (L_x + L_y + L_z) T
 * Local time step (Reading: per-cell, first-order explicit Euler in
 * pseudo time, Sec. 2):
 *   dt = cfl * min(1 / (lambda_x/h_x + lambda_y/h_y + lambda_z/h_z),
 *                  1 / (2 max(nu, alpha) (1/h_x^2 + 1/h_y^2 + 1/h_z^2)))
 */
typedef struct {
    double nu, alpha, rho, beta2_floor;
} orc_consts;

static orc_consts consts_of(const orc_problem* P)
{
    orc_consts c;
    c.nu = sqrt(P->Pr / P->Ra);
    c.alpha = 1.0 / sqrt(P->Ra * P->Pr);
    c.rho = 1.0;
    c.beta2_floor = P->kappa * P->u_ref * P->u_ref;
    return c;
}

static void cell_residual(const orc_problem* P, const orc_consts* C, const double* q,
                          int i, int j, int k, double R[NF], double* dt)
{
    const double nx = (double)P->ni, ny = (double)P->nj, nz = (double)P->nk;  /* 1/h */
#define Q(f, di, dj, dk) q[at(P, (f), i + (di), j + (dj), k + (dk))]
    const double p = Q(FP, 0, 0, 0), u = Q(FU, 0, 0, 0), v = Q(FV, 0, 0, 0),
                 w = Q(FW, 0, 0, 0), T = Q(FT, 0, 0, 0);

    /* first differences D */
    double dx[NF], dy[NF], dz[NF];
    for (int f = 0; f < NF; ++f) {
        dx[f] = (Q(f, 1, 0, 0) - Q(f, -1, 0, 0)) * (0.5 * nx);
        dy[f] = (Q(f, 0, 1, 0) - Q(f, 0, -1, 0)) * (0.5 * ny);
        dz[f] = (Q(f, 0, 0, 1) - Q(f, 0, 0, -1)) * (0.5 * nz);
    }
    /* Laplacian (L_x + L_y + L_z) q */
    double lap[NF];
    for (int f = 0; f < NF; ++f) {
        double c0 = Q(f, 0, 0, 0);
        double lx = ((Q(f, 1, 0, 0) + Q(f, -1, 0, 0)) - 2.0 * c0) * (nx * nx);
        double ly = ((Q(f, 0, 1, 0) + Q(f, 0, -1, 0)) - 2.0 * c0) * (ny * ny);
        double lz = ((Q(f, 0, 0, 1) + Q(f, 0, 0, -1)) - 2.0 * c0) * (nz * nz);
        lap[f] = lx + ly + lz;
    }
    /* fourth differences of p */
    double fxp = ((Q(FP, 2, 0, 0) + Q(FP, -2, 0, 0)) - 4.0 * (Q(FP, 1, 0, 0) + Q(FP, -1, 0, 0))) + 6.0 * p;
    double fyp = ((Q(FP, 0, 2, 0) + Q(FP, 0, -2, 0)) - 4.0 * (Q(FP, 0, 1, 0) + Q(FP, 0, -1, 0))) + 6.0 * p;
    double fzp = ((Q(FP, 0, 0, 2) + Q(FP, 0, 0, -2)) - 4.0 * (Q(FP, 0, 0, 1) + Q(FP, 0, 0, -1))) + 6.0 * p;
#undef Q

    /* artificial compressibility and characteristic speeds */
    double V2 = u * u + v * v + w * w;
    double beta2 = V2 > C->beta2_floor ? V2 : C->beta2_floor;
    double lam_x = 0.5 * (fabs(u) + sqrt(u * u + 4.0 * beta2));
    double lam_y = 0.5 * (fabs(v) + sqrt(v * v + 4.0 * beta2));
    double lam_z = 0.5 * (fabs(w) + sqrt(w * w + 4.0 * beta2));

    /* local pseudo-time step */
    double dt_conv = 1.0 / (lam_x * nx + lam_y * ny + lam_z * nz);
    double dmax = C->nu > C->alpha ? C->nu : C->alpha;
    double dt_visc = 1.0 / (2.0 * dmax * (nx * nx + ny * ny + nz * nz));
    *dt = P->cfl * (dt_conv < dt_visc ? dt_conv : dt_visc);

    /* Eq. 1 (times beta^2) */
    R[FP] = -beta2 * C->rho * (dx[FU] + dy[FV] + dz[FW])
            - P->eps4 * (lam_x * fxp * nx + lam_y * fyp * ny + lam_z * fzp * nz);
    /* Eq. 2, j = x, y, z */
    R[FU] = -(u * dx[FU] + v * dy[FU] + w * dz[FU]) - dx[FP] / C->rho + C->nu * lap[FU];
    R[FV] = -(u * dx[FV] + v * dy[FV] + w * dz[FV]) - dy[FP] / C->rho + C->nu * lap[FV];
    R[FW] = -(u * dx[FW] + v * dy[FW] + w * dz[FW]) - dz[FP] / C->rho + C->nu * lap[FW]
            + (T - P->t_inf);
    /* Eq. 3 */
    R[FT] = -(u * dx[FT] + v * dy[FT] + w * dz[FT]) + C->alpha * lap[FT];
}

/* R: 5 * ni*nj*nk values, field-major, interior cells (i fastest).
 * dt: ni*nj*nk values or NULL.  q must already hold its wall ghosts. */
void orc_residual(const orc_problem* P, const double* q, double* R, double* dt)
{
    orc_consts C = consts_of(P);
    size_t n = (size_t)P->ni * P->nj * P->nk;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nk; ++k)
        for (int j = 0; j < P->nj; ++j)
            for (int i = 0; i < P->ni; ++i) {
                double r[NF], d;
                cell_residual(P, &C, q, i, j, k, r, &d);
                size_t c = (size_t)i + (size_t)P->ni * ((size_t)j + (size_t)P->nj * k);
                for (int f = 0; f < NF; ++f) R[f * n + c] = r[f];
                if (dt) dt[c] = d;
            }
}

/* ------------------------------------------------------------------ */
/* Halo pack/unpack (Sec. 4.5, Listings 1-2; Optimized V3 adds j and k
 * faces).  Subdomain s = a + Pi*(b + Pj*c) owns interior cells
 * [a*ni/Pi, (a+1)*ni/Pi) along i, likewise along j, k (Sec. 3.2).  For each
 * s, each face -x,+x,-y,+y,-z,+z that is a cut (not a cavity wall), each
 * field p,u,v,w,T with width w > 0: the box of the w interior layers of s
 * next to that face, over the interior tangential extent of s, is one
 * segment, stored in (k, j, i) order, i fastest (Reading of Listing 1's
 * order, taken 0-based).  Reading: the receiver's ghost box beyond that face
 * covers the same cells, so with every subdomain in one array the unpack
 * writes each value back where the pack read it. */
typedef void (*seg_fn)(const orc_problem* P, int f, int i, int j, int k, size_t pos, void* ctx);

static size_t walk_segments(const orc_problem* P, const orc_halo* H, seg_fn fn, void* ctx)
{
    const int Pi = H->split[0], Pj = H->split[1], Pk = H->split[2];
    const int ex = P->ni / Pi, ey = P->nj / Pj, ez = P->nk / Pk;
    size_t pos = 0;
    for (int c = 0; c < Pk; ++c)
        for (int b = 0; b < Pj; ++b)
            for (int a = 0; a < Pi; ++a)
                for (int face = 0; face < 6; ++face) {
                    int axis = face / 2, high = face % 2;
                    int coord = axis == 0 ? a : axis == 1 ? b : c;
                    int parts = axis == 0 ? Pi : axis == 1 ? Pj : Pk;
                    if ((!high && coord == 0) || (high && coord == parts - 1)) continue;  /* wall */
                    for (int f = 0; f < NF; ++f) {
                        int wdt = H->width[f];
                        if (wdt == 0) continue;
                        int lo[3] = {a * ex, b * ey, c * ez};
                        int hi[3] = {(a + 1) * ex, (b + 1) * ey, (c + 1) * ez};
                        if (high) lo[axis] = hi[axis] - wdt;
                        else      hi[axis] = lo[axis] + wdt;
                        for (int k = lo[2]; k < hi[2]; ++k)
                            for (int j = lo[1]; j < hi[1]; ++j)
                                for (int i = lo[0]; i < hi[0]; ++i) {
                                    if (fn) fn(P, f, i, j, k, pos, ctx);
                                    ++pos;
                                }
                    }
                }
    return pos;
}

size_t orc_halo_elems(const orc_problem* P, const orc_halo* H)
{
    return walk_segments(P, H, NULL, NULL);
}

typedef struct { double* q; double* buf; } pk_ctx;

static void do_pack(const orc_problem* P, int f, int i, int j, int k, size_t pos, void* ctx)
{
    pk_ctx* c = (pk_ctx*)ctx;
    c->buf[pos] = c->q[at(P, f, i, j, k)];
}

static void do_unpack(const orc_problem* P, int f, int i, int j, int k, size_t pos, void* ctx)
{
    pk_ctx* c = (pk_ctx*)ctx;
    c->q[at(P, f, i, j, k)] = c->buf[pos];
}

void orc_halo_pack(const orc_problem* P, const orc_halo* H, const double* q, double* buf)
{
    pk_ctx c = {(double*)q, buf};
    walk_segments(P, H, do_pack, &c);
}

void orc_halo_unpack(const orc_problem* P, const orc_halo* H, const double* buf, double* q)
{
    pk_ctx c = {q, (double*)buf};
    walk_segments(P, H, do_unpack, &c);
}

/* ------------------------------------------------------------------ */
/* Mean Nusselt number of the hot wall x = 0 (Reading: the paper's cavity
 * transfers heat between its vertical walls, Sec. 2; the nondimensional
 * wall heat flux is -dT/dx, and the temperature scale is t_hot - t_cold).
 * dT/dx at the wall from the second-order one-sided difference through the
 * wall value T_w and the first two cell centres (x = h/2, 3h/2):
 *   dT/dx = (9 T_0 - T_1 - 8 T_w) / (3 h)
 * Nu = mean over (j, k) of -dT/dx / (t_hot - t_cold).  FP64 sums over k
 * planes in order. */
double orc_nusselt_hot(const orc_problem* P, const double* q)
{
    const double h = 1.0 / (double)P->ni;
    double total = 0.0;
    for (int k = 0; k < P->nk; ++k) {
        double plane = 0.0;
        for (int j = 0; j < P->nj; ++j) {
            const double tw = P->t_hot_field ? P->t_hot_field[j + (size_t)P->nj * k] : P->t_hot;
            const double t0 = q[at(P, FT, 0, j, k)], t1 = q[at(P, FT, 1, j, k)];
            const double dtdx = (9.0 * t0 - t1 - 8.0 * tw) / (3.0 * h);
            plane += -dtdx;
        }
        total += plane;
    }
    return total / ((double)P->nj * (double)P->nk) / (P->t_hot - P->t_cold);
}

/* ------------------------------------------------------------------ */
/* Pseudo-time stepping (Sec. 2; Sec. 3.1: a loop over all nodes inside the
 * pseudo-time loop).  Per step: wall ghosts, optional halo round trip,
 * residual + Euler update of every interior cell into q_tmp (Jacobi),
 * rescale of p at the centre cell (Sec. 2; Reading: cell (ni/2, nj/2, nk/2),
 * reference value 0), residual norms of the step (Reading: RMS of R over
 * the interior, Sec. 4.2), swap.  The newest state ends in q. */
void orc_step(const orc_problem* P, const orc_halo* H, double* q, double* q_tmp,
              double* buf, int nsteps, double* norms)
{
    orc_consts C = consts_of(P);
    double* cur = q;
    double* nxt = q_tmp;
    double* ksum = (double*)calloc((size_t)P->nk * NF, sizeof(double));
    const size_t ncell = (size_t)P->ni * P->nj * P->nk;
    for (int s = 0; s < nsteps; ++s) {
        orc_apply_bc(P, cur);
        if (H) {
            orc_halo_pack(P, H, cur, buf);
            orc_halo_unpack(P, H, buf, cur);
        }
#pragma omp parallel for schedule(static)
        for (int k = 0; k < P->nk; ++k) {
            double acc[NF] = {0.0, 0.0, 0.0, 0.0, 0.0};
            for (int j = 0; j < P->nj; ++j)
                for (int i = 0; i < P->ni; ++i) {
                    double r[NF], dt;
                    cell_residual(P, &C, cur, i, j, k, r, &dt);
                    for (int f = 0; f < NF; ++f) {
                        size_t x = at(P, f, i, j, k);
                        nxt[x] = cur[x] + dt * r[f];
                        acc[f] += r[f] * r[f];
                    }
                }
            for (int f = 0; f < NF; ++f) ksum[(size_t)k * NF + f] = acc[f];
        }
        double pc = nxt[at(P, FP, P->ni / 2, P->nj / 2, P->nk / 2)];
#pragma omp parallel for schedule(static)
        for (int k = 0; k < P->nk; ++k)
            for (int j = 0; j < P->nj; ++j)
                for (int i = 0; i < P->ni; ++i)
                    nxt[at(P, FP, i, j, k)] -= pc;
        if (norms) {
            for (int f = 0; f < NF; ++f) {
                double t = 0.0;
                for (int k = 0; k < P->nk; ++k) t += ksum[(size_t)k * NF + f];
                norms[f] = sqrt(t / (double)ncell);
            }
        }
        double* t = cur; cur = nxt; nxt = t;
    }
    if (cur != q) memcpy(q, cur, orc_state_elems(P) * sizeof(double));
    free(ksum);
}
