/*
 * cavity_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference ("oracle") of the cavity hot path of
 * Xue & Roy, arXiv:2006.02602.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product library never does.
 * It shares no code, header or constant with the GPU library.
 *
 * Layout: q holds 5 fields p,u,v,w,T (Listing 2's variable order), each
 * (nk+4)*(nj+4)*(ni+4) doubles with 2 ghost layers per side (as in the
 * arrays of Sec. 4.5, Listing 1), i fastest (Sec. 3.1).
 */
#ifndef CAVITY_ORACLE_H_
#define CAVITY_ORACLE_H_
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int ni, nj, nk;                 /* interior cells along x, y, z        */
    double Ra, Pr;                  /* Rayleigh and Prandtl numbers        */
    double cfl;                     /* pseudo-time CFL number              */
    double eps4;                    /* 4th-difference dissipation coeff.   */
    double kappa, u_ref;            /* beta^2 floor = kappa * u_ref^2      */
    double t_hot, t_cold, t_inf;    /* wall and reference temperatures     */
    const double* t_hot_field;      /* NULL, or nj*nk hot-wall T, j fastest */
} orc_problem;

typedef struct {
    int split[3];                   /* (Pi, Pj, Pk)                        */
    int width[5];                   /* ghost width per field p,u,v,w,T     */
} orc_halo;

size_t orc_state_elems(const orc_problem* P);
void   orc_init(const orc_problem* P, uint64_t seed, double amp, double* q);
void   orc_apply_bc(const orc_problem* P, double* q);
void   orc_residual(const orc_problem* P, const double* q, double* R, double* dt);
size_t orc_halo_elems(const orc_problem* P, const orc_halo* H);
void   orc_halo_pack(const orc_problem* P, const orc_halo* H, const double* q, double* buf);
void   orc_halo_unpack(const orc_problem* P, const orc_halo* H, const double* buf, double* q);
void   orc_step(const orc_problem* P, const orc_halo* H, double* q, double* q_tmp,
                double* buf, int nsteps, double* norms);
double orc_nusselt_hot(const orc_problem* P, const double* q);
uint64_t orc_splitmix64(uint64_t seed, uint64_t n);
int    orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
