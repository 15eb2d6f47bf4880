/*
 * lbm_oracle.h -- plain FP64 CPU oracle of the LBM-RANS hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no header, table, helper or constant with
 * the HIP library: the two are written independently from the paper
 * (Ponsin & Lozano, "Lattice Boltzmann wall boundary conditions for
 * RANS-based simulations with wall functions", arXiv 2506.03905).
 *
 * Everything is double precision, loops are plain and unfused, streaming uses
 * two buffers (pull), populations are stored as f_i (not deviations).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* geometry presets */
#define ORC_CHANNEL 0 /* periodic x (and z); walls at y = 0 and y = ny (halfway links) */
#define ORC_PLATE 1   /* D2Q9 only: Zou-He inlet x=0, copy outlet x=nx-1, symmetric top,
                         bottom symmetric for x < plate_start and wall downstream */

/* wall schemes */
#define ORC_BB_FIXED 0 /* halfway bounce-back, prescribed wall velocity (eq. 31) */
#define ORC_BB_SLIP 1  /* slip-velocity bounce-back (eq. 31 with eq. 35) */
#define ORC_HRFD 2     /* hybrid regularized reconstruction (eq. 19, 23, 26-28) */
#define ORC_CAI_DEGRIGNY 3 /* regularized reconstruction with the gradient of eq. 29 (eq. 30) */

/* bounce-back link rule (ORC_BB_FIXED / ORC_BB_SLIP) */
#define ORC_IBB_HALFWAY 0 /* halfway: the wall midway between nodes (eq. 31) */
#define ORC_IBB_BOUZIDI 1 /* Bouzidi's interpolated rule, wall at wall_dist from B (eq. 36) */
#define ORC_IBB_YU 2      /* Yu's interpolated rule through the wall point (eq. 37) */

/* collision operators */
#define ORC_BGK 0 /* BGK with Guo forcing */
#define ORC_CM 1  /* central-moment operator of eq. 7 */

/* wall laws */
#define ORC_REICHARDT 0 /* Reichardt's law, log-law intercept B */
#define ORC_SA_LAW 1    /* SA-consistent analytic law, eq. 15-16 */

typedef struct orc_params {
    int32_t q;           /* 9 (D2Q9) or 19 (D3Q19) */
    int32_t nx, ny, nz;  /* nz = 1 for D2Q9 */
    int32_t flow;        /* ORC_CHANNEL / ORC_PLATE */
    int32_t scheme;      /* ORC_BB_FIXED / ORC_BB_SLIP / ORC_HRFD / ORC_CAI_DEGRIGNY */
    int32_t law;         /* ORC_REICHARDT / ORC_SA_LAW */
    int32_t sa_on;       /* 1: couple Spalart-Allmaras; 0: laminar, nu_t = 0 */
    int32_t plate_start; /* first wall cell of the plate (ORC_PLATE) */
    int32_t collision;   /* ORC_BGK / ORC_CM */
    double nu;           /* molecular kinematic viscosity, lattice units */
    double rho0;         /* reference density */
    double force[3];     /* body force density F */
    double u_inlet;      /* plate inlet velocity (x) */
    double wall_u_bottom[3]; /* ORC_BB_FIXED wall velocities */
    double wall_u_top[3];
    double nut_init_ratio; /* initial nu_tilde / nu */
    double kappa, B;     /* wall law constants (kappa also the SA kappa) */
    double beta;         /* HRFD blending parameter, eq. 27 */
    double cb1, cb2, sigma, cw2, cw3, cv1, rlim; /* SA constants, eq. 10-14 */
    int32_t bb_interp;   /* ORC_IBB_* (bounce-back schemes) */
    int32_t pad_;
    double wall_dist;    /* distance from the first node B to the wall (1/2: halfway) */
} orc_params;

typedef struct orc orc;

/* --- threads (OpenMP over lattice rows; results do not depend on them) --- */
void orc_set_threads(int n); /* n > 0: use n threads */
int orc_get_threads(void);

/* --- whole-lattice oracle ------------------------------------------------ */
orc *orc_create(const orc_params *p, const double *u0 /* D*ncell SoA, or NULL = zero */);
void orc_destroy(orc *o);
void orc_step(orc *o, int64_t n);
int64_t orc_ncell(const orc *o);
int64_t orc_nwall(const orc *o);
int64_t orc_steps(const orc *o);
void orc_get_u(const orc *o, double *out);      /* D*ncell: u^n (last step) */
void orc_get_rho(const orc *o, double *out);    /* ncell: sum_i f*_i        */
void orc_get_nt(const orc *o, double *out);     /* ncell: nu_tilde entering next step */
void orc_get_nut(const orc *o, double *out);    /* ncell: nu_t = nu_tilde f_v1 */
void orc_get_f(const orc *o, double *out);      /* q*ncell: post-collision f* */
void orc_get_wall(const orc *o, double *utau, double *uw /* 3*nwall */,
                  double *tdir /* 3*nwall */, int64_t *cell /* nwall */);
void orc_totals(const orc *o, double *out4);    /* sum rho, sum rho*u (3) */

/* --- per-cell building blocks (the lattice oracle calls exactly these) --- */
int orc_lattice(int q, int *c /* q*3 */, double *w /* q */, int *opp /* q */);
void orc_feq(int q, double rho, const double *u, double *feq);
void orc_collide(int q, const double *f, double tau, const double *force,
                 double *fpost, double *rho_out, double *u_out);
void orc_collide_cm(int q, const double *f, double tau, const double *force,
                    double *fpost, double *rho_out, double *u_out);
double orc_uplus(int law, double yp, double kappa, double B);
double orc_duplus(int law, double yp, double kappa, double B);
double orc_solve_utau(int law, double ut, double y, double nu, double kappa, double B);
double orc_sa_rhs(const orc_params *p, int D, double nt0, const double *ntm,
                  const double *ntp, const double *u0, const double *um /* 3x3 [axis][comp] */,
                  const double *up, double d);
double orc_nut(const orc_params *p, double nt);
void orc_zou_he_west(double *f /* 9, unknowns overwritten */, double U);
void orc_regularized(int q, double rho, const double *u, const double *S /* 3x3 */,
                     double tau, double *f);
void orc_hrfd_cell(const orc_params *p, double *f, int side, const double *t, double utau,
                   double uF_t, double uFF_t, double dudx, double ntB);
double orc_cai_degrigny_grad(int law, double utau, double nu, double yB, double delta,
                             double kappa, double B);

#ifdef __cplusplus
}
#endif
#endif
