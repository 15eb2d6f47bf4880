/*
 * lbm.h -- C ABI of the MI355X (gfx950) LBM-RANS hot-path library.
 *
 * The library advances a lattice Boltzmann solution on a uniform Cartesian
 * lattice (D2Q9 or D3Q19) with a local relaxation time from the molecular
 * plus Spalart-Allmaras eddy viscosity, and with the wall treatments compared
 * in Ponsin & Lozano, "Lattice Boltzmann wall boundary conditions for
 * RANS-based simulations with wall functions" (arXiv 2506.03905):
 * slip-velocity bounce-back (Sec. 3.2, eq. 31 and 35) and the hybrid
 * regularized reconstruction (Sec. 3.1, eq. 19, 23, 26-28), both driven by a
 * per-wall-cell wall-function solve for u_tau (Sec. 3.1, eq. 20-22).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Lattice units: dx = dt = 1, c_s^2 = 1/3.
 * - Cell (x, y, z) has linear index x + nx*(y + ny*z); x is fastest.  y is the
 *   wall-normal direction.  For D2Q9, nz must be 1.
 * - Population order (used by checkpoints and population exports): rest
 *   first, then opposite pairs (2k-1, 2k).  D2Q9: (0,0) (1,0) (-1,0) (0,1)
 *   (0,-1) (1,1) (-1,-1) (1,-1) (-1,1).  D3Q19: (0,0,0), the six faces
 *   +-x, +-y, +-z, then (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1)
 *   (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1).
 * - Wall cells are the boundary nodes B (Sec. 3.1, Fig. 1), in this order:
 *   the bottom row (y = 0) z-major with x fastest, then for the channel the
 *   top row (y = ny-1) in the same order.  For the plate only bottom cells with
 *   x >= plate_start are wall cells.  B sits y_B = 1/2 from the wall; the
 *   wall-function reference node F is the second node, y_F = 3/2.
 * - Device memory: the caller allocates ONE device buffer of
 *   lbm_footprint(...) bytes (for instance a torch uint8 tensor) and passes
 *   it to lbm_create.  The library never frees it; the caller keeps it alive
 *   until lbm_destroy.  The stepping path allocates no device memory of its
 *   own; host-side copies (lbm_set_velocity, lbm_moments, lbm_nu_tilde and
 *   lbm_populations with host pointers) stage through a temporary device
 *   allocation that is freed before they return.
 * - Streams: every launch goes to the stream given at creation.  Calls are
 *   asynchronous unless stated otherwise.
 * - Errors: every int-returning call returns LBM_OK (0) or a negative code;
 *   lbm_last_error() returns a thread-local message for the last failure.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_PARAMS_VERSION 2

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* bad dimensions, enum, tau_eff <= 1/2, buffer too small */
    LBM_ENOMEM = -2,    /* host allocation failed / pool full */
    LBM_EHIP = -3,      /* a HIP runtime call failed */
    LBM_EDIVERGED = -4, /* NaN/Inf or non-positive density seen by a reduction */
    LBM_ESTATE = -5     /* call out of order (e.g. destroyed handle) */
};

typedef enum { LBM_D2Q9 = 9, LBM_D3Q19 = 19 } lbm_lattice_t;

/* Storage precision of the populations.  LBM_F64 stores f_i - w_i rho0 in
 * double and computes in double; the others store f_i - w_i rho0 in the given
 * type and compute in float.  Velocity and nu_tilde are kept in the compute
 * type; wall-function state and reductions are always double. */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16 = 2, LBM_BF16 = 3 } lbm_precision_t;

/* Geometry presets.
 * LBM_FLOW_CHANNEL: periodic in x (and z); walls at y = 0 and y = ny, each
 *   halfway between the first/last cell row and a virtual solid row
 *   (Sec. 4.1.1).
 * LBM_FLOW_PLATE (D2Q9 only, Sec. 4.2.1): Zou-He velocity inlet at x = 0
 *   (u = (u_inlet, 0)), outlet at x = nx-1 whose unknown populations are
 *   copied from column nx-2, symmetry (specular) plane at the top, symmetry
 *   plane at the bottom for x < plate_start and the wall for x >= plate_start.
 *   A bottom link whose crossing point is on the plate, the leading-edge point
 *   included, is a wall link. */
typedef enum { LBM_FLOW_CHANNEL = 0, LBM_FLOW_PLATE = 1 } lbm_flow_t;

/* Wall schemes (Table 1).
 * LBM_WALL_FIXED_BB: halfway bounce-back with a prescribed wall velocity
 *   (eq. 31); zero velocity gives the no-slip wall used by laminar checks.
 * LBM_WALL_SLIP_BB: eq. 31 with the slip velocity of eq. 35 from the wall
 *   function, nu_t|B = nu kappa y_B+, Delta_w = y_B, u_B the lattice velocity of
 *   the previous step.
 * LBM_WALL_HRFD: regularized reconstruction of every population at B
 *   (eq. 19) with rho_B from eq. 23, u_B from the wall function, and the
 *   blended wall-normal gradient of eq. 27-28 (beta = 0.28 calibrated in
 *   Sec. 4.1.2.1; beta = 0 gives the finite-difference regularized BC).
 *   D2Q9 only.
 * LBM_WALL_CAI_DEGRIGNY: the same reconstruction with the wall-normal
 *   gradient taken as the third-order one-sided difference of the wall law
 *   (eq. 29) in place of eq. 27 (Sec. 3.1.2, eq. 30: beta = 1 with the law's
 *   derivative replaced); the beta argument is ignored.  D2Q9 only. */
typedef enum {
    LBM_WALL_FIXED_BB = 0,
    LBM_WALL_SLIP_BB = 1,
    LBM_WALL_HRFD = 2,
    LBM_WALL_CAI_DEGRIGNY = 3
} lbm_wall_scheme_t;

/* Link rule of LBM_WALL_FIXED_BB / LBM_WALL_SLIP_BB (Sec. 3.2).
 * LBM_IBB_HALFWAY: the wall midway between nodes, eq. 31.
 * LBM_IBB_BOUZIDI: Bouzidi's interpolated bounce-back, eq. 36, with the wall
 *   at wall_dist from the first node along every wall-crossing link.
 * LBM_IBB_YU: Yu's rule, eq. 37: the incoming population is interpolated
 *   linearly to the wall point, reflected there with eq. 31's moving-wall
 *   term, and interpolated back to the node through the second node F.
 * The HRFD and Cai-Degrigny schemes use halfway walls (wall_dist = 1/2). */
typedef enum { LBM_IBB_HALFWAY = 0, LBM_IBB_BOUZIDI = 1, LBM_IBB_YU = 2 } lbm_ibb_t;

/* Collision operators (Sec. 2.1).
 * LBM_COLL_BGK: single relaxation time omega = 1/tau_eff with the second-order
 *   equilibrium and Guo forcing weighted by (1 - omega/2).
 * LBM_COLL_CM: the central-moment operator of eq. 7: the deviatoric
 *   second-order central moments relax with omega, every other central moment
 *   goes to its Maxwellian (fourth-order Hermite) value, and the forcing enters
 *   through (I - Lambda/2) R.  For D2Q9 this is Lambda = diag[1,1,1,1,omega,
 *   omega,1,1,1]; D3Q19 applies the same rule to its 19 central moments. */
typedef enum { LBM_COLL_BGK = 0, LBM_COLL_CM = 1 } lbm_collision_t;

/* Output type and location of the field exports (lbm_moments). */
typedef enum { LBM_OUT_F64 = 0, LBM_OUT_F32 = 1 } lbm_out_dtype_t;
typedef enum { LBM_ON_HOST = 0, LBM_ON_DEVICE = 1 } lbm_loc_t;

/* Wall laws for the u_tau solve: Reichardt's law with log-law intercept B
 * (constant C = B - ln(kappa)/kappa), or the SA-consistent analytic law of
 * eq. 16 (derivative eq. 15). */
typedef enum { LBM_LAW_REICHARDT = 0, LBM_LAW_SA = 1 } lbm_wall_law_t;

typedef struct lbm_params {
    int32_t size;         /* sizeof(lbm_params_t), set by lbm_params_default */
    int32_t version;      /* LBM_PARAMS_VERSION */
    int32_t precision;    /* lbm_precision_t */
    int32_t flow;         /* lbm_flow_t */
    int32_t scheme;       /* lbm_wall_scheme_t, may be changed by lbm_set_wall_bc */
    int32_t law;          /* lbm_wall_law_t */
    int32_t sa_on;        /* 1: couple SA (nu_eff = nu + nu_t); 0: laminar */
    int32_t plate_start;  /* plate: first wall column */
    int32_t reduce_every; /* run the residual reduction every K steps (0: only on demand) */
    int32_t collision;    /* lbm_collision_t */
    double nu;            /* molecular viscosity (lattice units), > 0 */
    double rho0;          /* reference density (populations stored as f - w rho0) */
    double force[3];      /* body force density F (eq. 5) */
    double u_init[3];     /* uniform initial velocity */
    double u_inlet;       /* plate inlet velocity */
    double u_ref;         /* reference velocity for Cf = 2 (u_tau / u_ref)^2 */
    double wall_u_bottom[3]; /* LBM_WALL_FIXED_BB wall velocities */
    double wall_u_top[3];
    double nut_init_ratio;   /* initial nu_tilde / nu (3) */
    double kappa, B;         /* von Karman constant (also the SA kappa), log-law intercept */
    double beta;             /* HRFD blending parameter (eq. 27) */
    double cb1, cb2, sigma, cw2, cw3, cv1, rlim; /* SA constants (after eq. 14) */
    double store_shift_u; /* populations are stored as f - f_eq(rho0, (store_shift_u, 0, 0));
                             0 (default) stores f - w rho0 */
    int32_t bb_interp;    /* link rule of the bounce-back schemes: lbm_ibb_t */
    int32_t pad_;
    double wall_dist;     /* distance q of the first node from the wall, in (0, 1]:
                             1/2 (default) for halfway walls, any value with
                             LBM_IBB_BOUZIDI / LBM_IBB_YU; the wall function then
                             reads B at y_B = q and F at y_F = 1 + q (Sec. 3.1) */
} lbm_params_t;

/* Reduction result (all double).  mass = sum rho, momentum = sum rho u over all
 * cells at the last step; l2_du_rel = ||u^n - u^(n-K)||_2 / (K ||u^n||_2) with K
 * the steps since the previous reduction; mean_u_tau over wall cells and its
 * relative change since the previous reduction (the convergence measure of
 * Sec. 4.1.1; -1 when there is no previous reduction); nan_flag = 1 if any
 * density or velocity was NaN/Inf or a density <= 0. */
typedef struct lbm_residual {
    int64_t step;
    int64_t steps_since_previous;
    double mass;
    double momentum[3];
    double l2_du_rel;
    double mean_u_tau;
    double d_u_tau_rel;
    double nan_flag;
} lbm_residual_t;

/* Kernel timing collected while lbm_set_timing is on (milliseconds). */
typedef struct lbm_timing {
    int64_t step_launches;  /* launches of the fused stream-collide-SA kernel */
    double step_ms;         /* their summed duration */
    int64_t wall_launches;  /* launches of the wall-function kernel */
    double wall_ms;
} lbm_timing_t;

typedef struct lbm lbm_t;

/* Fills *p with defaults: F32, channel, BGK, slip bounce-back, Reichardt,
 * kappa = 0.41, B = 5.2, beta = 0.28, SA on with the constants listed after
 * eq. 14, nu_tilde = 3 nu, rho0 = 1, reduce_every = 100. */
void lbm_params_default(lbm_params_t *p);

/* Device bytes needed by lbm_create for this lattice; < 0 on invalid input. */
int64_t lbm_footprint(lbm_lattice_t lattice, int nx, int ny, int nz, const lbm_params_t *p);

/* Creates a lattice in the caller's device buffer dev_buf (>= footprint
 * bytes, 256-byte aligned) on device-stream `stream` (a hipStream_t; NULL is
 * the null stream) and initializes it.  The problem is the paper's: a
 * uniform lattice (Sec. 2.1) for the periodic channel driven by a body force
 * (Sec. 4.1.1) or the zero-pressure-gradient plate (Sec. 4.2.1) at a given
 * viscosity (relaxation time from eq. 8 with nu + nu_t, eq. 10), wall scheme
 * and wall law.  Initial state: populations at equilibrium
 * f = f_eq(rho0, u_init), nu_tilde = nut_init_ratio * nu, then one
 * wall-function pass (Sec. 3.1, eq. 20-22) that sets u_tau, the wall velocity
 * and the Dirichlet nu_tilde of the wall cells.
 * Ownership: dev_buf stays the caller's; *out is a host handle released by
 * lbm_destroy.  Returns LBM_EINVAL for nx < 1, ny < 4, nz != 1 with D2Q9, a
 * plate with D3Q19 or nx < 4, HRFD with D3Q19, nu <= 0, or a buffer that is
 * too small; LBM_EHIP if a launch fails. */
int lbm_create(lbm_lattice_t lattice, int nx, int ny, int nz, const lbm_params_t *p, void *dev_buf,
               int64_t buf_bytes, void *stream, lbm_t **out);

/* Re-initializes populations to f_eq(rho0, u(x)) from a caller velocity field
 * (D components, SoA: u[a*ncell + cell]) in double, on host (on_device = 0)
 * or device (1); the stored velocity becomes u, nu_tilde is reset, the step
 * counter is reset to 0 and the wall function runs once. */
int lbm_set_velocity(lbm_t *h, const double *u, int on_device);

/* Selects the wall scheme (before the first step or between steps). */
int lbm_set_wall_bc(lbm_t *h, lbm_wall_scheme_t scheme, double beta);

/* Advances n >= 0 time steps, asynchronously on the handle's stream.  One
 * step is the paper's time step: streaming (eq. 3) with the wall links
 * (eq. 31 with the slip velocity of eq. 35, or the interpolated rules of
 * eq. 36-37) or the regularized reconstruction at the wall cells (eq. 19,
 * 23, 26-30), moments (eq. 4-5), collision with tau from nu + nu_t (eq. 7-8,
 * 10; BGK or the central-moment operator), the Spalart-Allmaras update
 * (eq. 11-14) and the wall function (Sec. 3.1, eq. 20-22).  Every
 * reduce_every steps an FP64 reduction (mass, momentum, residual, mean u_tau,
 * non-finite count) runs on the device, carried by the step itself on the
 * channel's even steps; a sticky divergence flag is copied to pinned host
 * memory without blocking and read by later lbm_step calls.  Returns
 * LBM_EDIVERGED (and takes no further step) once a completed reduction has
 * seen a NaN/Inf or a density <= 0; since the host runs ahead of the device,
 * a divergence inside one call is normally reported by the next call (or at
 * once by lbm_residual, which synchronizes).  LBM_EINVAL for n < 0. */
int lbm_step(lbm_t *h, int64_t n);

/* Copies the macroscopic fields of the last step into caller buffers (NULL
 * skips a field): the density rho = sum_i f_i (eq. 4, ncell values), the
 * velocity u of eq. 5 with the half-force shift (D*ncell values, SoA:
 * u[a*ncell + cell]) and the eddy viscosity nu_t = nu_tilde f_v1 (eq. 10,
 * ncell values).  dtype: LBM_OUT_F64 (double) or LBM_OUT_F32 (float; exact
 * for the FP32/FP16/BF16 storage variants, whose fields are float).
 * where: LBM_ON_DEVICE (device buffers, asynchronous on the handle's stream,
 * nothing allocated) or LBM_ON_HOST (host buffers, synchronous; the data is
 * staged through a temporary device allocation freed before the call
 * returns).  LBM_EINVAL for an unknown dtype or location. */
int lbm_moments(lbm_t *h, void *rho, void *u, void *nu_t, int dtype, int where);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lbm_moments
 * with the same arguments and results, whose host path stages through a
 * library-owned static device array of LBM_NOALLOC_SCRATCH_BYTES (one per
 * GPU, held until the process ends) instead of a temporary allocation; it
 * calls no allocating routine.  Returns LBM_EINVAL, with a message, when the
 * requested fields need more staging than that (bytes = ncell * (4 or 8) *
 * (number of requested scalar fields, u counting D)).  All calls on one GPU
 * share that array: calls that overlap on one GPU (several threads, or calls
 * racing on different streams) race and must be serialized by the caller.
 * The device path (LBM_ON_DEVICE) uses no staging. */
#define LBM_NOALLOC_SCRATCH_BYTES (32LL << 20)
int lbm_moments_noalloc(lbm_t *h, void *rho, void *u, void *nu_t, int dtype, int where);

/* Copies the SA working variable nu_tilde (ncell, double). */
int lbm_nu_tilde(lbm_t *h, double *nt, int on_device);

/* Post-collision populations of the last step, f*_i(x) of eq. 1 before
 * streaming (not deviations), in the canonical order, [i*ncell + cell],
 * double.  Every direction of every cell is reported, including those that
 * stream out through an open boundary at the next step (their post-collision
 * value, like the rest).  Synchronous, host only. */
int lbm_populations(lbm_t *h, double *f_host);

/* Per wall cell (in the wall-cell order above), from the wall function of
 * the last step (Sec. 3.1, eq. 20-22): the friction velocity u_tau >= 0, the
 * skin-friction coefficient Cf = 2 (u_tau / u_ref)^2 (the bulk form of
 * Sec. 4.1.2.6; u_ref = U_b for the channel, U_inf for the plate), the
 * tangential direction t of the velocity at F (3 per cell) and the wall
 * velocity u_w of the bounce-back link rule (eq. 35 for the slip scheme;
 * 3 per cell).  Host buffers of n >= nwall entries (NULL skips a field);
 * synchronous.  LBM_EINVAL if n < nwall. */
int lbm_wall(lbm_t *h, double *u_tau, double *cf, double *t, double *u_w, int64_t n);

/* Number of cells / wall cells / steps taken. */
int64_t lbm_ncell(const lbm_t *h);
int64_t lbm_nwall(const lbm_t *h);
int64_t lbm_steps(const lbm_t *h);

/* Runs the reduction on the current state if none ran at this step, then
 * synchronizes the stream and fills *out.  Returns LBM_EDIVERGED if the
 * nan_flag is set. */
int lbm_residual(lbm_t *h, lbm_residual_t *out);

/* Per-kernel timing with HIP events on the handle's stream: on = 0 off, 1 every
 * launch, k > 1 only the launches of the two steps that start at a multiple
 * of k (both step parities, fewer events between kernels). */
int lbm_set_timing(lbm_t *h, int on);
int lbm_get_timing(lbm_t *h, lbm_timing_t *out); /* synchronizes */

/* Checkpoint: lbm_checkpoint_bytes() host bytes hold the whole state (device
 * buffer and step counter).  save/load synchronize.  load requires a handle
 * created with the same lattice, dimensions and parameters. */
int64_t lbm_checkpoint_bytes(const lbm_t *h);
int lbm_save(lbm_t *h, void *host, int64_t bytes);
int lbm_load(lbm_t *h, const void *host, int64_t bytes);

/* Releases the handle's host state and events; the device buffer stays the
 * caller's. */
int lbm_destroy(lbm_t *h);

/* ---------------------------------------------------------------------------
 * Serving pool: many independent solves resident in one device buffer.
 *
 * Requests are admitted by footprint (first fit in the pool buffer) and
 * advanced together in two groups that overlap on the device:
 *  - small D2Q9 lattices (<= 2048 cells, channels <= 4096) on the caller's
 *    stream: one persistent launch per kind (storage, collision, flow, wall
 *    treatment) in which each lattice is owned by one workgroup that loops
 *    over the steps;
 *  - every other lattice on a second stream: each phase of a step (fused
 *    update, wall function, residual) is one launch over all resident
 *    lattices of a kind, whatever their number.
 * Every lattice stops on the device on convergence (at a reduction step:
 * residual of lbm_residual_t below `tol`, or relative change of the mean
 * u_tau since the previous reduction below `tol_utau`, the criterion of
 * Sec. 4.1.1 taken over the reduction interval), divergence (a non-finite
 * value or rho <= 0 seen by a reduction) or `max_steps`.
 * Results of one lattice do not depend on what else is resident.  The device
 * buffer also holds the slot descriptors, slot lists and block tables (about
 * 1/2000 of its size); the pool allocates a few pinned host pages.
 * ------------------------------------------------------------------------- */
typedef struct lbm_pool lbm_pool_t;

enum { LBM_SLOT_IDLE = 0, LBM_SLOT_RUNNING = 1, LBM_SLOT_CONVERGED = 2, LBM_SLOT_CAPPED = 3, LBM_SLOT_DIVERGED = 4 };

typedef struct lbm_pool_status {
    int32_t status;     /* LBM_SLOT_* */
    int32_t batched;    /* 1: advanced by the persistent small-lattice launch */
    int64_t steps;      /* steps taken */
    double residual;    /* last residual ||u^n - u^(n-K)|| / (K ||u^n||) */
    double mean_u_tau;  /* mean u_tau over the wall cells at the last residual */
    int64_t footprint;  /* bytes of the pool buffer held by the slot */
    double d_u_tau_rel; /* |mean u_tau - its previous value| / previous value over the
                           last reduction interval; -1 before the second reduction */
    int32_t converged_by; /* LBM_SLOT_CONVERGED: 1 residual < tol, 2 d_u_tau_rel < tol_utau */
    int32_t pad_;
} lbm_pool_status_t;

/* dev_buf: caller-owned device memory (256-byte aligned) of `bytes`; the first
 * max_slots descriptors live at its start.  `stream` carries the small-lattice
 * launches; the pool creates one more (default-priority) stream. */
int lbm_pool_create(void *dev_buf, int64_t bytes, int max_slots, void *stream, lbm_pool_t **out);

/* Largest contiguous free block (bytes). */
int64_t lbm_pool_free_bytes(const lbm_pool_t *pool);

/* Admits one solve: the lattice is created in the pool buffer and initialized
 * (optionally from a host velocity field, as lbm_set_velocity).  tol and
 * tol_utau are the two convergence thresholds (0 switches one off).  Returns
 * LBM_ENOMEM (nothing changed) if no slot or no block of lbm_footprint()
 * bytes is free.  *slot receives the slot index. */
int lbm_pool_admit(lbm_pool_t *pool, lbm_lattice_t lattice, int nx, int ny, int nz, const lbm_params_t *p,
                   const double *u0_host, double tol, double tol_utau, int64_t max_steps, int *slot);

/* Advances every running slot by up to `steps` steps and synchronizes. */
int lbm_pool_step(lbm_pool_t *pool, int64_t steps);

/* Continuous batching without blocking: for each group whose previous chunk
 * has finished, refreshes its slots' status and launches the next chunk of
 * `steps` steps for its running slots (slots admitted since are included);
 * returns at once.  *in_flight (may be NULL) receives the number of groups
 * (0-2) with a chunk on the device. */
int lbm_pool_pump(lbm_pool_t *pool, int64_t steps, int *in_flight);

/* Status of one slot (host data refreshed by lbm_pool_step / lbm_pool_pump). */
int lbm_pool_poll(lbm_pool_t *pool, int slot, lbm_pool_status_t *out);

/* The slot's lattice handle, for lbm_moments / lbm_wall / lbm_populations
 * (valid until lbm_pool_release); NULL for a bad slot. */
lbm_t *lbm_pool_lattice(lbm_pool_t *pool, int slot);

/* Frees the slot and its memory; if its group has a chunk on the device the
 * memory is returned when that chunk is harvested (the slot is gone at once). */
int lbm_pool_release(lbm_pool_t *pool, int slot);

/* Releases every slot and the pool's host state and stream; the buffer stays
 * the caller's. */
int lbm_pool_destroy(lbm_pool_t *pool);

/* Thread-local message describing the last error (empty if none). */
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
