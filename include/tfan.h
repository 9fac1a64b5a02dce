/*
 * tfan.h -- C ABI of the MI355X (gfx950) solver for the two-fluid
 * active-nematic mixture of arXiv 2511.00445 ("Phase separation dynamics and
 * active turbulence in a binary fluid mixture").
 *
 * One coupled time step (Numerical Simulation section) advances, on a 2D
 * periodic nx x ny lattice:
 *   - two D2Q9 BGK lattice-Boltzmann fluids with Guo forcing: the active
 *     fluid (velocity u_a, the paper's u1, Model Eq. 4) and the passive fluid
 *     (u_p, the paper's u2, Model Eq. 5), coupled by the drag
 *     F_drag = gamma c1 c2 (u_p - u_a);
 *   - the active fluid feels the Beris-Edwards elastic stress (Model, elastic
 *     stress display), the active stress -zeta c1 Q (Model, active force) and
 *     the share c1 of the capillary force -phi grad(mu) (Model, capillary force);
 *     the passive fluid feels the share c2 of the capillary force;
 *   - n_sub forward-Euler finite-difference sub-steps (h = 1/n_sub) of the
 *     Cahn-Hilliard equation for phi (Model, Eqs. 1-3) and of the Beris-Edwards
 *     equation for Q (Model, Eqs. 11-12), with u_a and u_c = c1 u_a + c2 u_p
 *     frozen at their start-of-step values.
 * Lattice units (dx = dt = 1).  phi in [-1, 1] is the composition order
 * parameter; c1 = (1 + phi)/2 and c2 = (1 - phi)/2 are the active and passive
 * fractions.  Q is symmetric and traceless, stored as (Qxx, Qxy).
 *
 * Arrays: every field is row-major [ny][nx] with x fastest; vector fields are
 * two such planes, x component first ([2][ny][nx]).  Host arrays are float64.
 *
 * Ownership: the caller owns every host array and the device workspace
 * (device memory of tfan_workspace_bytes() bytes, 256-byte aligned).  The
 * library never allocates device memory and never frees caller memory; it owns
 * only the opaque handle, released by tfan_destroy().  A handle is bound to one
 * HIP stream and one device; it is not thread-safe.
 *
 * Errors: every int-returning function returns TFAN_OK (0) or a negative
 * tfan_status; tfan_last_error() gives the message.  Launch errors are reported
 * by the launching call; errors during kernel execution surface at the next
 * synchronising call (get_fields, diagnostics, get_state, sync).
 */
#ifndef TFAN_H
#define TFAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tfan_status {
  TFAN_OK = 0,
  TFAN_EINVAL = -1,     /* bad parameter, size or NULL pointer                 */
  TFAN_ENOMEM = -2,     /* workspace or host buffer too small                  */
  TFAN_EHIP = -3,       /* HIP runtime or launch error (message kept)           */
  TFAN_ENONFINITE = -4, /* diagnostics found NaN/Inf in the state               */
  TFAN_EUNSTABLE = -5   /* diagnostics found max |u| above 0.3 (Mach guard)     */
} tfan_status;

/* Population storage format.  The populations are stored as the deviations
 * f_i - w_i rho0 from rest; TFAN_STORAGE_F16 keeps them as IEEE binary16
 * (round to nearest even) and does all arithmetic in float32, halving the
 * population bytes per step.  phi and Q are float32 in both formats. */
enum { TFAN_STORAGE_F32 = 0, TFAN_STORAGE_F16 = 1 };

/* Problem statement (Model and Numerical Simulation sections).  Limits:
 * 8 <= nx, ny <= 32768, nx*ny <= 2^28, tau > 1/2, 1 <= n_sub <= 8, all reals
 * finite, rho0 > 0, M >= 0, K >= 0, Gamma >= 0, gamma >= 0, kappa >= 0. */
typedef struct tfan_params {
  int32_t nx, ny;      /* periodic grid                                          */
  int32_t n_sub;       /* finite-difference sub-steps per lattice-Boltzmann step */
  int32_t storage;     /* TFAN_STORAGE_F32 or TFAN_STORAGE_F16                   */
  double rho0;         /* density of each fluid (rho_1 = rho_2)                  */
  double tau_a, tau_p; /* BGK relaxation times; viscosity (tau - 1/2)/3          */
  double gamma;        /* inter-fluid drag coefficient                           */
  double A_ch, kappa;  /* mu = A_ch (phi^3 - phi) - kappa lap(phi)               */
  double M;            /* Cahn-Hilliard mobility                                 */
  double A0, gamma_ldg; /* Landau-de Gennes bulk energy (Model Eq. 8) in the (A0,
                        * gamma) form (A0/2)(1 - gamma/3) TrQ^2 - (A0 gamma/3) TrQ^3
                        * + (A0 gamma/4)(TrQ^2)^2; the library uses A = A0 (1 - gamma/3)
                        * and C = 2 A0 gamma of (A/2) TrQ^2 + (C/4) TrQ^4.  gamma = 3 is
                        * the two-dimensional isotropic-nematic point (A = 0).          */
  double K;            /* Frank elastic constant                                 */
  double lam;          /* tumbling parameter lambda                              */
  double Gamma;        /* rotational diffusion constant                          */
  double zeta;         /* activity, > 0 extensile                                */
} tfan_params;

/* Diagnostics: sums over all sites, accumulated in float64 on the device from
 * the float32 state (Results section observables). */
typedef struct tfan_diag {
  int64_t step;        /* coupled steps taken since init_fields / set_state      */
  int64_t nonfinite;   /* NaN/Inf count over phi, Q and both population sets     */
  double phi_sum;      /* sum phi                                                */
  double phi_sq_sum;   /* sum phi^2 (std. deviation Delta of phi)                */
  double mass_a;       /* sum rho_a                                              */
  double mass_p;       /* sum rho_p                                              */
  double ke_a;         /* 1/2 sum rho_a |u_a|^2                                   */
  double ke_p;         /* 1/2 sum rho_p |u_p|^2                                   */
  double ke_c;         /* 1/2 sum |u_c|^2  (u_c = c1 u_a + c2 u_p)                */
  double ua_sq;        /* sum |u_a|^2                                            */
  double uc_sq;        /* sum |u_c|^2                                            */
  double enstrophy_a;  /* sum omega_a^2, omega = d_x u_y - d_y u_x                */
  double enstrophy_c;  /* sum omega_c^2                                          */
  double elastic;      /* sum (K/2) |grad Q|^2, |grad Q|^2 = sum_kij (d_k Q_ij)^2 */
  double s_mean;       /* mean of S over sites, S = sqrt(Qxx^2 + Qxy^2) (Q = 2S(pp - I/2)) */
  double umax;         /* max over sites of max(|u_a|, |u_p|)                    */
  double phi_absmax;   /* max over sites of |phi|                                */
} tfan_diag;

typedef struct tfan_sim tfan_sim;

/* Host-only validation of a parameter block; no GPU call. */
int tfan_check_params(const tfan_params* p);

/* Device workspace needed for p (0 if p is invalid); no GPU call. */
size_t tfan_workspace_bytes(const tfan_params* p);

/* Bind a solver to the caller's device workspace (on the current HIP device)
 * and stream (hipStream_t, NULL = default stream).  *out receives the handle.
 * TFAN_EINVAL for bad parameters, TFAN_ENOMEM if bytes is too small. */
int tfan_create(const tfan_params* p, void* dev_workspace, size_t bytes,
                void* hip_stream, tfan_sim** out);

/* Set the state at step 0 (Numerical Simulation: the initial composition,
 * director field and fluid velocities): phi, qxx, qxy [ny][nx]; u_a, u_p
 * [2][ny][nx] or NULL for zero.  Both population sets start at the D2Q9
 * equilibrium f^eq(rho0, u) of the BGK collision.  Non-finite inputs:
 * TFAN_EINVAL.  Synchronises the stream. */
int tfan_init_fields(tfan_sim* s, const double* phi, const double* qxx,
                     const double* qxy, const double* u_a, const double* u_p);

/* Enqueue n >= 0 coupled steps on the handle's stream; returns without
 * waiting.  One step (Numerical Simulation) is: pull streaming of both D2Q9
 * populations; moments; chemical potential mu (Model, Eq. 2 for the order
 * parameter phi); molecular field H (Eq. 7 with the bulk energy of Eq. 8);
 * elastic stress (Model, elastic stress display), active stress -zeta c1 Q and
 * capillary force -phi grad(mu) (Eq. 10), their forces on each fluid; the
 * half-force (Guo) velocities with the drag F_drag = gamma c1 c2 (u_p - u_a)
 * solved implicitly per site; BGK collision with the Guo source for both
 * fluids; then n_sub forward-Euler sub-steps of Eq. 1 (Cahn-Hilliard, advected
 * by u_c) and Eqs. 11-12 (Beris-Edwards, advected and rotated by u_a) with the
 * velocities frozen.  Gradients are second-order central differences and
 * Laplacians 5-point stencils, all periodic.  n < 0: TFAN_EINVAL; a failed
 * launch: TFAN_EHIP; execution errors surface at the next synchronising call. */
int tfan_step(tfan_sim* s, int64_t n);

/* Copy the current fields to host float64 arrays (any may be NULL):
 * phi, qxx, qxy, rho_a, rho_p [ny][nx]; u_a, u_p [2][ny][nx].  The velocities
 * are the half-force-corrected ones of the step's own velocity solve (Guo
 * forcing, Numerical Simulation: rho u = sum_i f_i c_i + F/2).
 * Synchronises the stream. */
int tfan_get_fields(tfan_sim* s, double* phi, double* qxx, double* qxy,
                    double* u_a, double* u_p, double* rho_a, double* rho_p);

/* Fill *out with the Results-section observables summed over the grid
 * (composition and its variance, kinetic energies, enstrophies of u_a and of
 * the mixture velocity, Frank elastic energy, mean order S) in float64.
 * Returns TFAN_OK, or TFAN_ENONFINITE / TFAN_EUNSTABLE (with *out still
 * filled) when the state is broken.  Synchronises the stream. */
int tfan_diagnostics(tfan_sim* s, tfan_diag* out);

/* Checkpoint: the raw device state (step counter int64, populations in their
 * storage format, phi, Q as float32).
 * tfan_state_bytes() gives the size; set_state restores it bit for bit. */
size_t tfan_state_bytes(const tfan_sim* s);
int tfan_get_state(tfan_sim* s, void* host, size_t bytes);
int tfan_set_state(tfan_sim* s, const void* host, size_t bytes);

/* Device-side state exchange (for the convolutional surrogate, tfan_cnn.h).
 * Layout [planes][ny][nx] float32, planes = 7: phi, Qxx, Qxy, u_a (x, y),
 * u_p (x, y); planes = 9: the same, then rho_a - rho0, rho_p - rho0.
 * tfan_exchange_bytes(s, planes) = planes nx ny 4 bytes (0 for other plane counts).
 * tfan_export_state writes the current state into dev_out; the velocities are
 * the ones tfan_get_fields returns (the step's own half-force velocity solve).
 * tfan_import_state sets phi and Q from dev_in and rebuilds both population sets
 * at equilibrium so that the next step's velocities (the half-force solve with
 * the implicit drag, under the forces of the imported phi and Q) are those of
 * dev_in, with the densities of dev_in (planes = 9) or, with planes = 7, the
 * densities of the populations the handle holds at the call (rho0 on a handle
 * that has had no tfan_init_fields, tfan_set_state or import yet).  Exporting
 * right after an import gives back dev_in up to float32 rounding; what is lost
 * is the populations' non-equilibrium part.  It sets the step counter to `step`
 * (>= 0).
 * The arrays are caller-owned device memory on the handle's GPU: a pointer the
 * HIP runtime does not know as a device allocation of that GPU gives
 * TFAN_EINVAL, and so does a plane count other than 7 or 9; fewer than
 * tfan_exchange_bytes(s, planes) bytes (the `bytes` argument, or what is left of
 * the allocation from the pointer on) give TFAN_ENOMEM.  Both are enqueued on the
 * solver's stream as kernels (no runtime copies) and do not synchronise; the
 * arrays must stay valid until the stream reaches them. */
size_t tfan_exchange_bytes(const tfan_sim* s, int32_t planes);
int tfan_export_state(tfan_sim* s, float* dev_out, size_t bytes, int32_t planes);
int tfan_import_state(tfan_sim* s, const float* dev_in, size_t bytes, int32_t planes, int64_t step);

/* Wait for the handle's stream; reports execution errors. */
int tfan_sync(tfan_sim* s);

/* Steps taken so far. */
int64_t tfan_step_count(const tfan_sim* s);

/* Kernel timing with HIP events on the handle's stream.  enable(cap) starts
 * recording up to cap launches (cap = 0 stops and frees the events);
 * tfan_kernel_times() synchronises, then fills ms_total[k] and launches[k] for
 * the first n kernel ids (k < tfan_kernel_count()).  Recording stops silently
 * once cap launches were recorded. */
int tfan_kernel_timing(tfan_sim* s, int64_t cap);
int tfan_kernel_times(tfan_sim* s, double* ms_total, int64_t* launches, int n);
int tfan_kernel_count(void);
const char* tfan_kernel_name(int id);

/* Launch shape of the hot kernels.  collide_rows: 1 or 2 rows of sites per
 * thread of the collision kernel on tiles of the default width (256 sites for
 * float32 storage, 128 for binary16); 11 or 12: the same on tiles of half that
 * width.  fd_shape selects the finite-difference launches: 1, 2, 4: one launch
 * per sub-step with that many rows per thread; 16, 32: all n_sub sub-steps of a
 * step in one launch on 64 x fd_shape tiles (temporal blocking; for n_sub > 5 the
 * 4-row per-sub-step launch runs); 162, 163: blocks of 2 or 3 sub-steps per
 * launch on 64 x 16 tiles; 165, 166: blocks of up to 5 sub-steps per launch on
 * 64 x 40 (165) or 64 x 32 (166) tiles, the phi (Cahn-Hilliard) and Q
 * (Beris-Edwards) sub-steps in separate thread blocks.  Default (1, 165) below
 * 2^21 sites, (2, 165) from there (a batch: (2, 165)).  Results are bitwise
 * identical for every shape; only the speed differs.  Other values: TFAN_EINVAL. */
int tfan_set_tuning(tfan_sim* s, int32_t collide_rows, int32_t fd_shape);
int tfan_get_tuning(const tfan_sim* s, int32_t* collide_rows, int32_t* fd_shape);

/* Autotuner: runs `steps` steps (after one warm-up step) with every launch
 * shape above (4 collision x 9 sub-step shapes, minus blocked shapes that
 * n_sub turns into the per-sub-step launch), keeps the fastest, restores the
 * state it started from (checkpoint through host memory) and reports the best
 * time per step (may be NULL). */
int tfan_autotune(tfan_sim* s, int32_t steps, double* best_ms_per_step);

/* Release the handle (never the workspace). NULL is ignored. */
void tfan_destroy(tfan_sim* s);

/* Message of the last failure on s; s = NULL gives the last failure of a call
 * without a valid handle (check_params, create). */
const char* tfan_last_error(const tfan_sim* s);

/* ------------------------------------------------------------------------
 * Batches of independent simulations (parameter sweeps).  Each member has its
 * own grid and parameters; all members share n_sub and the storage format.
 * tfan_batch_step advances every member by one collision launch and one launch
 * per sub-step over the tiles of all members, so small grids fill the GPU
 * together.  p points to `count` parameter blocks; the workspace holds every
 * member's state plus a small device table.  Member indices are 0..count-1.
 * Results of a member are bitwise identical to a single simulation with the
 * same parameters and launch shape.
 * ---------------------------------------------------------------------- */
typedef struct tfan_batch tfan_batch;

size_t tfan_batch_workspace_bytes(const tfan_params* p, int32_t count);   /* 0 if invalid */
int tfan_batch_create(const tfan_params* p, int32_t count, void* dev_workspace, size_t bytes,
                      void* hip_stream, tfan_batch** out);
int tfan_batch_count(const tfan_batch* b);
int tfan_batch_init_fields(tfan_batch* b, int32_t member, const double* phi, const double* qxx,
                           const double* qxy, const double* u_a, const double* u_p);
int tfan_batch_step(tfan_batch* b, int64_t n);                           /* async */
int tfan_batch_get_fields(tfan_batch* b, int32_t member, double* phi, double* qxx, double* qxy,
                          double* u_a, double* u_p, double* rho_a, double* rho_p);
int tfan_batch_diagnostics(tfan_batch* b, int32_t member, tfan_diag* out);
/* The same n >= 0 steps as tfan_batch_step in ONE persistent launch for all
 * members and all steps: a cooperative kernel whose blocks (1024 threads, as
 * many as are resident at once) take the collision tiles of every member, meet
 * at a grid-wide barrier, take the phi and Q sub-step tiles of every member (all
 * n_sub sub-steps of the step), meet again, and go on to the next step.  Requires
 * n_sub <= 5 (else TFAN_EINVAL); results are bitwise those of tfan_batch_step;
 * the launch shape set by tfan_batch_set_tuning does not apply.  Async; a launch
 * the device cannot run cooperatively gives TFAN_EHIP. */
int tfan_batch_step_persistent(tfan_batch* b, int64_t n);
/* Blocks of the last persistent launch (0 before the first). */
int tfan_batch_persistent_blocks(const tfan_batch* b);
int tfan_batch_set_tuning(tfan_batch* b, int32_t collide_rows, int32_t fd_shape);
int tfan_batch_get_tuning(const tfan_batch* b, int32_t* collide_rows, int32_t* fd_shape);
int tfan_batch_autotune(tfan_batch* b, int32_t steps, double* best_ms_per_step);
int tfan_batch_sync(tfan_batch* b);
void tfan_batch_destroy(tfan_batch* b);
const char* tfan_batch_last_error(const tfan_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* TFAN_H */
