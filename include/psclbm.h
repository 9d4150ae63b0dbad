/*
 * psclbm.h -- C ABI of the MI355X (gfx950) partially-saturated-cell lattice
 * Boltzmann library.
 *
 * The library implements the per-time-step hot path of the hybrid IBM-LBM-DEM
 * method of Liu & Wu, "A hybrid LBM-DEM framework with an improved immersed
 * moving boundary method for modelling complex particle-liquid flows involving
 * adhesive particles" (arXiv 1901.09745):
 *   - psc_rasterize: per-particle solid fractions by the linear approximation
 *     (Sec. 2.4, Eqs. 15-19, Table 1), binned into per-tile particle lists;
 *   - lbm_step: the fused collide-stream of the modified PSC lattice Boltzmann
 *     equation (Sec. 2.1-2.3, Eqs. 1-6, 10, 12-13) with the per-particle
 *     hydrodynamic force and torque of Eq. 14 and a global FP64 mass sum;
 *   - dem_step: the adhesive DEM step with the JKR normal force and
 *     Newton-Euler motion (Sec. 2.5, Eqs. 21, 25-27), optionally with the
 *     sliding, twisting and rolling friction of Eqs. 22, 28, 29, or with
 *     Hertz's contact without adhesion;
 *   - coupled_step: rasterise, step and DEM for many steps, fused;
 *   - adjoints: lbm_step_adjoint (with lbm_recompute and
 *     psc_rasterize_adjoint) for the lattice step, and dem_step_adjoint for a
 *     frictionless DEM step, which chain into gradients through coupled runs
 *     with moving particles.
 *
 * Conventions shared by every call:
 *   - All array arguments named d_* are DEVICE pointers; h_* are host pointers.
 *     The caller owns all memory; the library never allocates device memory.
 *     Lattice state, tile lists, particle snapshots, force accumulators and DEM
 *     contact state live in one caller-provided device workspace of
 *     psclbm_workspace_bytes() bytes.
 *   - All work is enqueued asynchronously on the HIP stream given to lbm_init
 *     (or psclbm_set_stream); one context per stream; calls on one context are
 *     not thread-safe.
 *   - Every call returns PSCLBM_OK (0) or a negative error code.  Argument
 *     errors are reported synchronously and leave the state untouched.
 *     Conditions detected on the device (slot or list overflow, contact
 *     overflow, invalid particle radius, non-finite mass) raise a sticky flag
 *     reported by the next psclbm_sync() or lbm_mass() call.
 *   - The canonical distribution layout is f[i][z][y][x] in FP64 (x fastest),
 *     with the velocity order
 *       D2Q9 : 0 (0,0) 1 (1,0) 2 (0,1) 3 (-1,0) 4 (0,-1) 5 (1,1) 6 (-1,1)
 *              7 (-1,-1) 8 (1,-1);
 *       D3Q19: 0 rest, 1/2 = +-x, 3/4 = +-y, 5/6 = +-z, then (1,1,0),(-1,-1,0),
 *              (1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1),
 *              (0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1).
 *     Cell (x, y, z) has its centre at the integer point (x, y, z).
 *   - Particle arrays are FP64 structure-of-arrays: x[3n], u[3n], omega[3n]
 *     (z components 0 in 2D; only omega_z is used in 2D) and radius[n].
 */
#ifndef PSCLBM_H
#define PSCLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define PSCLBM_OK 0
#define PSCLBM_EINVAL (-1)     /* invalid argument or configuration */
#define PSCLBM_ENOMEM (-2)     /* workspace smaller than required */
#define PSCLBM_EHIP (-3)       /* a HIP runtime call or launch failed */
#define PSCLBM_ESLOTS (-4)     /* a cell or tile list exceeded its capacity */
#define PSCLBM_ECONTACTS (-5)  /* a particle exceeded max_contacts, or a DEM bin overflowed */
#define PSCLBM_ENONFINITE (-6) /* the lattice mass is not finite */
#define PSCLBM_ESTATE (-7)     /* call out of order (e.g. lbm_step before psc_rasterize) */

/* ---- face boundary kinds (faces: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+) ------ */
#define PSCLBM_PERIODIC 0      /* both faces of the axis must be periodic */
#define PSCLBM_BOUNCE_BACK 1   /* resting wall at -1/2 or L-1/2, halfway bounce-back (Eq. 6) */
#define PSCLBM_MOVING_WALL 2   /* bounce-back with the wall-momentum term
                                  -2 w_i rho (e_i . u_w) / c_s^2, u_w = face_velocity */
#define PSCLBM_INLET_EQ 3      /* boundary layer reset to f^eq(rho0, face_velocity) before
                                  every collision */
#define PSCLBM_OUTLET_EQ 4     /* boundary layer reset to f^eq(rho0, u of the adjacent interior
                                  cell) before every collision */

/* ---- precision forms --------------------------------------------------- */
#define PSCLBM_FP64 0          /* FP64 storage of f, FP64 arithmetic */
#define PSCLBM_FP32 1          /* FP32 storage of g_i = f_i - w_i rho0, FP32 arithmetic */
#define PSCLBM_FP32_FP16STORE 2 /* FP16 storage of (f_i - w_i rho0) / w_i, FP32 arithmetic */

/* Solid weighting of the partially saturated cells (Sec. 2.3). */
#define PSCLBM_WEIGHT_MODIFIED 0
#define PSCLBM_WEIGHT_ORIGINAL 1
/* In every form the particle force/torque accumulation, the mass sum and the
 * DEM are FP64. */

typedef struct {
  int lattice;                /* 9 (D2Q9, requires nz == 1) or 19 (D3Q19) */
  int nx, ny, nz;             /* lattice size, >= 1 each */
  double tau;                 /* BGK relaxation time, > 1/2 (Eq. 2) */
  double body_force[3];       /* constant fluid body-force density F (Eqs. 4-5) */
  int face_bc[6];             /* PSCLBM_PERIODIC ... PSCLBM_OUTLET_EQ per face */
  double face_velocity[6][3]; /* wall / inlet velocity per face */
  double rho0;                /* reference density: initial state, inlet and outlet density */
  double shell_h;             /* half-width h of the solid-fraction shell (Sec. 2.4), >= 0 */
  int precision;              /* PSCLBM_FP64, PSCLBM_FP32 or PSCLBM_FP32_FP16STORE */
  int max_particles;          /* capacity of the particle snapshot, >= 0 */
  double max_radius;          /* largest particle radius the DEM bins are sized for */
  int max_tile_particles;     /* capacity of each tile's particle list (e.g. 256) */
  int max_contacts;           /* DEM contact capacity per particle (e.g. 16) */
  int weighting;              /* PSCLBM_WEIGHT_MODIFIED (Eqs. 12-14, cell total clamped, Table 1) or
                                 PSCLBM_WEIGHT_ORIGINAL (Eqs. 7-9, 11: each particle's
                                 weight from its own fraction, B_n their sum) */
} psclbm_config;

typedef struct {
  int n;                      /* number of particles, 0 <= n <= max_particles */
  const double* x;            /* d_x[3n]: centre positions */
  const double* u;            /* d_u[3n]: translational velocities U_s */
  const double* omega;        /* d_omega[3n]: angular velocities Omega_s */
  const double* radius;       /* d_radius[n]: radii, r^2 > 1/4 (2D) or > 1/2 (3D) */
} psclbm_particles;

typedef struct {
  double rho_p, rho_f;        /* particle and fluid density */
  double E_p, poisson;        /* Young modulus and Poisson ratio (Eq. 25) */
  double gamma;               /* surface energy (Eq. 27); work of adhesion 2 gamma */
  double eta_n;               /* normal damping coefficient (Eq. 26) */
  double g[3];                /* gravity; G = (rho_p - rho_f) V g */
  double dt;                  /* coupling step (one LBM step) */
  int n_sub;                  /* DEM sub-cycles per coupling step (lambda), >= 1 */
  int kinematic;              /* nonzero: prescribed motion, x += dt u only */
  double k_t;                 /* tangential stiffness k_T (Eq. 28), > 0 when mu_f > 0 */
  double eta_t;               /* tangential dissipation coefficient eta_T (Eq. 28), >= 0 */
  double mu_f;                /* friction coefficient (Eq. 29), >= 0; 0: no sliding or
                                 twisting friction (zero-initialised callers get none) */
  double theta_r;             /* critical rolling angle theta_crit (Eq. 29), >= 0; 0: no
                                 rolling resistance */
} psclbm_dem_params;

typedef struct psclbm_ctx psclbm_ctx;

/* Bytes of device workspace that lbm_init needs for cfg (0 if cfg is invalid).
 * Host-only. */
size_t psclbm_workspace_bytes(const psclbm_config* cfg);

/* Create a context on d_workspace (device memory of at least
 * psclbm_workspace_bytes(cfg) bytes, 256-byte aligned, owned by the caller
 * and kept alive until lbm_free) and initialise f = f^eq(rho0, 0) (Eq. 3).
 * hip_stream is a hipStream_t (NULL: the null stream).  *out receives the
 * context (a small host allocation).  Errors: EINVAL (tau <= 1/2, lattice /
 * nz mismatch, unpaired periodic faces, open face on an axis shorter than 3
 * cells, negative capacities, one direction's array of 4 GiB or more),
 * ENOMEM (workspace too small), EHIP. */
int lbm_init(const psclbm_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
             psclbm_ctx** out);

/* Release the host-side context (the workspace stays the caller's). */
void lbm_free(psclbm_ctx* ctx);

/* Change the stream used by later calls. */
int psclbm_set_stream(psclbm_ctx* ctx, void* hip_stream);

/* Load / store the state in the canonical FP64 layout (Q*N doubles, device),
 * whatever the storage precision and streaming parity.  lbm_set_f converts to
 * the storage form (rounding in the FP32 / FP16 forms). */
int lbm_set_f(psclbm_ctx* ctx, const double* d_f);
int lbm_get_f(psclbm_ctx* ctx, double* d_f);

/* f = f^eq(rho, u) per cell (Eq. 3); d_rho[N] or NULL (rho0), d_u[3N] or NULL
 * (rest). */
int lbm_set_equilibrium(psclbm_ctx* ctx, const double* d_rho, const double* d_u);

/* Density and velocity of the current state (Eq. 5, with the half-force
 * shift): d_rho[N], d_u[3N] (either may be NULL). */
int lbm_get_macros(psclbm_ctx* ctx, double* d_rho, double* d_u);

/* Snapshot the particle state and bin every particle into the lattice tiles
 * its shell box X +- (r + h) touches (the candidate cells of Table 1).  The following
 * lbm_step calls use this snapshot for positions, velocities and radii; the
 * solid fractions eps_{n,s} (Eqs. 15-19, Table 1) are evaluated per
 * cell inside lbm_step.  Errors: EINVAL (n out of range, NULL arrays), EHIP;
 * sticky ESLOTS if a tile list overflows, sticky EINVAL for a radius outside
 * the domain of Eqs. 17/19. */
int psc_rasterize(psclbm_ctx* ctx, const psclbm_particles* p);

/* Materialise the rasterised solid fractions for inspection: d_eps_total[N]
 * = min(sum_s eps_{n,s}, 1) (the clamped total of Table 1); optionally the first kslots
 * recorded particles per cell in ascending id, d_slot_id[N*kslots] (-1 when
 * empty) and d_slot_eps[N*kslots] (either may be NULL). */
int psc_get_solid_fraction(psclbm_ctx* ctx, double* d_eps_total, int* d_slot_id,
                           double* d_slot_eps, int kslots);

/* Advance the lattice nsteps >= 1 time steps: per step, per cell, the moments
 * (Eq. 5), the modified PSC collision (Eqs. 3-4, 10, 12-13) with the solid
 * fractions of the rasterised particles, the hydrodynamic force and torque of
 * Eq. 14 on every particle, and in-place streaming with periodic, bounce-back
 * (Eq. 6), moving-wall and inlet/outlet boundaries.  Errors: ESTATE if
 * particles were never rasterised (use psc_rasterize with n = 0 for pure
 * fluid), EINVAL, EHIP; sticky ESLOTS if a cell is covered by more particles
 * than the kernel's slot capacity (4). */
int lbm_step(psclbm_ctx* ctx, int nsteps);

/* Copy the FP64 hydrodynamic force and torque (Eq. 14) of the most recent
 * lbm_step to d_force[3n] and d_torque[3n] (n of the snapshot; either pointer
 * may be NULL).  The torque is about the particle centre; in 2D only its z
 * component is nonzero. */
int particle_forces(psclbm_ctx* ctx, double* d_force, double* d_torque);

/* One DEM coupling step (Eq. 21) for n particles, updating d_x, d_u, d_omega
 * in place: n_sub semi-implicit Euler sub-steps of dt/n_sub with the
 * hydrodynamic force d_force[3n] and torque d_torque[3n] held fixed (Sec. 2.5),
 * gravity (rho_p - rho_f) V g, and JKR normal contacts (Eqs. 25-27, with the
 * jump-on / pull-off hysteresis) between particles and with the walls of
 * non-periodic axes (flat walls at -1/2 and L-1/2).  With mu_f > 0 every
 * contact also carries sliding and twisting friction (Eqs. 22, 28, 29), each a
 * linear spring-dashpot-slider: the tangential force k_T xi + eta_T v_t capped
 * at mu_f |F_ne + 2 F_C| (F_ne the JKR elastic force), its torque r_i n x F
 * about the centre, and the twisting moment (a^2/2)(k_T theta + eta_T Omega_t)
 * capped at 3 pi a F_crit / 16 (a the JKR contact radius); v_t is the slip of
 * the partner's surface point relative to the particle's, xi and theta the
 * slip and twist integrated since the contact began, reset to the capped
 * value while capped.  With theta_r > 0 (and gamma > 0) the rolling
 * displacement xr, the integral of R (omega_i - omega_j) x n with R the
 * effective radius, meets the moment 4 F_C (a/a0)^{3/2} (xr x n), xr clamped
 * at |xr| = theta_r R.  Walls are at rest, and a 2D disk moves in its plane
 * and spins about z.  gamma == 0 gives Hertz's contact without adhesion,
 * F = (4/3) E sqrt(R) delta^{3/2}.  Positions wrap into [0, L) on periodic
 * axes.  2D: disks of unit depth.  Contact history (ids, and with friction each contact's
 * springs; a step without friction leaves every spring unloaded) lives in the
 * workspace (dem_reset_contacts clears it).  d_force and d_torque may
 * both be NULL: the force and torque of the most recent lbm_step are then
 * read from the workspace (n must equal the rasterised count; ESTATE
 * otherwise).  The contact forces of a particle are summed in neighbour-bin
 * order.  Errors: EINVAL (bad params, among them a negative or non-finite
 * k_t, eta_t, mu_f or theta_r, or k_t == 0 with mu_f > 0; n > max_particles, only one
 * of the two force pointers NULL, a contact reach delta_C of 1 or more), EHIP;
 * sticky ECONTACTS on contact or bin overflow. */
int dem_step(psclbm_ctx* ctx, const psclbm_dem_params* prm, double* d_x, double* d_u,
             double* d_omega, const double* d_radius, int n, const double* d_force,
             const double* d_torque);

/* nsteps coupled time steps in the order of Sec. 2.5: each step rasterises
 * the particles at their current state (psc_rasterize), takes one lbm_step
 * and advances the particles by one dem_step driven by that step's force and
 * torque, in place in d_x, d_u, d_omega (n particles, d_radius[n]).  The
 * result is that of those three calls in turn, up to the order of the FP64
 * sums of contact forces.  With n_sub == 1 the work of consecutive steps is
 * fused: the DEM wave of a particle, having integrated it, writes its
 * snapshot and enters it in the tile lists and DEM bins of the next step, so
 * a step is two kernels (plus one at the start of the call).  Without
 * friction and with adhesion the contacts are gathered by workgroups of the
 * step kernel; with friction (mu_f > 0 or theta_r > 0) or the Hertz contact
 * (gamma == 0) by the DEM kernel, which also records the spins the next
 * step's contacts read.  Afterwards the context holds the last step's
 * rasterisation and force / torque accumulators, as after the three calls.
 * Errors: those of psc_rasterize, lbm_step and dem_step (EINVAL, EHIP;
 * sticky ESLOTS, ECONTACTS). */
int coupled_step(psclbm_ctx* ctx, const psclbm_dem_params* prm, double* d_x, double* d_u,
                 double* d_omega, const double* d_radius, int n, int nsteps);

/* Adjoint of the DEM step just taken (Sec. 2.5, Eq. 21 with Eqs. 25-27; the
 * most recent dem_step, or the last step of coupled_step, with no DEM call
 * since): given dJ/d(x', u', omega') of the step's result (d_gx, d_gu, d_gw,
 * [3n] each), writes dJ/d(x, u, omega) of its input (d_ax, d_au, d_aw) and
 * dJ/d(force, torque) of the hydrodynamic force and torque it was driven by
 * (d_aF, d_aT), all [3n], none aliasing an input.  d_x, d_u, d_omega,
 * d_radius: the particle state before the step (a copy the caller kept;
 * omega is not read).  The step's contact set is held fixed: the contact
 * lists the step formed are read, and the jump-on / pull-off switches
 * contribute nothing.  Frictionless steps with n_sub == 1 only (JKR or
 * Hertz, normal damping, gravity).  2D: the out-of-plane parts of
 * d_aF and the in-plane parts of d_aT are zero.  Errors: EINVAL (bad
 * params, friction, n_sub != 1, kinematic, n > max_particles, null
 * pointers), EHIP. */
int dem_step_adjoint(psclbm_ctx* ctx, const psclbm_dem_params* prm, const double* d_x,
                     const double* d_u, const double* d_omega, const double* d_radius, int n,
                     const double* d_gx, const double* d_gu, const double* d_gw, double* d_ax,
                     double* d_au, double* d_aw, double* d_aF, double* d_aT);

/* Forget all DEM contacts (no pair is bonded). */
int dem_reset_contacts(psclbm_ctx* ctx);

/* Copy the current DEM contact lists, those the most recent DEM step formed
 * (Sec. 2.5: the bonds of the jump-on / pull-off hysteresis), to caller
 * device buffers: d_count[max_particles] contacts per particle and
 * d_ids[max_particles * max_contacts] partner ids (particles, walls -1-face),
 * each particle's first d_count entries valid.  dem_set_contacts copies such
 * lists back as the current ones (friction springs are not saved: contacts
 * restored this way start unloaded).  Together they let a reverse pass put
 * back the contact set of the step it differentiates (dem_step_adjoint reads
 * the current lists).  Asynchronous on the context's stream.  Errors:
 * EINVAL (null pointers), EHIP. */
int dem_get_contacts(psclbm_ctx* ctx, int* d_count, int* d_ids);
int dem_set_contacts(psclbm_ctx* ctx, const int* d_count, const int* d_ids);

/* Synchronise the stream and return the total mass sum_n sum_i f_i of the
 * current state in FP64 (*h_mass), or the sticky error if one is set
 * (ENONFINITE if the mass is not finite). */
int lbm_mass(psclbm_ctx* ctx, double* h_mass);

/* Synchronise the stream; return and clear the sticky device error. */
int psclbm_sync(psclbm_ctx* ctx);

/* Static description of an error code. */
const char* psclbm_strerror(int code);

/* Number of completed lbm_step time steps since lbm_init / lbm_set_f /
 * lbm_set_equilibrium (the in-place streaming parity is its low bit). */
long long lbm_step_count(const psclbm_ctx* ctx);

/* ---- without allocation ------------------------------------------------- */

/* Bytes of the fixed device array psc_solid_fraction_noalloc works in. */
#define PSCLBM_NOALLOC_SCRATCH_BYTES 33554432

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * solid fractions that psc_rasterize followed by psc_get_solid_fraction give
 * (same kernels, same results), for the lattice cfg describes and the
 * particles p, with no context and no workspace.  Outputs as in
 * psc_get_solid_fraction: d_eps_total[N], and with kslots > 0 d_slot_id and
 * d_slot_eps [N*kslots] (both then required).  The tile lists and the
 * particle snapshot live in a fixed device array of
 * PSCLBM_NOALLOC_SCRATCH_BYTES bytes inside the library, one per GPU, held
 * until the process ends; the call uses the current device's copy, clears
 * what must start at zero, enqueues its kernels on hip_stream and then
 * synchronises that stream to read the device error word back (so it
 * returns once the outputs are written).  Calls that overlap on one GPU
 * (from several threads or streams) share the array and race.  Errors:
 * EINVAL (invalid cfg, n outside [0, max_particles], null pointers, or
 * tile lists and snapshot needing more than PSCLBM_NOALLOC_SCRATCH_BYTES:
 * 8 + 4 ntiles (2 + max_tile_particles) + 144 n bytes, about, with ntiles =
 * N / 256), EHIP, ESLOTS (a tile list or a cell overflowed), EINVAL for a
 * radius outside the domain of Eqs. 17/19.  Nothing is allocated. */
int psc_solid_fraction_noalloc(const psclbm_config* cfg, const psclbm_particles* p,
                               double* d_eps_total, int* d_slot_id, double* d_slot_eps,
                               int kslots, void* hip_stream);

/* ---- adjoint ------------------------------------------------------------ */

/* Adjoint of one lbm_step (FP64), for gradients of any function J of the
 * state and of the per-particle forces and torques: the transpose of the
 * step's Jacobian (Eqs. 1, 3-6, 10, 12-14, Table 1) applied to the given
 * sensitivities.
 *   d_f          canonical FP64 state f(t) entering the step (as lbm_get_f
 *                returned it before the step), Q*N doubles;
 *   d_lambda_in  dJ/df(t+1), canonical, Q*N doubles;
 *   d_lambda_out receives dJ/df(t) (through this step), canonical, Q*N
 *                doubles, must not alias d_lambda_in;
 *   d_dJ_dF, d_dJ_dT  dJ/dF_s and dJ/dT_s of the forces and torques this step
 *                produced (3n each, or NULL for zero);
 *   d_g_x, d_g_u, d_g_omega  += dJ/dX_s, dJ/dU_s, dJ/dOmega_s through this
 *                step (3n each, or NULL), X entering through the solid
 *                fractions (Table 1) and the rigid-body velocity and torque
 *                arms;
 *   d_g_face_velocity  += dJ/d(face velocity) [6][3] (inlet and moving-wall
 *                faces), or NULL.
 * The particles are those of the last psc_rasterize (their state at step t).
 * The derivative of the Table 1 clamps is taken as zero at their kinks.
 * Errors: EINVAL (also for the original weighting, which has no adjoint),
 * ESTATE (no rasterisation), EHIP. */
int lbm_step_adjoint(psclbm_ctx* ctx, const double* d_f, const double* d_lambda_in,
                     double* d_lambda_out, const double* d_dJ_dF, const double* d_dJ_dT,
                     double* d_g_x, double* d_g_u, double* d_g_omega,
                     double* d_g_face_velocity);

/* Recompute for checkpoint-and-recompute adjoints: from the canonical FP64
 * state d_f0 (Q*N doubles, caller-owned), runs nsteps lbm_step time steps
 * (Eqs. 1-6, 10, 12-13, Table 1) with the particles of the last psc_rasterize
 * and writes the state after step k (k = 1..nsteps) to d_ring + (k-1)*Q*N,
 * canonical FP64 (caller-owned, nsteps*Q*N doubles, must not overlap d_f0).
 * The arithmetic is FP64 for every precision form; each step reads one ring
 * slot and writes the next, so no state copy is made.  The context's own
 * state, step count, force / torque accumulators and mass are left as they
 * were.  Errors: EINVAL (null pointers, nsteps < 1, overlap, N*8 bytes not
 * below 4 GiB), ESTATE (no rasterisation), EHIP. */
int lbm_recompute(psclbm_ctx* ctx, const double* d_f0, int nsteps, double* d_ring);

/* Adjoint of the solid fractions alone (Eqs. 15-18, Table 1): for
 * sensitivities dJ/deps_{n,s} given per recorded slot in the layout of
 * psc_get_solid_fraction (d_g_slot_eps[N*kslots], slots in ascending particle
 * id), adds dJ/dX_s = sum_n dJ/deps_{n,s} (x_n - X_s)/|x_n - X_s| over the
 * cells on the linear band of Table 1 to d_g_x[3n].  Errors: EINVAL, ESTATE,
 * EHIP. */
int psc_rasterize_adjoint(psclbm_ctx* ctx, const double* d_g_slot_eps, int kslots,
                          double* d_g_x);

#ifdef __cplusplus
}
#endif

#endif /* PSCLBM_H */
