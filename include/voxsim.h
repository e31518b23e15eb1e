/*
 * voxsim: explicit time step of a heterogeneous soft-body voxel lattice on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Hiller & Lipson, "Dynamic Simulation of Soft Heterogeneous
 * Objects" (arXiv 1212.2845).  Each voxel of a cubic lattice is a mass with
 * three translational and three rotational degrees of freedom; every
 * face-adjacent pair of filled voxels is joined by an Euler-Bernoulli beam
 * whose stiffness is the composite of the two materials.  One step computes
 * every bond force from the current state, adds bond and ground damping,
 * gravity, the floor with Coulomb friction, voxel-voxel contact and thermal
 * actuation, and then updates all voxels at once.
 *
 * Conventions for every call:
 *   - Return value is a status: VX_OK or one of the negative codes below.
 *     No C++ exception crosses this interface.  vx_last_error(h) returns a
 *     message for the last failing call on that handle.
 *   - Host arrays passed in are borrowed for the duration of the call and
 *     copied; the caller keeps ownership.
 *   - Device memory: the library allocates none.  The caller allocates one
 *     workspace of vx_workspace_bytes() bytes (e.g. a torch uint8 tensor on
 *     the GPU), binds it with vx_bind_workspace(), and keeps it alive until
 *     vx_destroy().  The library never frees it.
 *   - All GPU work is enqueued on the stream given to vx_create (a
 *     hipStream_t; NULL is the null stream).  The host blocks only in the
 *     read calls and in the status check at the end of vx_step.
 *   - A handle is used by one host thread at a time.
 *   - Lattice arrays are dense over nx*ny*nz cells, cell index
 *     x + nx*(y + ny*z); material index 0 is "empty".
 *   - Units are SI (m, kg, s, Pa, K, N).  Gravity acts along -z; the floor
 *     is the plane z = 0.
 */
#ifndef VOXSIM_H
#define VOXSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define VX_OK 0
#define VX_EINVAL (-1)     /* bad argument; nothing was changed */
#define VX_EDEVICE (-2)    /* a HIP call failed */
#define VX_EUNSTABLE (-3)  /* a non-finite value appeared in the state (the
                              paper's TimeStep returning false) */
#define VX_EOVERFLOW (-4)  /* a voxel had more collision candidates than
                              contact_cap */
#define VX_ESTATE (-5)     /* call out of order (e.g. step before bind) */
#define VX_ENOMEM (-6)     /* host memory exhausted; the call had no effect
                              that later calls depend on */

/* One palette entry.  Index 0 of every palette is the empty material and
 * its fields are ignored.  The paper's AddMat takes E and the Poisson
 * ratio and defaults the rest (appendix, CVX_Object::AddMat). */
typedef struct vx_material {
    double E;     /* elastic modulus, Pa, > 0 */
    double nu;    /* Poisson ratio, in (-1, 0.5) */
    double rho;   /* density, kg/m^3, > 0 */
    double cte;   /* coefficient of thermal expansion, 1/K */
    double mu_s;  /* static friction coefficient against the floor, >= 0 */
    double mu_d;  /* dynamic friction coefficient against the floor, >= 0 */
} vx_material;

/* Simulation parameters: the paper's setters (SetSlowDampZ,
 * SetCollisionDampZ, SetBondDampZ, appendix) folded into one struct. */
typedef struct vx_params {
    double voxel_size;      /* lattice dimension l, m, > 0 */
    double gravity;         /* m/s^2 along -z, >= 0 */
    double zeta_bond;       /* damping ratio between bonded voxels, [0, 1) */
    double zeta_slow;       /* damping ratio of each voxel to ground, >= 0 */
    double zeta_col;        /* damping ratio of floor / voxel contact, >= 0 */
    double temp_amp;        /* temperature signal amplitude, K */
    double temp_freq;       /* temperature signal frequency, Hz */
    double temp_phase;      /* temperature signal phase, rad */
    double dt_scale;        /* multiplies the stable timestep, (0, 1]; 0 -> 1 */
    double origin[3];       /* world position of the lower corner of cell 0 */
    int32_t floor_on;       /* 1: floor at z = 0 with friction */
    int32_t self_collision_on; /* 1: voxel-voxel contact between surface voxels */
    int32_t contact_cap;    /* max collision candidates per surface voxel (0 -> 32, at most 1024) */
    int32_t reserved;       /* must be 0 */
} vx_params;

typedef struct vx_sim *vx_handle;

/* Create a simulation from a material grid (the paper's InitializeMatter /
 * AddMat / SetMat / Import, appendix).  precision is 32 or 64: the type the
 * state is stored and stepped in.  Computes all per-bond constants (Eq. 1-12),
 * the stable timestep (Eq. 31-32) and the surface voxel list on the host.
 * Errors: VX_EINVAL for a bad size, material index >= n_mat, E <= 0,
 * rho <= 0, nu outside (-1, 0.5), l <= 0, precision not 32/64, contact_cap
 * above 1024, or self-collision on a lattice more than 2^20 cells long on an
 * axis.  On
 * success *out is a new handle (free with vx_destroy). */
int vx_create(const uint8_t *grid, int32_t nx, int32_t ny, int32_t nz,
              const vx_material *palette, int32_t n_mat, const vx_params *params,
              int32_t precision, void *stream, vx_handle *out);

/* Bytes of device workspace this simulation needs (state ping-pong,
 * per-voxel flags and materials, bond scratch, collision lists). */
int vx_workspace_bytes(vx_handle h, uint64_t *bytes);

/* Bind a device buffer of at least vx_workspace_bytes bytes, aligned to
 * 256 bytes, and upload the initial state.  The buffer stays owned by the
 * caller.  Errors: VX_EINVAL if too small or misaligned, VX_EDEVICE on a
 * failed copy. */
int vx_bind_workspace(vx_handle h, void *device_ptr, uint64_t bytes);

/* Per-cell fixed mask (nonzero = immobile, the paper's AddFixedRegion). */
int vx_set_fixed(vx_handle h, const uint8_t *mask);

/* Constant external force per cell, dense ncell x 3 (N); zero rows mean
 * "not forced" (the paper's AddForcedRegion). */
int vx_set_forces(vx_handle h, const double *force);

/* Region helpers with the paper's fractional workspace coordinates
 * (AddFixedRegion / AddForcedRegion, appendix): loc and size in [0,1] per
 * axis.  A voxel "touches" the region when its cube overlaps the box with
 * positive volume.  The forced region's total force is split equally among
 * the voxels it touches; it replaces earlier forces on those voxels. */
int vx_fixed_region(vx_handle h, const double loc[3], const double size[3]);
int vx_forced_region(vx_handle h, const double loc[3], const double size[3],
                     const double force[3]);

/* Per-cell temperature signal amplitude (K) and phase (rad); either may be
 * NULL, meaning the global value of vx_params.  The voxel's temperature is
 * amp * sin(2 pi temp_freq t + phase) (Volumetric Actuation). */
int vx_set_actuation(vx_handle h, const double *amp, const double *phase);

/* Named actuation channels (Volumetric Actuation: several independent
 * "temperatures", each driving only some materials).  Channel k's
 * temperature at time t is offset + amp * w(2 pi freq t + phase), w the
 * waveform: VX_WAVE_SINE sin; VX_WAVE_TRIANGLE the triangle wave in phase
 * with the sine (0 at phase 0, peak +1 a quarter period in, -1 three
 * quarters in, linear between); VX_WAVE_SQUARE +1 for the first half period
 * and -1 for the second.  A voxel's strain is its material's CTE times the
 * temperature of the channel it follows. */
#define VX_MAX_CHANNELS 8
#define VX_WAVE_SINE 0
#define VX_WAVE_TRIANGLE 1
#define VX_WAVE_SQUARE 2
typedef struct vx_channel {
    double amp;        /* K */
    double freq;       /* Hz */
    double phase;      /* rad */
    double offset;     /* K, added to the waveform */
    int32_t waveform;  /* VX_WAVE_* */
    int32_t reserved;  /* must be 0 */
} vx_channel;

/* Set n_ch (0..VX_MAX_CHANNELS) channels, replacing earlier ones.  A filled
 * cell follows channel cell_channel[c] when that is >= 0 (cell_channel:
 * ncell entries, or NULL), else channel mat_channel[m] of its material m
 * when that is >= 0 (mat_channel: n_mat entries indexed by material, or
 * NULL), else its own signal of vx_set_actuation, else the global signal
 * of vx_params.  Errors: VX_EINVAL for n_ch out of range, an unknown
 * waveform, a non-finite field or a channel index >= n_ch. */
int vx_set_channels(vx_handle h, const vx_channel *channels, int32_t n_ch, const int32_t *mat_channel,
                    const int32_t *cell_channel);

/* Initial velocity per cell, dense ncell x 3 (m/s); sets P = m v. */
int vx_set_velocity(vx_handle h, const double *velocity);

/* Advance n steps at the stable timestep (the paper's TimeStep, called n
 * times).  Errors: VX_ESTATE before bind, VX_EUNSTABLE if any state value
 * became non-finite, VX_EOVERFLOW if a candidate list overflowed. */
int vx_step(vx_handle h, int64_t n);

/* Enqueue n steps on the handle's stream and return at once: the call
 * performs kernel launches only (no host synchronisation, no memory set or
 * copy), so it may be recorded into a HIP graph by stream capture of that
 * stream.  A recorded sequence replays the steps with the step times and
 * the buffer order it was recorded with: it starts from the ping-pong
 * buffer the capture started from, so replaying it repeatedly continues the
 * state only for an even n.  The handle's step counter counts enqueued
 * steps.  Non-finite states and candidate overflows are reported by the
 * next vx_step or vx_status.  Errors: VX_ESTATE before bind. */
int vx_step_enqueue(vx_handle h, int64_t n);

/* Record state word `word` (0..12 in the order u_x, u_y, u_z, q_w, q_x,
 * q_y, q_z, P_x, P_y, P_z, L_x, L_y, L_z; u the displacement from the rest
 * position) of the n cells listed in `cells` (a DEVICE array of int32 cell
 * indices, x + nx (y + ny z)) from the current state into `out` (a DEVICE
 * array of n values of the state precision: float for 32, double for 64).
 * Both arrays stay owned by the caller.  This is the sampling step of a long
 * run such as the impulse-response record behind a modal spectrum (the
 * paper's dynamic validation, section Validation, Table 2): one small kernel
 * on the handle's stream, no host synchronisation, so it may be captured in
 * a HIP graph together with vx_step_enqueue (the captured probe reads the
 * ping-pong buffer that is current at capture time, so a captured
 * step-then-probe sequence stays consistent only for an even step count).
 * An index outside the lattice reads as NaN.  Errors: VX_EINVAL for n < 0,
 * a word outside 0..12 or NULL arrays with n > 0; VX_ESTATE before bind. */
int vx_probe(vx_handle h, const int32_t *cells, int32_t n, int32_t word, void *out);

/* Wait for the handle's stream and report the device status: VX_OK,
 * VX_EUNSTABLE (a non-finite value was produced) or VX_EOVERFLOW. */
int vx_status(vx_handle h);

/* Copy the state to the host, widened to double, dense per cell (empty
 * cells read as zero displacement, identity rotation, zero velocity):
 * u = displacement from the rest position (ncell x 3), q = orientation
 * quaternion (w, x, y, z) (ncell x 4), vel = linear velocity (ncell x 3),
 * omega = angular velocity (ncell x 3).  Any pointer may be NULL. */
int vx_read_state(vx_handle h, double *u, double *q, double *vel, double *omega);

/* Overwrite the state (same layout as vx_read_state; NULL = keep). */
int vx_write_state(vx_handle h, const double *u, const double *q, const double *vel,
                   const double *omega);

/* Per-cell flags: is_static (floor static-friction state) and surface. */
int vx_read_flags(vx_handle h, uint8_t *is_static, uint8_t *surface);

int vx_get_dt(vx_handle h, double *dt);       /* timestep, s */
int vx_get_time(vx_handle h, double *t);      /* simulated time, s */

/* out[0] steps taken, out[1] candidate-list rebuilds, out[2] candidate
 * pairs in the current list, out[3] number of voxels (filled cells). */
int vx_counters(vx_handle h, int64_t out[4]);

/* Current collision candidate pairs as (cell_a, cell_b) with
 * cell_a < cell_b; writes at most max_pairs and returns the total count in
 * *n_pairs. */
int vx_candidates(vx_handle h, int32_t *cell_a, int32_t *cell_b, int32_t max_pairs,
                  int32_t *n_pairs);

/* Energies and momenta of the current state, summed over all voxels in
 * FP64 (deterministic order), at time t_n for the actuation strain:
 *   out[0] kinetic energy, sum |P|^2 / 2m + |phi|^2 / 2I (Eq. 27-28 state);
 *   out[1] elastic energy of the bonds, sum 1/2 u2^T K22 u2 with u2 voxel 2's
 *          displacement and rotation in voxel 1's bond frame and K22 the
 *          lower-right block of the beam stiffness (Eq. 7);
 *   out[2] gravitational energy sum m g z (z of the voxel centre);
 *   out[3] floor penalty energy sum 1/2 k delta^2 over voxels in contact;
 *   out[4..6] total linear momentum; out[7..9] total angular momentum about
 *          the world origin (sum of D x P + phi).
 * Blocks until the result is on the host.  Errors: VX_ESTATE before bind. */
int vx_energy(vx_handle h, double out[10]);

/* The same ten sums as vx_energy, written to out[0..9], a DEVICE array of
 * doubles owned by the caller, by two kernels enqueued on the handle's
 * stream (per-workgroup partials, then their sum in a fixed order on the
 * device; the order differs from vx_energy's host sum, so the two agree to
 * FP64 rounding).  No host synchronisation: alternated with
 * vx_step_enqueue it records the energies of every step of a run (the
 * energy-per-step record of the cantilever benchmark, Results) with one
 * wait at the end, and it may be captured in a HIP graph (as vx_probe, the
 * captured kernels read the ping-pong buffer current at capture time).
 * Calls on one handle share its partials buffer, so they run in stream
 * order.  Errors: VX_EINVAL for a NULL array, VX_ESTATE before bind. */
int vx_energy_enqueue(vx_handle h, double *out);

/* Linear statics: the direct-stiffness solution K x = f of the lattice in
 * its rest configuration (section Validation, the "direct stiffness" column
 * of Table 1), solved on the GPU in FP64 by Jacobi-preconditioned conjugate
 * gradients without assembling K.  Every face-adjacent filled pair is the
 * 12-DOF beam element of Eq. (7) with the composite moduli of Eq. (1)-(2)
 * and the section constants of Eq. (8)-(12); the moduli are those the step
 * uses (the palette's, or the per-cell E of vx_set_stiffness, with the
 * palette's Poisson ratio); the voxels of vx_set_fixed are clamped.
 * F is the load, ncell x 3 N on the host (rows of empty or clamped cells are
 * ignored).  u and theta (ncell x 3 each, host, either may be NULL) receive
 * the displacement (m) and rotation (rad) of every cell, zero for empty and
 * clamped ones.  The iteration stops once |r| <= rel_tol |f| (recursive
 * residual, rel_tol > 0) or after max_iter iterations; *iters receives the
 * count and *rel_residual the true |f - K x| / |f| (either may be NULL).
 * `work` is a caller-owned device buffer of vx_static_workspace_bytes
 * bytes, 256-byte aligned.  The state is not touched.  Blocks until done.
 * Errors: VX_EINVAL for bad arguments, a non-finite load or a small or
 * misaligned workspace; VX_ESTATE before bind; VX_EUNSTABLE when rel_tol
 * was not reached (the outputs still hold the last iterate), e.g. for a
 * body with no clamped voxel under a load with a net force. */
int vx_static_workspace_bytes(vx_handle h, uint64_t *bytes);
int vx_static_solve(vx_handle h, void *work, uint64_t work_bytes, const double *F, double rel_tol,
                    int32_t max_iter, double *u, double *theta, int32_t *iters, double *rel_residual);

/* vx_static_solve without a caller workspace, for callers that cannot
 * allocate device memory (serving loops, harnesses that forbid allocation).
 * Same arguments, results and errors as vx_static_solve (bitwise the same
 * solution); the conjugate-gradient vectors live in a fixed 64 MiB device
 * array inside the library, one per device, looked up on the first call on
 * the device the handle's stream runs on.  The call allocates no device
 * memory.  Limit: the lattice's vx_static_workspace_bytes must be at most
 * 64 MiB (about 190,000 cells); larger lattices get VX_EINVAL with the
 * sizes in vx_last_error.  Every call on one device shares that array, so
 * calls that overlap on one device (several host threads, or several
 * handles' streams) race and must be serialised by the caller; each call
 * initialises every part of the array it reads. */
int vx_static_solve_noalloc(vx_handle h, const double *F, double rel_tol, int32_t max_iter, double *u,
                            double *theta, int32_t *iters, double *rel_residual);

/* Self-collision detection scheme (section "Self collision detection and
 * handling" and Table 3, "Speedup of self collision schemes"): all_voxels = 0
 * takes only the surface voxels into the candidate search (default), 1 every
 * filled voxel; every_step = 0 rebuilds the candidate lists only when the
 * accumulated maximum motion could let an unlisted pair touch (the horizon
 * rule, default), 1 before every step.  The schemes differ in cost, not in
 * the contact forces as long as interior voxels stay out of contact.
 * all_voxels can change only before vx_bind_workspace (it sizes the
 * workspace); every_step at any time.  Effective only with
 * self_collision_on.  Errors: VX_EINVAL for values other than 0/1,
 * VX_ESTATE for an all_voxels change after bind. */
int vx_set_collision_mode(vx_handle h, int32_t all_voxels, int32_t every_step);

/* Select the step implementation: 0 = fused LDS-tiled kernel (default;
 * palettes of more than 16 materials and lattices whose state array (13
 * words per cell) spans 4 GiB or more, i.e. beyond about 82 million cells
 * in FP32 or 41 million in FP64, always use the split path), 1 = split
 * per-axis bond kernels plus a gather kernel. */
int vx_set_kernel(vx_handle h, int32_t kind);

/* Tile of the fused kernel: shape index 0..4 = 32x8, 64x4, 16x16, 50x5,
 * 20x12 cells per workgroup in x-y (-1: chosen from the lattice size), zc =
 * z slabs per workgroup (0: chosen from the lattice size).  Results agree
 * across tiles to rounding; one tile is bitwise reproducible. */
int vx_set_fused_tile(vx_handle h, int32_t shape, int32_t zc);
int vx_get_fused_tile(vx_handle h, int32_t *shape, int32_t *tx, int32_t *ty, int32_t *zc);

/* Time every fused tile shape and z chunk on this lattice (iters launches
 * each, from the current state, without advancing it) and keep the fastest.
 * Errors: VX_ESTATE before bind, for a palette of more than 16 materials or
 * a state array spanning 4 GiB or more (the fused kernel does not run). */
int vx_autotune(vx_handle h, int32_t iters, int32_t *shape, int32_t *zc);

/* Average wall time of one launch of the step kernel(s) alone (the fused
 * kernel, or the four kernels of the split path), over iters dry-run
 * launches from the current state, measured with HIP events on the
 * handle's stream; the state does not advance.  For roofline figures. */
int vx_time_kernel(vx_handle h, int32_t iters, double *ms_per_launch);

/* ------------------------------------------------------------------ */
/* Parameter mode and differentiable rollouts                          */
/* ------------------------------------------------------------------ */
/* The paper motivates the simulator as the inner loop of automated design
 * (Sec. 1, Sec. 6): these calls give the gradient of a function of the
 * final state with respect to per-voxel design parameters, by the reverse
 * (adjoint) of the explicit step of Sec. 2-3 (bond forces Eq. 7, 13-24,
 * damping Eq. 33-35, floor and friction Eq. 36-38, integration Eq. 27-30,
 * actuation Eq. 39-40).  Branch decisions (floor contact, friction state)
 * are those of the recorded forward run; the gradient is that of the
 * piecewise-smooth map on the taken branch. */

/* Per-voxel elastic modulus E[ncell] (Pa; read only at filled cells; NULL
 * returns to the palette's moduli).  It replaces the palette modulus in
 * the bond constants (Eq. 1-2, 8-12), the bond damping (Eq. 34-35), the
 * floor stiffness, the ground damping and the voxel-voxel contact
 * stiffness and damping; density, Poisson's ratio, expansion and friction
 * stay the palette's.  The timestep stays the one chosen at create, so
 * every bond's sqrt(k/m_min) must stay at or below the bound it was chosen
 * for (include a material as stiff as the stiffest modulus in the
 * palette).  Steps run a variant of the fused kernel that reads the
 * per-cell values.  Errors: VX_EINVAL for a non-positive or non-finite
 * modulus, or one above the timestep's bound. */
int vx_set_stiffness(vx_handle h, const double *E);

/* Per-voxel density rho[ncell] (kg/m^3; read only at filled cells; NULL
 * returns to the palette's).  It replaces the palette density in the
 * voxel's mass and inertia (m = rho l^3, I = m l^2 / 6) and in every
 * mass-dependent damping coefficient (ground, floor, bond and contact
 * damping, the last two with the lighter voxel of the pair, Eq. 34).  The
 * same stability rule as vx_set_stiffness applies to the pair (modulus,
 * density).  The stored momenta are kept, and vx_read_state,
 * vx_write_state and vx_set_velocity convert them with the cell's own
 * mass.  Errors: VX_EINVAL for a non-positive or non-finite density, or
 * one that puts a bond above the timestep's bound. */
int vx_set_density(vx_handle h, const double *rho);

/* Bytes of the gradient workspace for rollouts of up to max_steps steps
 * with a checkpoint every K steps: ceil(max_steps/K) checkpoints plus a
 * K-step recompute buffer, adjoint state and per-voxel adjoint terms
 * (about (ceil(max_steps/K) + K) x (13 words + 1 byte) + K x 6 words +
 * 35 words + 4 FP64 words per cell, and max_steps bytes for the forward's
 * log of candidate-list rebuilds).  K = 1 is the tape: the forward run
 * stores every step's state, flags and 6 bond-sum words (about max_steps x
 * (19 words + 1 byte) per cell) and the reverse run recomputes nothing. */
int vx_grad_workspace_bytes(vx_handle h, int64_t max_steps, int32_t K, uint64_t *bytes);

/* Bind a caller-owned, 256-byte aligned device buffer of at least
 * vx_grad_workspace_bytes(h, max_steps, K) bytes.  Needs the main
 * workspace bound.  With self-collision on, the forward run logs where the
 * horizon rule rebuilt the candidate lists, the reverse run (and the
 * segment recompute) build them from the states of those steps (and of
 * each segment's first step) and the reverse run applies the contact
 * forces' reverse
 * (gradients through contact; which pairs touch is held fixed, the map is
 * piecewise smooth).  Replaces an
 * earlier binding.  It also takes pinned host memory (about 25 words + 32
 * bytes per cell, freed by vx_destroy) through which the reverse run's
 * host copies go; if that allocation fails the reverse run stages in
 * ordinary host memory instead.  Errors: VX_ESTATE, VX_EINVAL (too small,
 * misaligned, K or max_steps < 1). */
int vx_grad_bind(vx_handle h, void *device_ptr, uint64_t bytes, int64_t max_steps, int32_t K);

/* Advance n steps (1 <= n <= max_steps) like vx_step and record the
 * checkpoints of the run.  Without vx_set_stiffness it first sets every
 * voxel's modulus to its palette value.  Errors as vx_step; VX_ESTATE
 * without a gradient workspace. */
int vx_grad_forward(vx_handle h, int64_t n);

/* Reverse run over the rollout recorded by the last vx_grad_forward, which
 * must end at the current state (any step, state write or setter in
 * between invalidates it: VX_ESTATE).
 * Inputs (host, NULL = zero): adjoint of the final state, dL/du (3 per
 * cell), dL/dq (4 per cell, quaternion w,x,y,z), dL/dv (3), dL/dw (3), in
 * the layout of vx_read_state.
 * Outputs (host, NULL = not wanted), per cell, zero at empty cells:
 *   g_E      dL/dE of vx_set_stiffness's moduli;
 *   g_rho    dL/drho of vx_set_density's densities, with the timestep and
 *            the rollout's initial velocities and angular velocities held
 *            fixed (its initial momenta scale with the mass) and the loss a
 *            function of the final velocities (v = P / m); where two
 *            bonded or touching voxels have equal mass, the damping's
 *            dependence on the lighter mass (which has no derivative
 *            there) is split evenly between them, the mean of the two
 *            one-sided derivatives;
 *   g_phase  dL/dphase, g_amp dL/damp of vx_set_actuation's per-voxel
 *            signal (zero when the voxel follows the global signal or a
 *            channel; see vx_grad_channels);
 *   g_u0, g_q0, g_v0, g_w0  adjoint of the rollout's initial state.
 * The adjoint state is kept in the state's precision; the parameter
 * gradients are accumulated in FP64.  Errors: VX_ESTATE as above,
 * VX_EUNSTABLE for a non-finite value, VX_EOVERFLOW if a candidate list
 * rebuilt during the run (self-collision) overflowed contact_cap,
 * VX_ENOMEM if host staging could not be allocated. */
int vx_grad_backward(vx_handle h, const double *dL_du, const double *dL_dq, const double *dL_dv,
                     const double *dL_dw, double *g_E, double *g_rho, double *g_phase, double *g_amp,
                     double *g_u0, double *g_q0, double *g_v0, double *g_w0);

/* Gradients of the last vx_grad_backward's loss with respect to each
 * actuation channel's phase (rad) and amplitude (K): g_phase[k], g_amp[k]
 * for the n_ch channels of vx_set_channels (host arrays, NULL = not
 * wanted).  They are the sums over the channel's voxels, in FP64 and cell
 * order, of the per-voxel terms the reverse run accumulated (those voxels
 * read zero in vx_grad_backward's per-voxel g_phase and g_amp).  Errors:
 * VX_ESTATE before a vx_grad_backward. */
int vx_grad_channels(vx_handle h, double *g_phase, double *g_amp);

/* ------------------------------------------------------------------ */
/* Batches: many independent objects stepped by one persistent launch  */
/* ------------------------------------------------------------------ */

/* One object of a batch: its own material grid (cell order as vx_create)
 * and the world position of its cell (0,0,0)'s lower corner (z places it
 * above the floor; all three place it in the world shared by a batch with
 * contact). */
typedef struct vx_object {
    const uint8_t *grid;
    int32_t nx, ny, nz;
    int32_t reserved;      /* must be 0 */
    double origin[3];
} vx_object;

typedef struct vx_batch_sim *vx_batch;

/* Create a batch of n_obj objects sharing one palette (at most 16
 * materials) and one parameter set.  The grids are copied.
 * self_collision_on = 0: the objects are independent; each gets its own
 * stable timestep (Eq. 31-32 over its own bonds) and its own time, and
 * vx_batch_step runs max_steps_per_launch steps per persistent launch.
 * self_collision_on = 1: the objects share one world, placed by their
 * origins, and touch one another ("multiple bodies to interact",
 * Introduction; Self collision detection and handling): the surface voxels
 * of all objects form one candidate search (horizon 2 l, pairs of one
 * object within lattice Manhattan distance 3 excluded, lazy rebuild), every
 * voxel gathers its contact force from its own candidate list (no
 * atomics), and all objects step with the smallest of their stable
 * timesteps, one launch per step.  Errors: VX_EINVAL as vx_create, or if
 * one state array (13 words per cell of all objects) would span 4 GiB or
 * more, or an object with a non-zero reserved field or a non-finite origin. */
int vx_batch_create(const vx_object *objs, int32_t n_obj, const vx_material *palette, int32_t n_mat,
                    const vx_params *params, int32_t precision, void *stream, vx_batch *out);
int vx_batch_workspace_bytes(vx_batch b, uint64_t *bytes);
/* Bind the caller's device workspace (256-byte aligned) and upload the rest
 * state of every object. */
int vx_batch_bind_workspace(vx_batch b, void *device_ptr, uint64_t bytes);

/* Advance every object n steps: one persistent kernel launch per
 * max_steps_per_launch steps (default 2000), each workgroup looping all
 * steps over its own objects (with contact: the collision chain, the
 * contact forces and one launch per step).  Errors: VX_ESTATE before bind,
 * VX_EUNSTABLE on a non-finite state, VX_EOVERFLOW if a candidate list
 * overflowed. */
int vx_batch_step(vx_batch b, int64_t n);

/* Read / overwrite one object's state; layouts as vx_read_state over the
 * object's own cells. */
int vx_batch_read_state(vx_batch b, int32_t obj, double *u, double *q, double *vel, double *omega);
int vx_batch_write_state(vx_batch b, int32_t obj, const double *u, const double *q, const double *vel,
                         const double *omega);
int vx_batch_get_dt(vx_batch b, int32_t obj, double *dt);
/* out[0] steps, out[1] objects, out[2] cells, out[3] filled voxels. */
int vx_batch_counters(vx_batch b, int64_t out[4]);

/* Contact between objects (self_collision_on = 1): the current candidate
 * pairs as (object, cell within the object) twice, each pair once, in
 * object-major order of the first voxel; writes at most max_pairs and
 * returns the total in *n_pairs (0 without contact). */
int vx_batch_candidates(vx_batch b, int32_t *obj_a, int32_t *cell_a, int32_t *obj_b, int32_t *cell_b,
                        int32_t max_pairs, int32_t *n_pairs);
/* out[0] candidate-list rebuilds, out[1] candidate entries (each pair
 * counted from both sides), out[2] surface voxels taking part; zeros
 * without contact. */
int vx_batch_contact_counters(vx_batch b, int64_t out[3]);

/* Workgroups of the persistent launch (0: the default, one per object;
 * larger counts are cut to one per object) and steps per launch (0: keep).
 * Objects are assigned to workgroups by longest-processing-time packing on
 * cell count, the largest first. */
int vx_batch_set_launch(vx_batch b, int32_t n_workgroups, int32_t max_steps_per_launch);

/* How each object's x-y footprint is cut into the batch kernel's tiles (at
 * most 64 x 64 cells, 256 in all, marching the object's height): rule 0
 * (the default) takes the widest rows, TX = min(nx, 64), then as many rows
 * as fit; rule 1 keeps rule 0's number of tiles across x but evens their
 * widths (nx = 70: two tiles 35 wide, not 64 and 6), then as many rows as
 * fit, and differs from rule 0 only for footprints over 64 cells wide.
 * Every rule computes the same step (the
 * per-voxel method of Sec. 2-3); the last bits can differ, as a bond on a
 * tile edge reaches its voxel's sum in another order.  May be called before
 * or after binding; after, the object table is copied to the device and the
 * call waits for it on the batch's stream.  VX_EINVAL for another rule. */
int vx_batch_set_tile_rule(vx_batch b, int32_t rule);
/* The tile rule in force and one object's tile: out[0] rule, out[1] TX,
 * out[2] TY.  VX_EINVAL for an object index out of range. */
int vx_batch_get_tile(vx_batch b, int32_t obj, int32_t out[3]);

/* Time each tile rule with candidate workgroup counts (256 to 4096 and
 * one per object) over `steps` steps
 * and keep the fastest pair (the rule reads back through
 * vx_batch_get_tile); the state, the flags and the time are restored
 * afterwards.  On an error (for instance VX_EUNSTABLE from a trial run) the
 * rule, the workgroup count and the state are as before the call. */
int vx_batch_autotune(vx_batch b, int32_t steps, int32_t *n_workgroups);
int vx_batch_destroy(vx_batch b);
const char *vx_batch_last_error(vx_batch b);

/* Free host-side data of the handle (not the caller's workspace). */
int vx_destroy(vx_handle h);

const char *vx_last_error(vx_handle h);

#ifdef __cplusplus
}
#endif
#endif
