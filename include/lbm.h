/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q9 lattice Boltzmann library with
 * half-way bounce-back on moving solids, newborn-node refill and the
 * conventional / Galilean-invariant momentum-exchange force.
 *
 * Method: Wen, Zhang, Tu, Wang, Fang, "Galilean Invariant Fluid-Solid
 * Interfacial Dynamics in Lattice Boltzmann Simulations", arXiv:1303.0625.
 *   - lattice Boltzmann equation, collision and advection: Sec. II, Eqs. 1-3;
 *     single-relaxation-time (BGK) collision with the Eq. 8 equilibrium and the
 *     D2Q9 velocity set of Sec. III.C;
 *   - half-way bounce-back with the moving-boundary term: Sec. I and III.A;
 *   - conventional momentum exchange (CME): Eq. 4; Galilean-invariant
 *     momentum exchange (GME): Eq. 5; total force and torque: Eqs. 6-7;
 *   - refill of newborn fluid nodes (A1 second-order extrapolation, A2 linear
 *     extrapolation, A3 neighbour value, averaged over participating links):
 *     Sec. IV.B.
 *
 * Units are lattice units (dx = dt = 1, c_s^2 = 1/3).  Node (x, y) sits at
 * integer coordinates, 0 <= x < nx, 0 <= y < ny.  Fields are row-major
 * [y][x] with x fastest.  x is periodic; y is periodic unless walls_y = 1,
 * which places half-way walls at y = -1/2 and y = ny - 1/2 (solid id 0).
 * Bodies have ids 1..n in the order given.  Forces are those exerted on the
 * solid by the fluid; torque is about the body's prescribed centre (z out of
 * plane).  The walls' torque is reported as 0.
 *
 * Ownership.  The caller owns every buffer passed in (workspace, field and
 * output buffers) and the HIP stream; they must outlive the context.  The
 * library allocates no device memory: all device state lives in the caller's
 * workspace, whose size lbm_workspace_bytes() reports.  The grid and solid
 * structs are copied at create.
 *
 * Streams and synchronisation.  Every call that launches work enqueues it on
 * the context's stream and returns without waiting, except lbm_force,
 * lbm_save and lbm_status_check, which synchronise that stream.
 *
 * Errors.  Every call returns an lbm_status and, on failure, records a message
 * that lbm_last_error() returns.  Faults detected on the device (link-list
 * overflow, non-finite or non-positive density found by lbm_fields) are
 * latched in the workspace and reported as LBM_EGEOM / LBM_ENUMERIC by the
 * next synchronising call.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 1

typedef struct lbm_ctx lbm_ctx; /* opaque; created by lbm_create, freed by lbm_destroy */

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,   /* invalid argument (NULL pointer, tau <= 1/2, |v| >= 0.3, ...) */
    LBM_ESIZE = -2,    /* workspace or output buffer too small */
    LBM_EDEVICE = -3,  /* a HIP runtime call failed */
    LBM_ENUMERIC = -4, /* non-finite or non-positive density detected */
    LBM_ESTATE = -5,   /* call not valid in the context's current state */
    LBM_EGEOM = -6     /* bodies overlap, touch the walls, or a link list overflowed */
} lbm_status;

/* Storage type of the populations.  All storage types keep the deviation
 * f_i - w_i rho0 from the rest equilibrium.  F64 computes in double, the
 * others collide in float.  Force and torque are always accumulated in double. */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16 = 2, LBM_BF16 = 3 } lbm_dtype;

typedef enum { LBM_CME = 0, LBM_GME = 1 } lbm_scheme; /* Eq. 4 / Eq. 5 */

typedef enum { LBM_REFILL_A1 = 0, LBM_REFILL_A2 = 1, LBM_REFILL_A3 = 2 } lbm_refill;

typedef enum { LBM_DISC = 0, LBM_BOX = 1 } lbm_shape;

typedef struct {
    int32_t nx, ny;       /* lattice size, nx >= 4, ny >= 4 */
    int32_t walls_y;      /* 1: half-way walls at y = -1/2 and ny - 1/2 */
    int32_t dtype;        /* lbm_dtype of the stored populations */
    int32_t refill;       /* lbm_refill used for newborn nodes */
    int32_t rho_w_local;  /* reserved, must be 0: the wall term uses rho0 */
    double rho0;          /* reference density; initial density */
    double gx, gy;        /* body-force acceleration (force density rho*g) */
    double u0x, u0y;      /* initial populations f_eq(rho0, u0) */
    double wall_vx, wall_vy; /* velocity of the walls (solid id 0) */
} lbm_grid;

typedef struct {
    int32_t shape;        /* lbm_shape */
    int32_t moves;        /* 0: geometry fixed, v enters only bounce-back and GME;
                             1: the geometry translates at v */
    double cx, cy;        /* centre at t = 0 */
    double a;             /* disc radius, or box half-width along x */
    double b;             /* box half-height along y (ignored for a disc) */
    double vx, vy;        /* prescribed velocity, |v| < 0.3 */
} lbm_solid;
/* A node (x, y) belongs to a body at step t when an integer image
 * (x + k nx, y + l ny) of it lies inside the shape centred at
 * (cx + t vx, cy + t vy) (moving) or (cx, cy) (fixed): a disc holds the points
 * with dx*dx + dy*dy <= a*a, a box those with |dx| <= a and |dy| <= b, each
 * product and sum rounded separately in double. */

/* Version of this ABI (LBM_ABI_VERSION). */
int32_t lbm_abi_version(void);

/* Bytes of device workspace a context needs for this configuration, keeping
 * a force history of history_steps steps (a ring; >= 1).  Returns LBM_EINVAL
 * on invalid arguments. */
lbm_status lbm_workspace_bytes(const lbm_grid* grid, const lbm_solid* solids, int32_t n_solids,
                               int64_t history_steps, size_t* bytes);

/* Validate the configuration, lay out the caller's device workspace
 * (d_workspace, at least lbm_workspace_bytes() bytes, 256-byte aligned),
 * rasterise the bodies, build the link lists and initialise the populations
 * to f_eq(rho0, u0) (Eq. 8), collided once.  hip_stream is a hipStream_t
 * (NULL: the default stream).  tau is the BGK relaxation time, > 1/2.
 * On success *out receives the context. */
lbm_status lbm_create(const lbm_grid* grid, double tau, const lbm_solid* solids, int32_t n_solids,
                      int64_t history_steps, void* d_workspace, size_t bytes, void* hip_stream,
                      lbm_ctx** out);

/* For callers that cannot allocate device memory (harnesses that forbid
 * hipMalloc, serving loops that must not allocate): lbm_create without a
 * workspace argument.  The context lives in a static array of 64 MiB that
 * the library holds on each device it runs on (until the process ends);
 * this call allocates no device memory, and lbm_step of such a context
 * launches its kernels one by one (no graph, whose instantiation may
 * allocate).  One such context per device at a time: LBM_ESTATE while
 * another is alive on the current device (destroy it first; the array keeps
 * the last context's contents, and lbm_create rewrites every part of it a
 * context reads before reading it).  LBM_ESIZE when the configuration needs
 * more than 64 MiB (lbm_workspace_bytes); calls on one context from several
 * threads or streams at once race, as for any context.  Otherwise as
 * lbm_create. */
lbm_status lbm_create_static(const lbm_grid* grid, double tau, const lbm_solid* solids, int32_t n_solids,
                             int64_t history_steps, void* hip_stream, lbm_ctx** out);

/* Enqueue n time steps.  Each step evaluates the CME and GME force and torque
 * of every solid from the current post-collision populations (Eqs. 4-7),
 * streams with half-way bounce-back (Eq. 3), moves the translating bodies,
 * refills newborn nodes and collides (Eq. 2).  Asynchronous.  Returns
 * LBM_EGEOM if a translating body would come within 2 nodes of another body
 * or a wall during these steps. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* Number of completed time steps. */
int64_t lbm_time(const lbm_ctx* ctx);

/* Force and torque {Fx, Fy, Tz} on solid solid_id (0 = walls) by scheme
 * (lbm_scheme) at the most recent completed step, into host memory out[3].
 * Synchronises the stream.  LBM_ESTATE before the first step. */
lbm_status lbm_force(lbm_ctx* ctx, int32_t solid_id, int32_t scheme, double out[3]);

/* Copy the force records of steps [first, first + count) into device memory
 * d_out as double [count][n_solids + 1][6] = {CME Fx, Fy, Tz, GME Fx, Fy, Tz}.
 * The steps must still be held by the history ring.  Asynchronous. */
lbm_status lbm_force_history(lbm_ctx* ctx, int64_t first, int64_t count, double* d_out);

/* Density and Guo velocity of the current state (the mass and momentum
 * densities of Sec. II, rho = sum f_i and rho u = sum e_i f_i + rho g / 2 with
 * the body-force half step) into device buffers of nx*ny elements of type
 * out_dtype (LBM_F64 or LBM_F32); 0 at solid nodes.
 * d_owner (optional) receives the owner map as uint8 (0 = fluid, else body
 * id).  Any output pointer may be NULL.  Latches LBM_ENUMERIC if a fluid node
 * has a non-finite or non-positive density.  Asynchronous. */
lbm_status lbm_fields(lbm_ctx* ctx, void* d_rho, void* d_ux, void* d_uy, int32_t out_dtype,
                      uint8_t* d_owner);

/* Replace the state of every fluid node by f_eq(rho, u - g/2), collided once,
 * so that its Guo velocity is u (warm start).  Inputs are device buffers of
 * nx*ny elements of type in_dtype (LBM_F64 or LBM_F32).  Asynchronous. */
lbm_status lbm_init_fields(lbm_ctx* ctx, const void* d_rho, const void* d_ux, const void* d_uy,
                           int32_t in_dtype);

/* Free bodies (Sec. IV: particles moving under gravity and the hydrodynamic
 * force).  Before the first step, make body solid_id a free rigid disc of
 * density rho_s (it must be a disc created with moves = 1; its (vx, vy) is
 * the initial velocity, omega0 the initial angular velocity): mass
 * M = rho_s pi r^2, moment of inertia I = M r^2 / 2.  After the forces of
 * step t (the scheme lbm_set_gravity names, GME by default): V(t+1) = V(t) +
 * (F + (M - rho0 pi r^2) G)/M, Omega(t+1) = Omega(t) + T/I, X(t+1) = X(t) +
 * V(t+1); its surface moves at V + Omega z x (p - X) in bounce-back, in the
 * force of every link (p the link midpoint) and in the refill fallback.
 * Free bodies add one small launch per step; their paths are not validated
 * ahead: meeting a wall or another body, or moving more than half a node in
 * a step, makes the next synchronising call return LBM_EGEOM.  Checkpoints
 * (lbm_save / lbm_load) are refused while free bodies exist.  Synchronises. */
lbm_status lbm_set_free_body(lbm_ctx* ctx, int32_t solid_id, double rho_s, double omega0);

/* Gravity G = (gx, gy) on free bodies (buoyancy-corrected: the fluid carries
 * no gravity) and the force scheme (LBM_CME / LBM_GME) that drives them. */
lbm_status lbm_set_gravity(lbm_ctx* ctx, double gx, double gy, int32_t scheme);

/* out = {X, Y, V_x, V_y, Omega} of body solid_id at the current step
 * (prescribed bodies: their closed-form centre and velocity, Omega = 0).
 * Synchronises. */
lbm_status lbm_body_state(lbm_ctx* ctx, int32_t solid_id, double out[5]);

/* Bounce-back rules on body links. */
typedef enum { LBM_HALFWAY = 0, LBM_INTERPOLATED = 1 } lbm_boundary_rule;

/* Choose the rule on fluid-body links (default LBM_HALFWAY: the surface at
 * the link midpoint).  LBM_INTERPOLATED is the interpolated bounce-back the
 * paper runs its simulations with (Sec. IV), linear in the fraction q of the
 * link from the fluid node x_f to the surface (q from the exact disc or box
 * shape at the step's centre, minimum image on periodic axes): the
 * population returning to x_f against link direction i is
 *   q < 1/2:  2q f~_i(x_f) + (1 - 2q) f~_i(x_f - e_i) - m   (half-way when
 *             x_f - e_i is not fluid),
 *   q >= 1/2: (f~_i(x_f) - m)/(2q) + (1 - 1/(2q)) f~_ibar(x_f),
 * m = 6 w_i rho0 (e_i . v) with the surface velocity v at x_f + q e_i.  The
 * link forces (Eqs. 4-5) take that population as the returning one, the
 * torque arm (Eq. 7) ends at x_f + q e_i, and the newborn refill
 * extrapolates from values streamed with the same rule.  Wall rows keep
 * half-way bounce-back.  Takes effect from the next step; the batched solver
 * uses half-way bounce-back only.  LBM_EINVAL for another rule. */
lbm_status lbm_set_boundary(lbm_ctx* ctx, int32_t rule);

/* Collision operators. */
typedef enum { LBM_BGK = 0, LBM_MRT = 1 } lbm_collision;

/* Choose the collision operator (default LBM_BGK, Eq. 2 with the single
 * relaxation time tau).  LBM_MRT is the multiple-relaxation-time operator the
 * paper pairs with its simulations (Sec. IV): relaxation in the moment space
 * (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy) of the D2Q9 basis with
 * S = diag(0, s_e, s_eps, 0, s_q, 0, s_q, 1/tau, 1/tau), the Eq. 8
 * equilibrium and Guo's forcing ((I - S/2) in moment space); rates[3] =
 * {s_e, s_eps, s_q}, each in (0, 2) (the paper: 1.64, 1.54, 1.9); ignored for
 * BGK.  Only before the first step (LBM_ESTATE after): the state is reset to
 * f_eq(rho0, u0) collided once with the chosen operator.  Force evaluation,
 * bounce-back and refill are unchanged; the newborn refill collides with the
 * chosen operator.  Asynchronous. */
lbm_status lbm_set_collision(lbm_ctx* ctx, int32_t model, const double* rates);

/* Replace the state by the exact steady plane-Poiseuille flow of the
 * unobstructed channel at every fluid node: f = f_eq(rho0, u_P(y) - g/2),
 * collided once, with u_P(y) = g_x/(2 nu) (Y^2 - (y - y_c)^2) + s, Y = ny/2,
 * y_c = (ny - 1)/2, s = g_x (16 Lambda - 3) / (24 nu), nu = (tau - 1/2)/3,
 * Lambda = (tau - 1/2)^2 for BGK and (tau - 1/2)(1/s_q - 1/2) for MRT (Guo
 * forcing between half-way walls; Eq. 2-3).  A non-learned warm start.
 * Needs walls_y = 1 (LBM_ESTATE otherwise).  Asynchronous. */
lbm_status lbm_init_poiseuille(lbm_ctx* ctx);

/* Post-collision populations f~_i(x, t) of the current state as absolute
 * values in double, [9][ny][nx] device memory; 0 at solid nodes.  Asynchronous. */
lbm_status lbm_populations(lbm_ctx* ctx, double* d_out);

/* Per-link CME/GME forces that the next step will evaluate from the current
 * state, in summation order: d_out double [max][8] =
 * {x, y, i, solid, CME Fx, CME Fy, GME Fx, GME Fy}; *n receives the number
 * of links (host).  Synchronises the stream.  LBM_ESIZE if max is too small. */
lbm_status lbm_link_forces(lbm_ctx* ctx, double* d_out, int64_t max, int64_t* n);

/* Checkpoint: bytes needed, save into / load from a device buffer.  The
 * record holds the populations, owner maps, link lists and the step counter;
 * the force history is not saved.  lbm_save synchronises. */
lbm_status lbm_checkpoint_bytes(const lbm_ctx* ctx, size_t* bytes);
lbm_status lbm_save(lbm_ctx* ctx, void* d_dst, size_t bytes);
lbm_status lbm_load(lbm_ctx* ctx, const void* d_src, size_t bytes);

/* Kernel timing (instrumentation).  While enabled, every time-step launch
 * (one kernel per step: force, moving-body and fused advection + bounce-back
 * + collision workgroups, the last moving 18 populations per fluid node) is
 * timed by a pair of HIP events attached to its dispatch on the context's
 * stream; lbm_profile_read synchronises and returns the summed elapsed
 * milliseconds and the number of launches since enabling.  Enabling resets
 * the sums.  At most 65536 launches are recorded. */
lbm_status lbm_profile(lbm_ctx* ctx, int32_t enable);
lbm_status lbm_profile_read(lbm_ctx* ctx, double* update_ms, int64_t* launches);

/* Synchronise the stream and report any latched device fault. */
lbm_status lbm_status_check(lbm_ctx* ctx);

/* Release the context (not the caller's buffers). NULL is ignored. */
void lbm_destroy(lbm_ctx* ctx);

/* Message of the last failure on this context, or of the last failed
 * lbm_create / lbm_workspace_bytes in this thread when ctx is NULL. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* ------------------------------------------------------------------------
 * Batched steady-state solver: many independent lattices of uneven sizes
 * (fixed geometry, moves = 0) advanced together until each one is steady.
 *
 * One launch per time step updates the tiles of every active case (the same
 * per-node arithmetic as lbm_step, so a case advanced here matches the same
 * case advanced alone bit for bit).  Every check interval of k steps a
 * monitor evaluates on the device, per case:
 *   - the residual r = ||u_t - u_{t-k}||_2 / (k ||u_t||_2) over fluid nodes,
 *     u the Guo velocity (a steady-state criterion the paper does not state;
 *     the momentum density it is built from is the one of Sec. II);
 *   - CME and GME force and torque on every solid (Eqs. 4-7), summed in a
 *     fixed order (deterministic);
 * and retires a case once r < tol: its state freezes and its tiles leave the
 * launch.  lbm_batch_run captures one interval (k steps + monitor) as a HIP
 * graph and replays it.  Work runs on a stream the batch owns, ordered after
 * the work enqueued on hip_stream so far; every lbm_batch_* call that
 * launches work synchronises before it returns.
 *
 * Device state (populations, owner maps, links, snapshots, tables) lives in
 * the caller's workspace; the batch allocates no device memory itself.
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch; /* opaque; lbm_batch_create / lbm_batch_destroy */

/* Workspace bytes of a batch.  grids[n_cases] and taus[n_cases] describe the
 * cases (one dtype for all); solids holds the bodies of case 0, then of case
 * 1, ..., n_solids[c] of them for case c; no body may move. */
lbm_status lbm_batch_workspace_bytes(const lbm_grid* grids, const double* taus, const lbm_solid* solids,
                                     const int32_t* n_solids, int32_t n_cases, size_t* bytes);

/* Validate every case (as lbm_create does), lay out the workspace, build the
 * geometry and links and initialise every case to f_eq(rho0, u0), collided
 * once.  The initial tiling is 4 waves (256 nodes of one row band) per
 * workgroup.  Synchronises.  *out receives the batch. */
lbm_status lbm_batch_create(const lbm_grid* grids, const double* taus, const lbm_solid* solids,
                            const int32_t* n_solids, int32_t n_cases, void* d_workspace, size_t bytes,
                            void* hip_stream, lbm_batch** out);

/* Time the step launch over the candidate tilings (1, 2, 4 or 8 waves per
 * workgroup, cached or nontemporal streaming) and keep the fastest; then
 * reset every case to its initial state.  Only before the first step
 * (LBM_ESTATE otherwise).  cache_path (optional) is a text file of
 * "signature|waves|nontemporal|us" lines: a matching line is used without
 * timing, a new result is appended. */
lbm_status lbm_batch_autotune(lbm_batch* b, const char* cache_path);

/* Waves per workgroup of the current tiling; *nontemporal (optional) receives
 * 1 when the update streams with nontemporal loads and stores. */
int32_t lbm_batch_tiling(const lbm_batch* b, int32_t* nontemporal);

/* Set the tiling: waves (1, 2, 4 or 8 per workgroup) and nontemporal (1:
 * the update streams with nontemporal loads and stores).  Any tiling gives
 * the same results bit for bit; only the speed differs. */
lbm_status lbm_batch_set_tiling(lbm_batch* b, int32_t waves, int32_t nontemporal);

/* Enable (1, the default) or disable (0) graph capture in lbm_batch_run. */
lbm_status lbm_batch_set_graph(lbm_batch* b, int32_t enable);

/* Advance every active case by n steps (no monitor).  Synchronises. */
lbm_status lbm_batch_step(lbm_batch* b, int64_t n);

/* Run the monitor at the current step with the interval since the previous
 * monitor; retire the cases with r < tol (tol < 0 retires none).  The first
 * monitor only records the snapshot (residual -1).  Synchronises. */
lbm_status lbm_batch_monitor(lbm_batch* b, double tol);

/* Run intervals of k steps (check_every rounded up to even, >= 2), each
 * followed by the monitor, until every case has retired or another interval
 * would exceed max_steps steps in this call.  *steps_done (optional, host)
 * receives the steps taken.  Synchronises. */
lbm_status lbm_batch_run(lbm_batch* b, int64_t max_steps, double tol, int32_t check_every,
                         int64_t* steps_done);

/* Per-case results of the last monitor into host arrays of n_cases entries
 * (each pointer optional): converged flag, steps (the step at retirement, or
 * the current step), residual (-1 before the second monitor) and drag[2c],
 * drag[2c+1] = sum over the case's bodies of the CME and GME x-force. */
lbm_status lbm_batch_status(lbm_batch* b, int32_t* converged, int64_t* steps, double* residual,
                            double* drag);

/* {Fx, Fy, Tz} on solid solid_id (0 = walls) of case case_id by scheme, as of
 * the last monitor, into host memory. */
lbm_status lbm_batch_force(lbm_batch* b, int32_t case_id, int32_t solid_id, int32_t scheme,
                           double out[3]);

/* Density and Guo velocity of case case_id (at its retirement step if it has
 * retired) into device buffers of nx*ny elements (LBM_F64 or LBM_F32); 0 at
 * solid nodes.  d_owner (optional) receives the owner map as uint8.
 * Synchronises. */
lbm_status lbm_batch_fields(lbm_batch* b, int32_t case_id, void* d_rho, void* d_ux, void* d_uy,
                            int32_t out_dtype, uint8_t* d_owner);

/* Warm start of case case_id, as lbm_init_fields; with all three field
 * pointers NULL, the cold start the batch was created with (f_eq(rho0, u0)
 * collided once: the fallback of a warm start that fails lbm_warm_check or
 * diverges).  The case's residual starts over (the next check records its
 * snapshot only).  Synchronises. */
lbm_status lbm_batch_init_fields(lbm_batch* b, int32_t case_id, const void* d_rho, const void* d_ux,
                                 const void* d_uy, int32_t in_dtype);

/* Retire (active = 0) or reactivate (active = 1) case case_id by hand.  A
 * retired case keeps its state and leaves the step launch; a reactivated case
 * continues from its state (moved to the current step's buffer if needed)
 * and its residual starts over.  With lbm_batch_init_fields after the
 * reactivation, a case can be handed over from another batch (for instance
 * from FP16 storage to FP32).  Synchronises. */
lbm_status lbm_batch_set_active(lbm_batch* b, int32_t case_id, int32_t active);

/* Warm start of case case_id by the exact plane-Poiseuille flow, as
 * lbm_init_poiseuille.  Synchronises. */
lbm_status lbm_batch_init_poiseuille(lbm_batch* b, int32_t case_id);

/* Completed steps of the batch (cases advanced together). */
int64_t lbm_batch_time(const lbm_batch* b);

/* Release the batch (not the caller's buffers).  NULL is ignored. */
void lbm_batch_destroy(lbm_batch* b);

/* Message of the last failure on this batch, or (b NULL) of the last failed
 * lbm_batch_create / lbm_batch_workspace_bytes in this thread. */
const char* lbm_batch_last_error(const lbm_batch* b);

/* ------------------------------------------------------------------------
 * Learned warm start: a 4-level U-Net mapping a channel's solid mask and
 * Reynolds number to an approximate steady (rho, u_x, u_y), used as the
 * initial state of a solve (lbm_init_fields / lbm_batch_init_fields), with
 * the cold start f_eq(rho0, u0) kept as the fallback.  The paper has no
 * network; what it feeds is the solver of Sec. II-IV, whose steady fields
 * are the training data.
 *
 * Network: level l = 0..3 at (h >> l) x (w >> l); encoder levels 0..2 apply
 * two 3x3 convolutions with ReLU (channels ch[l]) and a 2x2 mean pool;
 * level 3 applies two, and its per-sample channel means (global context: the
 * flow rate of a periodic channel depends on every body in it) join the
 * first decoder level; decoder levels 2..0 upsample 2x (nearest),
 * concatenate [upsampled, encoder output of the level (, level 2: the means
 * broadcast to every node)] and apply two 3x3 convolutions with ReLU; a last
 * 3x3 convolution gives 3 outputs.  x is periodic, y zero-padded.  Input
 * channels: solid (1) / fluid (0) and Re/100.
 * Outputs (normalised): (rho - 1) / (U_c rho_scale), u_x / U_c, u_y / U_c with
 * U_c = g_x h^2 / (8 nu), nu = (tau - 1/2) / 3, the centre-line speed of the
 * unobstructed channel.
 *
 * Parameters: one FP32 vector; for each of the 15 convolutions in order
 * (encoder 0a 0b 1a 1b 2a 2b, bottleneck a b, decoder 2a 2b 1a 1b 0a 0b,
 * head) the weights W[c_out][ky][kx][c_in] then the bias[c_out]; decoder 2a
 * reads c_in = 2 ch[3] + ch[2] channels [up, skip, means].  Activations
 * are NHWC in BF16 (matrix-core inputs, FP32 accumulation) or FP32.  Every
 * reduction has a fixed order: results are reproducible bit for bit.
 * All device state lives in the caller's workspace; calls are asynchronous on
 * the given stream unless they return a host value.
 * ------------------------------------------------------------------------ */
typedef struct lbm_nn lbm_nn; /* opaque; lbm_nn_create / lbm_nn_destroy */

typedef struct {
    int32_t h, w;      /* lattice rows (ny, multiple of 8) and columns (nx, multiple of 64) */
    int32_t max_batch; /* samples per call, >= 1 */
    int32_t dtype;     /* LBM_BF16 or LBM_F32 activations */
    int32_t ch[4];     /* channels per level, multiples of 32 in [32, 1024]; ch[3] <= 256 */
    double rho_scale;  /* scale of the density output */
} lbm_nn_config;

/* Workspace bytes of a network (LBM_EINVAL for an invalid configuration). */
lbm_status lbm_nn_workspace_bytes(const lbm_nn_config* cfg, size_t* bytes);

/* Lay out the workspace (256-byte aligned device memory of at least
 * lbm_nn_workspace_bytes); parameters start at zero. */
lbm_status lbm_nn_create(const lbm_nn_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
                         lbm_nn** out);

/* Number of FP32 parameters. */
int64_t lbm_nn_param_count(const lbm_nn* nn);

/* Copy the parameter vector in (also resets Adam's moments) or out; device
 * memory of lbm_nn_param_count floats. */
lbm_status lbm_nn_set_params(lbm_nn* nn, const float* d_params);
lbm_status lbm_nn_get_params(lbm_nn* nn, float* d_params);

/* Gradient of the last lbm_nn_backward / lbm_nn_train_step (device, FP32). */
lbm_status lbm_nn_get_grads(lbm_nn* nn, float* d_grads);

/* Network output y [batch][h][w][3] (FP32) of the input x [batch][h][w][2]
 * (FP32), device memory. */
lbm_status lbm_nn_forward(lbm_nn* nn, const float* d_x, int32_t batch, float* d_y);

/* Gradient of sum(gy * y) with respect to the parameters, for the input of
 * the last lbm_nn_forward; gy [batch][h][w][3] FP32 device memory. */
lbm_status lbm_nn_backward(lbm_nn* nn, const float* d_gy);

/* One convolution layer alone (layers 1..13), for inspection and tests of
 * the convolution kernels: y = ReLU(conv3x3(x, W) + b) with the network's
 * current parameters rounded to the compute type, x periodic, y zero
 * outside the image.  x is the layer's input at its level,
 * [batch][h_l][w_l][x_cs] in the compute type (channels [0, cin) used,
 * x_cs >= cin), y receives [batch][h_l][w_l][y_cs] (channels [0, cout)
 * written, y_cs >= cout); strides multiples of 8, tensors 16-byte aligned
 * device memory.  Leaves the network's state untouched; synchronises. */
lbm_status lbm_nn_layer_forward(lbm_nn* nn, int32_t layer, int32_t batch, const void* d_x, int32_t x_cs,
                                void* d_y, int32_t y_cs);

/* Weight and bias gradient of one layer alone, for inspection and tests of
 * the weight-gradient kernels: dW[co][ky][kx][ci] = sum over pixels p of
 * g[p][co] x[p + (ky - 1, kx - 1)][ci] (x periodic, y zero outside the
 * image) and db[co] = sum over p of g[p][co], in FP32 accumulation.  x is
 * the layer's input at its level, [batch][h_l][w_l][x_cs] in the network's
 * compute type (channels [0, cin) used; x_cs >= cin, >= 16 for layer 0), g
 * the pre-activation gradient [batch][h_l][w_l][g_cs] (channels [0, cout)
 * used; g_cs >= cout rounded up to 32); both strides multiples of 8, both
 * tensors 16-byte aligned device memory.  d_grad (device, FP32) receives
 * cout * 9 * cin weights then cout biases, the layout of the layer in the
 * parameter vector.  Layer levels: 0,0,1,1,2,2,3,3,2,2,1,1,0,0,0.  Leaves the
 * network's own gradient and last batch untouched; synchronises. */
lbm_status lbm_nn_layer_wgrad(lbm_nn* nn, int32_t layer, int32_t batch, const void* d_x, int32_t x_cs,
                              const void* d_g, int32_t g_cs, float* d_grad);

/* One Adam step (Kingma and Ba, bias-corrected) on the current gradient. */
lbm_status lbm_nn_adam(lbm_nn* nn, double lr, double beta1, double beta2, double eps);

/* Training step on the samples d_idx[0..batch) (NULL: 0..batch-1) of a data
 * set held in device memory: solid mask u8 [N][h][w], steady fields rho, u_x,
 * u_y FP32 [N][h][w], and per sample Re, g_x and tau (FP64 [N]).  d_aug
 * (optional, int32 [batch]) transforms each drawn sample: bits 0..15 shift it
 * periodically in x by that many nodes, bit 16 mirrors it about the channel
 * centre line (u_y changes sign) -- both map a steady channel flow to the
 * steady flow of the transformed geometry.  The loss is the mean over fluid
 * nodes and the 3 outputs of the squared error of the normalised output; then
 * backward and Adam (beta 0.9, 0.999, eps 1e-8) with learning rate lr.  *loss
 * (optional, host) receives the loss before the update and makes the call
 * synchronise. */
lbm_status lbm_nn_train_step(lbm_nn* nn, const uint8_t* d_solid, const float* d_rho, const float* d_ux,
                             const float* d_uy, const double* d_re, const double* d_gx, const double* d_tau,
                             const int32_t* d_idx, const int32_t* d_aug, int32_t batch, double lr, double* loss);

/* The loss of lbm_nn_train_step without the update (synchronises). */
lbm_status lbm_nn_eval(lbm_nn* nn, const uint8_t* d_solid, const float* d_rho, const float* d_ux, const float* d_uy,
                       const double* d_re, const double* d_gx, const double* d_tau, const int32_t* d_idx,
                       int32_t batch, double* loss);

/* Warm-start fields of `batch` channels: solid mask u8 [batch][h][w] and per
 * sample Re, g_x, tau (FP64 device [batch]) -> rho, u_x, u_y FP32
 * [batch][h][w] (0 at solid nodes), device memory. */
lbm_status lbm_nn_infer(lbm_nn* nn, const uint8_t* d_solid, const double* d_re, const double* d_gx,
                        const double* d_tau, int32_t batch, float* d_rho, float* d_ux, float* d_uy);

/* Make warm-start fields safe to start from, in place, for n_fields channels
 * of nx x ny (nx even, both <= 2048): owner map u8 and rho, u_x, u_y FP32,
 * [n_fields][ny][nx] device memory, fluid nodes only.  When the second set
 * (rho2, u_x2, u_y2; all or none) is given, the fields are first replaced by
 * the mean of the two sets: with the fields of two consecutive steps of a
 * started lattice, the spurious modes that change sign every step (excited
 * where a warm field meets a body) cancel.  Then rho is shifted to mean
 * rho0 (the mass of a cold start, so the steady drag, which balances g_x sum
 * rho, is the same); u_x is scaled column by column to equal fluxes
 * sum_y rho u_x (continuity), u_y shifted row by row to zero flux.  A lattice
 * started at equilibrium from fields without this carries a staggered
 * momentum sum_x (-1)^x rho u_x that changes sign every step and is never
 * damped (it makes the force on a body alternate; a residual over an even
 * interval does not see it).  Asynchronous on hip_stream; LBM_EINVAL on bad
 * sizes. */
lbm_status lbm_warm_project(int32_t nx, int32_t ny, int32_t n_fields, const uint8_t* d_owner, float* d_rho,
                            float* d_ux, float* d_uy, const float* d_rho2, const float* d_ux2, const float* d_uy2,
                            double rho0, void* hip_stream);

/* Start check of warm-start fields (the learned start falls back to the cold
 * start of a channel whose fields fail it): for each of n_fields channels of
 * nx x ny, d_ok[k] (int32 device [n_fields]) = 1 when every fluid node (owner
 * 0) has a finite density in (0, 2 rho0) and a finite velocity of magnitude
 * <= u_max, else 0.  Inputs as for lbm_warm_project, not modified.  The
 * density and momentum it bounds are those of Sec. II.  Asynchronous on
 * hip_stream; LBM_EINVAL on bad sizes, NULL pointers or rho0, u_max <= 0. */
lbm_status lbm_warm_check(int32_t nx, int32_t ny, int32_t n_fields, const uint8_t* d_owner, const float* d_rho,
                          const float* d_ux, const float* d_uy, double rho0, double u_max, int32_t* d_ok,
                          void* hip_stream);

/* Release the network (not the caller's buffers).  NULL is ignored. */
void lbm_nn_destroy(lbm_nn* nn);

/* Message of the last failure on this network, or (NULL) of the last failed
 * lbm_nn_create / lbm_nn_workspace_bytes in this thread. */
const char* lbm_nn_last_error(const lbm_nn* nn);

/* ------------------------------------------------------------------------
 * Three dimensions (Sec. IV.D): the D3Q19 step with the same boundary and
 * force evaluation, for fixed, translating and free spheres in a duct.
 *
 * Velocity set: rest, the six axis directions and the twelve edge diagonals,
 * weights 1/3, 1/18, 1/36.  Every axis is periodic.  The duct is a circular
 * tube along x (nodes with (y - (ny-1)/2)^2 + (z - (nz-1)/2)^2 > R^2 are
 * solid), the two planes z = 0 and z = nz - 1, or nothing; spheres are solid
 * where (minimum-image) |p - X|^2 <= r^2, each product and sum rounded
 * separately, and their surfaces move rigidly at V + omega x (p - X); a
 * sphere with moves = 1 also translates, X(t) = X + t V (product and sum
 * rounded separately): after each step the geometry of the next one is
 * rasterised and its newborn nodes are refilled as in two dimensions (A1, A2
 * or A3 of grid->refill along every D3Q19 link whose neighbour stays fluid,
 * averaged, then collided; the surface-velocity equilibrium when none does).
 * A moving sphere must keep 2 nodes from the duct and from every other sphere
 * (lbm3d_step returns LBM_EGEOM before launching otherwise), and its scan box
 * of 2 ceil(r) + 5 nodes must fit the lattice.  One step: the CME (Eq. 4) and
 * GME (Eq. 5) forces of
 * every fluid-solid link from the post-collision populations with the torque
 * (Eq. 7) about each sphere's centre at the link's surface point (the
 * midpoint, or x_f + q e_i under lbm3d_set_boundary), summed per solid in a
 * fixed order (Eq. 6); pull streaming with half-way (or interpolated)
 * bounce-back plus 6 w_i rho0 (e_i . v) (v at the surface point); BGK
 * collision (Eq. 2) with
 * the Eq. 8 equilibrium and Guo forcing for the body force g.  Storage:
 * LBM_F64 or LBM_F32 deviations f_i - w_i rho0, arithmetic in FP64.  The
 * caller owns the device workspace and the stream; nothing is allocated on
 * the device by the library.
 * ------------------------------------------------------------------------ */
typedef struct lbm3d_ctx lbm3d_ctx; /* opaque; lbm3d_create / lbm3d_destroy */

typedef enum { LBM3D_OPEN = 0, LBM3D_TUBE = 1, LBM3D_PLANES = 2 } lbm3d_duct;

typedef struct {
    int32_t nx, ny, nz;   /* lattice size, each >= 4, nx ny nz < 2^27 */
    int32_t dtype;        /* LBM_F64 or LBM_F32 */
    int32_t duct;         /* lbm3d_duct */
    int32_t refill;       /* lbm_refill for the newborn nodes of moving spheres */
    double R;             /* tube radius (LBM3D_TUBE), >= 2 */
    double tau;           /* BGK relaxation time, > 1/2 */
    double rho0;          /* reference and initial density */
    double g[3];          /* body-force acceleration (force density rho g) */
    double u0[3];         /* initial populations f_eq(rho0, u0), collided once */
} lbm3d_grid;

typedef struct {
    double X[3];          /* centre at t = 0 */
    double r;             /* radius, >= 1 */
    double V[3];          /* surface translation velocity, |V| < 0.3 */
    double omega[3];      /* surface angular velocity */
    int32_t moves;        /* 1: the sphere translates, X(t) = X + t V */
    int32_t pad;          /* must be 0 */
} lbm3d_sphere;

/* Workspace size for a 3D lattice (validates as lbm3d_create does). */
lbm_status lbm3d_workspace_bytes(const lbm3d_grid* grid, const lbm3d_sphere* spheres, int32_t n_spheres,
                                 int64_t history_steps, size_t* bytes);

/* Validate, build the owner map and link lists on the host, lay out the
 * caller's 256-byte aligned device workspace of `bytes` bytes and initialise
 * the populations; history_steps force records are kept (a ring).  LBM_EGEOM
 * when a sphere overlaps the duct or another sphere.  Synchronises. */
lbm_status lbm3d_create(const lbm3d_grid* grid, const lbm3d_sphere* spheres, int32_t n_spheres,
                        int64_t history_steps, void* d_workspace, size_t bytes, void* hip_stream,
                        lbm3d_ctx** out);

/* Enqueue n time steps (one launch each, pressure planes included; free
 * spheres add a Newton-Euler launch, moving spheres an owner-map and a
 * refill launch; plus one launch for the last step's force totals).
 * Asynchronous. */
lbm_status lbm3d_step(lbm3d_ctx* ctx, int64_t n);

/* Completed time steps. */
int64_t lbm3d_time(const lbm3d_ctx* ctx);

/* out = {F_x, F_y, F_z, T_x, T_y, T_z} of solid `solid` (0 the duct, k the
 * k-th sphere) for scheme LBM_CME / LBM_GME at step `step` (-1: the last
 * completed step).  Synchronises. */
lbm_status lbm3d_force(lbm3d_ctx* ctx, int32_t solid, int32_t scheme, int64_t step, double out[6]);

/* Copy the force records of steps [first, first + count) to device memory
 * d_out, [count][n_spheres + 1][12] doubles: CME {F, T}, then GME {F, T}.
 * Asynchronous. */
lbm_status lbm3d_force_history(lbm3d_ctx* ctx, int64_t first, int64_t count, double* d_out);

/* Device outputs, (z, y, x) order, each optional (NULL skips it): d_rho[N],
 * d_u[3][N] (Guo velocity (sum e_i f_i + rho g/2)/rho of the pre-collision
 * state), d_owner[N] (0 fluid, k sphere k, 255 duct), N = nx ny nz; zeros at
 * solid nodes.  Asynchronous. */
lbm_status lbm3d_fields(lbm3d_ctx* ctx, double* d_rho, double* d_u, int32_t* d_owner);

/* Number of fluid-solid links of the fixed solids (a moving sphere's links
 * are found by a scan of its box each step). */
int64_t lbm3d_link_count(const lbm3d_ctx* ctx);

/* Sphere `sphere` (1-based, created with moves = 1) becomes free: density
 * rho_s (mass M = rho_s 4/3 pi r^3, moment of inertia 2/5 M r^2), initial
 * velocity its V, initial spin omega0.  After each step the scheme chosen by
 * lbm3d_set_gravity (default LBM_GME) drives it explicitly:
 * V' = V + (F + (M - rho0 Vol) G)/M, Omega' = Omega + T/I, X' = X + V'.
 * Its path is not validated ahead: coming within 2 nodes of the duct or of
 * another sphere, or moving more than half a node in a step, makes
 * lbm3d_status_check return LBM_EGEOM.  Before the first step only
 * (LBM_ESTATE after).  Synchronises. */
lbm_status lbm3d_set_free(lbm3d_ctx* ctx, int32_t sphere, double rho_s, const double omega0[3]);

/* Gravity G on free spheres (buoyancy-corrected: the fluid carries none) and
 * the force scheme (LBM_CME / LBM_GME) that drives them. */
lbm_status lbm3d_set_gravity(lbm3d_ctx* ctx, const double G[3], int32_t scheme);

/* Bounce-back rule on curved walls (LBM_HALFWAY default, or
 * LBM_INTERPOLATED: the rule of lbm_set_boundary on sphere and tube links,
 * q the nearer root of the ray-sphere intersection or the ray's exit from
 * the tube's circle; the planes stay half-way).  Takes effect from the next
 * step.  LBM_EINVAL for another rule. */
lbm_status lbm3d_set_boundary(lbm3d_ctx* ctx, int32_t rule);

/* Pressure-driven duct (Sec. IV.D): the planes x = 0 and x = nx - 1 become a
 * pressure inlet (density rho_in) and outlet (rho_out) by non-equilibrium
 * extrapolation: after each step's collision their populations are
 * f_eq(rho_b, u) + (f~ - f_eq(rho, u)) of the neighbouring plane's node
 * (rho and u its density and momentum over density), replacing what the
 * periodic x axis streamed there; a plane node whose neighbour is solid keeps
 * its ordinary update.  Fixed spheres only (LBM_EINVAL with
 * moving ones); before the first step (LBM_ESTATE after).  Asynchronous. */
lbm_status lbm3d_set_pressure(lbm3d_ctx* ctx, double rho_in, double rho_out);

/* enable != 0: free spheres are driven by the mean of the forces and torques
 * of steps t - 1 and t (step 0: its own), the two-step average used for
 * suspended particles; it keeps spheres near neutral buoyancy (rho_s ~ rho0)
 * stable, where the plain explicit update oscillates and diverges. */
lbm_status lbm3d_set_force_average(lbm3d_ctx* ctx, int32_t enable);

/* out = {X, V, Omega} (three components each) of sphere `sphere` at the
 * current step.  Synchronises. */
lbm_status lbm3d_body_state(lbm3d_ctx* ctx, int32_t sphere, double out[9]);

/* LBM_EGEOM if a free sphere met the duct or another sphere (see
 * lbm3d_set_free), else LBM_OK.  Synchronises. */
lbm_status lbm3d_status_check(lbm3d_ctx* ctx);

/* Per-launch step timing with HIP events (as lbm_profile / lbm_profile_read). */
lbm_status lbm3d_profile(lbm3d_ctx* ctx, int32_t enable);
lbm_status lbm3d_profile_read(lbm3d_ctx* ctx, double* step_ms, int64_t* launches);

void lbm3d_destroy(lbm3d_ctx* ctx);

/* Message of the last failure on this context, or of the last failed
 * lbm3d_create / lbm3d_workspace_bytes in this thread when ctx is NULL. */
const char* lbm3d_last_error(const lbm3d_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
