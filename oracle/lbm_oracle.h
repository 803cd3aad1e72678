/*
 * lbm_oracle.h -- plain, slow FP64 CPU oracle for the D2Q9 lattice Boltzmann
 * time step with half-way bounce-back on moving solids, newborn-node refill,
 * and the conventional (CME, Eq. 4) and Galilean-invariant (GME, Eq. 5)
 * momentum-exchange force and torque (Eqs. 6-7) of Wen et al.,
 * "Galilean Invariant Fluid-Solid Interfacial Dynamics in Lattice Boltzmann
 * Simulations" (arXiv:1303.0625).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent reference that
 * the GPU path is checked against.  It shares no code, header, table or
 * helper with the GPU library; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.
 *
 * Conventions (lattice units, dx = dt = 1, c_s^2 = 1/3):
 *   - node (x, y) sits at integer coordinates, 0 <= x < nx, 0 <= y < ny;
 *     arrays are row-major [y][x], populations [9][ny][nx];
 *   - x is periodic; y is periodic unless walls_y = 1, in which case virtual
 *     solid rows at y = -1 and y = ny (solid id 0) put half-way walls at
 *     y = -1/2 and y = ny - 1/2, moving at (wall_vx, wall_vy);
 *   - body s (1-based) occupies node (x, y) at step t iff an integer image of
 *     the node lies inside its shape centred at (cx + t*vx, cy + t*vy) when it
 *     moves, or at (cx, cy) when it does not;
 *   - g is an acceleration: the body-force density is rho*g (Guo forcing);
 *   - forces are those on the solid, by the fluid.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_DISC = 0, ORC_BOX = 1 };
enum { ORC_CME = 0, ORC_GME = 1 };
enum { ORC_A1 = 0, ORC_A2 = 1, ORC_A3 = 2 };

typedef struct orc_body {
    int kind;        /* ORC_DISC or ORC_BOX */
    int moves;       /* 0: fixed geometry, v only enters bounce-back and GME */
    double cx, cy;   /* centre at t = 0 */
    double a;        /* disc radius, or box half-width along x */
    double b;        /* box half-height along y (unused for a disc) */
    double vx, vy;   /* prescribed body velocity */
} orc_body;

typedef struct orc_sim orc_sim;

/* Returns NULL on invalid arguments (tau <= 1/2, nx or ny < 1, refill out of range). */
orc_sim* orc_create(int nx, int ny, int walls_y, double tau, double rho0,
                    double gx, double gy, double u0x, double u0y,
                    double wall_vx, double wall_vy, int refill, int rho_w_local,
                    int n_bodies, const orc_body* bodies);
void orc_destroy(orc_sim* s);

/* Advance n time steps. */
void orc_step(orc_sim* s, long n);
long orc_time(const orc_sim* s);

/* rho, ux, uy of the current pre-collision state (Guo velocity); 0 at solid
 * nodes.  owner receives 0 for fluid and the body id for solid nodes.  Any
 * pointer may be NULL. */
void orc_fields(const orc_sim* s, double* rho, double* ux, double* uy, int* owner);

/* Force record of step `step` (0-based, < orc_time), solid `solid`
 * (0 = walls, 1..n = bodies): out = {Fx, Fy, Tz} for the scheme. Returns 0 on
 * success, -1 on an out-of-range request. */
int orc_force(const orc_sim* s, long step, int solid, int scheme, double out[3]);

/* Per-link records of the most recent completed step, in summation order.
 * Writes up to max records; returns the total count.  rec[k*8 + ...] =
 * {x, y, i, solid, cme_fx, cme_fy, gme_fx, gme_fy}. */
long orc_links(const orc_sim* s, long max, double* rec);

/* Pre-collision populations f(t), [9][ny][nx]; zero at solid nodes. */
void orc_get_f(const orc_sim* s, double* f);
void orc_set_f(orc_sim* s, const double* f);

/* Replace the state by f = f_eq(rho, u - g/2) so that the Guo velocity of the
 * new state is u (warm start). */
void orc_init_fields(orc_sim* s, const double* rho, const double* ux, const double* uy);

/* ---- building blocks, exposed for pinning ---- */

/* Eq. 8 equilibrium for all nine directions. */
void orc_feq(double rho, double ux, double uy, double out[9]);

/* Eq. 4 (scheme = ORC_CME) or Eq. 5 (ORC_GME) on one link in direction i,
 * given a = post-collision f_i at the fluid node, b = post-collision f_ibar
 * leaving the boundary node, and the boundary velocity v. */
void orc_link_force(int i, double a, double b, double vx, double vy,
                    int scheme, double out[2]);

/* One BGK + Guo collision of one node's nine populations. */
void orc_collide_node(const double f[9], double tau, double gx, double gy,
                      double out[9]);

/* Make disc `body` (1-based) a free body (Sec. IV: particles moving under
 * gravity and the hydrodynamic force) before the first step: density rho_s,
 * mass M = rho_s pi r^2, moment of inertia I = M r^2 / 2, initial velocity
 * its (vx, vy), initial angular velocity omega0.  Each step, after the
 * forces of step t (scheme of orc_set_gravity), V(t+1) = V(t) + (F +
 * (M - rho0 pi r^2) G)/M, Omega(t+1) = Omega(t) + T/I, X(t+1) = X(t) +
 * V(t+1); its surface moves at V + Omega z x (p - X) in bounce-back, in the
 * force of every link (at the link midpoint) and in the refill fallback.
 * Returns 0, or -1 (not a disc, t > 0, rho_s <= 0, bad index). */
int orc_set_free(orc_sim* s, int body, double rho_s, double omega0);

/* Interpolated bounce-back on body links (Sec. IV; linear in the fraction q
 * of the link from the fluid node x_f to the surface): the population
 * returning to x_f in direction ibar is
 *   q < 1/2:  2q f~_i(x_f) + (1 - 2q) f~_i(x_f - e_i) + m_ibar
 *             (half-way bounce-back when x_f - e_i is not fluid),
 *   q >= 1/2: f~_i(x_f)/(2q) + (2q - 1)/(2q) f~_ibar(x_f) + m_ibar/(2q),
 * m_ibar = 6 w_i rho_w (e_ibar . v) with the surface velocity v at x_f + q e_i;
 * the link force (Eqs. 4-5) takes this population as the returning one and
 * the torque arm ends at x_f + q e_i.  Wall rows keep half-way bounce-back. */
void orc_set_ibb(orc_sim* s, int on);

/* q of the link from fluid node (x, y) in direction i into body `body` at
 * the current step (test access). */
double orc_link_q(const orc_sim* s, int body, long x, long y, int i);

/* Gravity G on free bodies (buoyancy-corrected: (M - rho0 A) G) and the force
 * scheme (ORC_CME / ORC_GME) that drives them. */
void orc_set_gravity(orc_sim* s, double Gx, double Gy, int scheme);

/* out = {X, Y, V_x, V_y, Omega} of body `body` at the current step. */
int orc_body_state(const orc_sim* s, int body, double out[5]);

/* Switch the collision to the multiple-relaxation-time operator of Sec. IV
 * with S = diag(0, s_e, s_eps, 0, s_q, 0, s_q, 1/tau, 1/tau) over the moments
 * (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy); same equilibrium (Eq. 8) and
 * Guo forcing.  Applies from the next step on. */
void orc_set_mrt(orc_sim* s, double s_e, double s_eps, double s_q);

/* One MRT collision of one node with the nine moment rates s[9]. */
void orc_collide_node_mrt(const double f[9], const double s[9], double gx, double gy, double out[9]);

/* The moment matrix M (row-major 9 x 9) and its inverse (Gauss-Jordan). */
void orc_mrt_matrix(double out[81]);
void orc_mrt_inverse(double inv[81]);

/* Newborn refill of node (x, y) from post-stream values fpost [9][ny][nx] of
 * the nodes marked old-fluid (oldfluid[y*nx+x] != 0).  Periodic wrap in x,
 * and in y unless walls_y.  When no direction participates, out = f_eq(rho0, v).
 * Returns the number of participating directions. */
int orc_refill_node(int nx, int ny, int walls_y, const double* fpost,
                    const int* oldfluid, int x, int y, int scheme,
                    double rho0, double vx, double vy, double out[9]);

#ifdef __cplusplus
}
#endif
#endif
