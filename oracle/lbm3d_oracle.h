/* lbm3d_oracle.h -- FP64 CPU oracle of the D3Q19 momentum-exchange step
 * (test infrastructure only).  Sec. IV.D: the method in three dimensions. */
#pragma once

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC3_CME = 0, ORC3_GME = 1 };
enum { ORC3_OPEN = 0, ORC3_TUBE = 1, ORC3_PLANES = 2 };
enum { ORC3_A1 = 0, ORC3_A2 = 1, ORC3_A3 = 2 };

typedef struct orc3_sim orc3_sim;

/* nx x ny x nz periodic lattice, BGK relaxation time tau, reference density
 * rho0, body force (acceleration) g, initial velocity u0 (f = f_eq(rho0, u0)).
 * duct: ORC3_TUBE (nodes with (y - (ny-1)/2)^2 + (z - (nz-1)/2)^2 > R^2 are
 * solid), ORC3_PLANES (z = 0 and z = nz - 1 solid) or ORC3_OPEN.  spheres:
 * ns records {X, Y, Z, r, Vx, Vy, Vz, Omx, Omy, Omz} (rigid surface motion;
 * fixed unless orc3_set_moving / orc3_set_free).  NULL when a sphere touches
 * the duct or another sphere. */
orc3_sim* orc3_create(int nx, int ny, int nz, double tau, double rho0, const double g[3], const double u0[3],
                      int duct, double R, int ns, const double* spheres);
void orc3_destroy(orc3_sim* s);
long orc3_time(const orc3_sim* s);
void orc3_step(orc3_sim* s, long n);

/* rho[N], u[3][N] (Guo velocity) and owner[N] (0 fluid, k sphere k, 255
 * duct), N = nx ny nz in (z, y, x) order. */
void orc3_fields(const orc3_sim* s, double* rho, double* u, int* owner);

/* {F, T} of solid `solid` (0 the duct, k sphere k) at step `step` for
 * scheme ORC3_CME / ORC3_GME; -1 out of range. */
int orc3_force(const orc3_sim* s, long step, int solid, int scheme, double out[6]);

void orc3_feq(double rho, const double u[3], double out[19]);
void orc3_collide_node(const double f[19], double tau, const double g[3], double out[19]);
void orc3_link_force(int i, double a, double b, const double v[3], int scheme, double out[3]);

/* Sphere `sphere` (1-based) translates at its V from step 0 on (before the
 * first step only); refill: the newborn scheme for all moving spheres.
 * -1 when rejected. */
int orc3_set_moving(orc3_sim* s, int sphere, int moving, int refill);
void orc3_refill_node(int nx, int ny, int nz, const double* fn, const unsigned char* own_t,
                      const unsigned char* own_n, int x, int y, int z, int scheme, int* np, double out[19]);
/* Sphere `sphere` (created moving) becomes free: density rho_s, initial spin
 * omega0, initial velocity its V (before the first step only). */
int orc3_set_free(orc3_sim* s, int sphere, double rho_s, const double omega0[3]);
/* Drive free spheres with the mean of the forces and torques of steps t - 1
 * and t (step 0: its own), the two-step average of particle suspensions. */
void orc3_set_force_average(orc3_sim* s, int on);
/* Interpolated bounce-back (linear in the link fraction q, as in two
 * dimensions) on sphere and tube links; the planes stay half-way. */
void orc3_set_ibb(orc3_sim* s, int on);
/* q of the link from node (x, y, z) along direction i into sphere `sphere`
 * at the current step. */
double orc3_link_q(const orc3_sim* s, int sphere, int x, int y, int z, int i);
/* q of the link from node (., y, z) along direction i to the tube wall. */
double orc3_tube_q(const orc3_sim* s, int y, int z, int i);
/* Pressure inlet x = 0 (density rho_in) and outlet x = nx - 1 (rho_out) by
 * non-equilibrium extrapolation of the post-collision populations from the
 * neighbouring plane; no moving spheres; before the first step. */
int orc3_set_pressure(orc3_sim* s, double rho_in, double rho_out);
/* Gravity on free spheres (buoyancy-corrected) and the scheme that drives them. */
void orc3_set_gravity(orc3_sim* s, const double G[3], int scheme);
/* {X, V, Omega} of sphere `sphere` at the current step. */
int orc3_body_state(const orc3_sim* s, int sphere, double out[9]);
/* Non-zero when a moving sphere met the duct or another sphere. */
int orc3_error(const orc3_sim* s);

/* Keep per-link records of each step (at most cap links; 0 turns them off),
 * and copy those of the last step: 11 doubles per link, {x, y, z, i, solid
 * (0 the duct), CME force (3), GME force (3)}; returns the count. */
void orc3_record_links(orc3_sim* s, long cap);
long orc3_links(const orc3_sim* s, double* out, long max);

/* pre-collision populations [19][nz][ny][nx] */
void orc3_get_f(const orc3_sim* s, double* out);
void orc3_set_f(orc3_sim* s, const double* in);
/* post-collision populations of the last step [19][nz][ny][nx]; the pressure
 * planes hold their extrapolated state (the one the next streaming reads) */
void orc3_get_ft(const orc3_sim* s, double* out);

#ifdef __cplusplus
}
#endif
