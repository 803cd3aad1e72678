/* lbm3d_oracle.c -- plain FP64 CPU oracle of the three-dimensional
 * momentum-exchange step (test infrastructure only; shares no code with the
 * GPU library).
 *
 * Sec. IV.D carries the method over to three dimensions (a sphere in a tube
 * Poiseuille flow).  This file is the D3Q19 version of the two-dimensional
 * oracle's fixed-geometry step, in the same order:
 *   collide   Eq. 2 (BGK) with the Eq. 8 equilibrium written for D3Q19 and
 *             Guo's forcing for the body force g (ρu = Σ e_i f_i + ρg/2)
 *   forces    Eq. 4 (CME) and Eq. 5 (GME) on every fluid-solid link from the
 *             post-collision population a leaving the fluid node and the
 *             bounced population b = a - 6 w_i ρ0 (e_i . v), summed per solid
 *             (Eq. 6) with the torque r x F about the sphere's centre (Eq. 7),
 *             r from the centre to the link midpoint
 *   advect    Eq. 3; a population whose source node is solid is the half-way
 *             bounce-back of the node's own opposite population plus
 *             6 w_i ρ0 (e_i . v), v the surface velocity at the link midpoint
 * Spheres carry a rigid surface motion V + Ω x (p - X); a sphere marked
 * moving also translates, X(t) = X0 + t V (product and sum rounded
 * separately), and after advection the geometry of step t + 1 is rasterised:
 * nodes it covers leave the fluid, newborn nodes (solid at t, fluid at t + 1)
 * are refilled from the post-advection values of old-fluid neighbours along
 * every participating direction k (A1: 3 f(x+e_k) - 3 f(x+2e_k) + f(x+3e_k),
 * A2: 2 f(x+e_k) - f(x+2e_k), A3: f(x+e_k), falling back A1 -> A2 -> A3 where
 * the farther nodes are not old fluid), averaged over the participants, or
 * f_eq(rho0, v) at the node's surface velocity when none participates
 * (Sec. IV.B written for D3Q19).  A free sphere (density rho_s, mass
 * M = rho_s 4/3 pi r^3, moment of inertia 2/5 M r^2) takes, after the forces
 * of step t, the explicit Newton-Euler step of the two-dimensional free
 * discs: V' = V + (F + (M - rho0 Vol) G)/M, Omega' = Omega + T/I,
 * X' = X + V', with the chosen scheme's F and T; its surface then moves at
 * V + Omega x (p - X) with the state of the step.  The duct is a circular tube along x (nodes
 * farther than R from the axis are solid), two solid planes z = 0 and
 * z = nz - 1, or nothing.
 * Every axis is periodic (the duct walls are solid nodes).  Summation orders
 * are fixed: nodes in (z, y, x) order, directions in index order.
 *
 * Velocity set: rest, the six axis directions, the twelve edge diagonals;
 * weights 1/3, 1/18, 1/36 (the D3Q19 weights for which the equilibrium's
 * second moment is ρ/3 I + ρ u u, pinned in the tests).
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "lbm3d_oracle.h"

static const int E[19][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                             {0, 0, 1},   {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                             {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                             {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double weight(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
static int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

struct orc3_sim {
    int nx, ny, nz;
    double tau, rho0, g[3];
    int duct;
    double R;
    int ns;
    double* sp;  /* ns x 10: X[3], r, V[3], Om[3] */
    int* moving; /* per sphere: translates at V */
    int* free_;  /* per sphere: Newton-Euler motion */
    double* dyn; /* per sphere: X, V, Om at the current step, then X', V', Om' (18) */
    double* mass; /* per sphere: M, I, volume */
    double G[3];
    int dyn_scheme;
    int force_avg; /* drive free spheres with the mean force of steps t - 1 and t */
    int pressure;  /* inlet x = 0 at rho_in, outlet x = nx - 1 at rho_out */
    int ibb;       /* interpolated bounce-back on sphere links */
    double rho_in, rho_out;
    int advanced; /* dyn holds step t + 1 in its second half */
    int refill;  /* ORC3_A1 / A2 / A3 */
    int err;     /* geometry error met while stepping */
    unsigned char* own;
    unsigned char* own_n;
    double *f, *ft, *fn; /* [19][nz][ny][nx] */
    long t;
    double* hist; /* per step (ns + 1) x 12: CME F, T, GME F, T */
    long hist_cap;
    double* rec;  /* link records of the last step (x, y, z, i, solid, CME F, GME F), or NULL */
    long rec_n, rec_cap;
};

static long nidx(const orc3_sim* s, int x, int y, int z) {
    return ((long)z * s->ny + y) * s->nx + x;
}
static long pidx(const orc3_sim* s, int i, int x, int y, int z) {
    return (long)i * s->nx * s->ny * s->nz + nidx(s, x, y, z);
}
static int wrap(int a, int n) { return ((a % n) + n) % n; }

/* Centre of sphere k at step t (a free sphere: its state at step t, or at
 * t + 1 once the step's dynamics are done). */
static void centre(const orc3_sim* s, int k, long t, double X[3]) {
    const double* p = s->sp + 10 * k;
    if (s->free_[k]) {
        const double* D = s->dyn + 18 * k + ((s->advanced && t == s->t + 1) ? 9 : 0);
        for (int d = 0; d < 3; ++d) X[d] = D[d];
        return;
    }
    for (int d = 0; d < 3; ++d) X[d] = s->moving[k] ? p[d] + (double)t * p[4 + d] : p[d];
}

/* Translation and spin of sphere k at step t. */
static void motion(const orc3_sim* s, int k, long t, double V[3], double Om[3]) {
    const double* p = s->sp + 10 * k;
    const double* src = p + 4;
    const double* som = p + 7;
    if (s->free_[k]) {
        const double* D = s->dyn + 18 * k + ((s->advanced && t == s->t + 1) ? 9 : 0);
        src = D + 3;
        som = D + 6;
    }
    for (int d = 0; d < 3; ++d) {
        V[d] = src[d];
        Om[d] = som[d];
    }
}
static double min_image(double d, int n) { return d - (double)n * floor(d / (double)n + 0.5); }

/* Solid membership at step t: the duct first, then the spheres (minimum
 * image). */
static int classify(const orc3_sim* s, int x, int y, int z, long t, int* overlap) {
    int duct = 0;
    if (s->duct == ORC3_TUBE) {
        double dy = (double)y - 0.5 * (s->ny - 1), dz = (double)z - 0.5 * (s->nz - 1);
        duct = dy * dy + dz * dz > s->R * s->R;
    } else if (s->duct == ORC3_PLANES) {
        duct = (z == 0 || z == s->nz - 1);
    }
    int owner = duct ? 255 : 0;
    for (int k = 0; k < s->ns; ++k) {
        const double* p = s->sp + 10 * k;
        double X[3];
        centre(s, k, t, X);
        double dx = min_image((double)x - X[0], s->nx);
        double dy = min_image((double)y - X[1], s->ny);
        double dz = min_image((double)z - X[2], s->nz);
        if (dx * dx + dy * dy + dz * dz <= p[3] * p[3]) {
            if (owner != 0) *overlap = 1;
            owner = k + 1;
        }
    }
    return owner;
}

/* Rigid surface velocity of solid `owner` at point (px, py, pz) at step t;
 * the duct is at rest. */
static void surface_velocity(const orc3_sim* s, int owner, long t, double px, double py, double pz, double v[3],
                             double r[3]) {
    v[0] = v[1] = v[2] = 0.0;
    r[0] = r[1] = r[2] = 0.0;
    if (owner == 255 || owner == 0) return;
    double X[3], V[3], Om[3];
    centre(s, owner - 1, t, X);
    motion(s, owner - 1, t, V, Om);
    r[0] = min_image(px - X[0], s->nx);
    r[1] = min_image(py - X[1], s->ny);
    r[2] = min_image(pz - X[2], s->nz);
    v[0] = V[0] + (Om[1] * r[2] - Om[2] * r[1]);
    v[1] = V[1] + (Om[2] * r[0] - Om[0] * r[2]);
    v[2] = V[2] + (Om[0] * r[1] - Om[1] * r[0]);
}

/* Fraction q in (0, 1] of the link from fluid node (x, y, z) along e into
 * sphere k at step t: the nearer root of |P + q e|^2 = r^2, P the node's
 * minimum-image offset from the centre. */
static double sphere_q(const orc3_sim* s, int k, long t, int x, int y, int z, const int e[3]) {
    double X[3];
    centre(s, k, t, X);
    const double P[3] = {min_image((double)x - X[0], s->nx), min_image((double)y - X[1], s->ny),
                         min_image((double)z - X[2], s->nz)};
    const double r = s->sp[10 * k + 3];
    double a2 = 0.0, b2 = 0.0, c2 = -r * r;
    for (int d = 0; d < 3; ++d) {
        a2 += (double)(e[d] * e[d]);
        b2 += 2.0 * P[d] * e[d];
        c2 += P[d] * P[d];
    }
    double disc = b2 * b2 - 4.0 * a2 * c2;
    if (disc < 0.0) disc = 0.0;
    double q = (-b2 - sqrt(disc)) / (2.0 * a2);
    if (q <= 0.0) q = 1e-12;
    return q > 1.0 ? 1.0 : q;
}

/* Fraction q in (0, 1] of the link from fluid node (x, y, z) along e to the
 * tube wall: the larger root of |P + q e|^2 = R^2 in the (y, z) plane, P the
 * node's offset from the axis (the node lies inside, its neighbour outside). */
static double tube_q(const orc3_sim* s, int y, int z, const int e[3]) {
    const double py = (double)y - 0.5 * (s->ny - 1), pz = (double)z - 0.5 * (s->nz - 1);
    const double a2 = (double)(e[1] * e[1] + e[2] * e[2]);
    const double b2 = 2.0 * (py * e[1] + pz * e[2]);
    const double c2 = py * py + pz * pz - s->R * s->R;
    double disc = b2 * b2 - 4.0 * a2 * c2;
    if (disc < 0.0) disc = 0.0;
    double q = (-b2 + sqrt(disc)) / (2.0 * a2);
    if (q <= 0.0) q = 1e-12;
    return q > 1.0 ? 1.0 : q;
}

/* Link fraction of a fluid-solid link (half-way for the planes). */
static double link_q3(const orc3_sim* s, int o, long t, int x, int y, int z, const int e[3]) {
    if (!s->ibb) return 0.5;
    if (o != 255) return sphere_q(s, o - 1, t, x, y, z, e);
    return s->duct == ORC3_TUBE ? tube_q(s, y, z, e) : 0.5;
}

double orc3_tube_q(const orc3_sim* s, int y, int z, int i) {
    if (i < 1 || i > 18 || (E[i][1] == 0 && E[i][2] == 0)) return -1.0;
    return tube_q(s, y, z, E[i]);
}

double orc3_link_q(const orc3_sim* s, int sphere, int x, int y, int z, int i) {
    if (sphere < 1 || sphere > s->ns || i < 1 || i > 18) return -1.0;
    return sphere_q(s, sphere - 1, s->t, x, y, z, E[i]);
}

void orc3_set_ibb(orc3_sim* s, int on) { s->ibb = on ? 1 : 0; }

void orc3_feq(double rho, const double u[3], double out[19]) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < 19; ++i) {
        double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
        out[i] = rho * weight(i) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

void orc3_collide_node(const double f[19], double tau, const double g[3], double out[19]) {
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
        rho += f[i];
        for (int d = 0; d < 3; ++d) j[d] += E[i][d] * f[i];
    }
    double u[3], F[3];
    for (int d = 0; d < 3; ++d) {
        F[d] = rho * g[d];
        u[d] = (j[d] + 0.5 * F[d]) / rho;
    }
    double feq[19];
    orc3_feq(rho, u, feq);
    for (int i = 0; i < 19; ++i) {
        double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
        double src = 0.0;
        for (int d = 0; d < 3; ++d) src += (3.0 * (E[i][d] - u[d]) + 9.0 * eu * E[i][d]) * F[d];
        out[i] = f[i] - (f[i] - feq[i]) / tau + (1.0 - 0.5 / tau) * weight(i) * src;
    }
}

void orc3_link_force(int i, double a, double b, const double v[3], int scheme, double out[3]) {
    for (int d = 0; d < 3; ++d) {
        if (scheme == ORC3_CME)
            out[d] = E[i][d] * a + E[i][d] * b; /* e_i a - e_ibar b */
        else
            out[d] = (E[i][d] - v[d]) * a + (E[i][d] + v[d]) * b; /* (e_i - v) a - (e_ibar - v) b */
    }
}

orc3_sim* orc3_create(int nx, int ny, int nz, double tau, double rho0, const double g[3], const double u0[3],
                      int duct, double R, int ns, const double* spheres) {
    if (nx < 2 || ny < 2 || nz < 2 || !(tau > 0.5) || ns < 0 || ns > 200) return NULL;
    orc3_sim* s = (orc3_sim*)calloc(1, sizeof(orc3_sim));
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->tau = tau;
    s->rho0 = rho0;
    for (int d = 0; d < 3; ++d) s->g[d] = g[d];
    s->duct = duct;
    s->R = R;
    s->ns = ns;
    s->sp = (double*)malloc(sizeof(double) * 10 * (ns > 0 ? ns : 1));
    if (ns > 0) memcpy(s->sp, spheres, sizeof(double) * 10 * ns);
    s->moving = (int*)calloc((size_t)(ns > 0 ? ns : 1), sizeof(int));
    s->free_ = (int*)calloc((size_t)(ns > 0 ? ns : 1), sizeof(int));
    s->dyn = (double*)calloc((size_t)18 * (ns > 0 ? ns : 1), sizeof(double));
    s->mass = (double*)calloc((size_t)3 * (ns > 0 ? ns : 1), sizeof(double));
    s->dyn_scheme = ORC3_GME;
    long N = (long)nx * ny * nz;
    s->own = (unsigned char*)calloc((size_t)N, 1);
    s->own_n = (unsigned char*)calloc((size_t)N, 1);
    s->f = (double*)calloc((size_t)(19 * N), sizeof(double));
    s->ft = (double*)calloc((size_t)(19 * N), sizeof(double));
    s->fn = (double*)calloc((size_t)(19 * N), sizeof(double));
    int overlap = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) s->own[nidx(s, x, y, z)] = (unsigned char)classify(s, x, y, z, 0, &overlap);
    if (overlap) {
        orc3_destroy(s);
        return NULL;
    }
    double fe[19];
    orc3_feq(rho0, u0, fe);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                if (s->own[nidx(s, x, y, z)] == 0)
                    for (int i = 0; i < 19; ++i) s->f[pidx(s, i, x, y, z)] = fe[i];
    return s;
}

void orc3_destroy(orc3_sim* s) {
    if (!s) return;
    free(s->rec);
    free(s->sp);
    free(s->moving);
    free(s->free_);
    free(s->dyn);
    free(s->mass);
    free(s->own);
    free(s->own_n);
    free(s->f);
    free(s->ft);
    free(s->fn);
    free(s->hist);
    free(s);
}

long orc3_time(const orc3_sim* s) { return s->t; }

static double* hist_row(orc3_sim* s, long t) {
    const long row = (long)(s->ns + 1) * 12;
    if (t >= s->hist_cap) {
        long cap = s->hist_cap ? 2 * s->hist_cap : 64;
        while (cap <= t) cap *= 2;
        s->hist = (double*)realloc(s->hist, sizeof(double) * (size_t)(cap * row));
        s->hist_cap = cap;
    }
    return s->hist + t * row;
}

/* Refill of newborn node (x, y, z) from post-advection values fn
 * [19][nz][ny][nx]: the average over participating directions k (x + e_k old
 * fluid: fluid in own_t and own_n) of A1/A2/A3 along k, the scheme falling
 * back A1 -> A2 -> A3 where x + 2e_k or x + 3e_k is not old fluid.  *np
 * receives the participant count (out is untouched when it is zero). */
void orc3_refill_node(int nx, int ny, int nz, const double* fn, const unsigned char* own_t,
                      const unsigned char* own_n, int x, int y, int z, int scheme0, int* np_out, double out[19]) {
    const long N = (long)nx * ny * nz;
    double acc[19] = {0.0};
    int np = 0;
    for (int k = 1; k < 19; ++k) {
        long q[4] = {0, 0, 0, 0};
        int old[4] = {0, 0, 0, 0};
        for (int m = 1; m <= 3; ++m) {
            q[m] = ((long)wrap(z + m * E[k][2], nz) * ny + wrap(y + m * E[k][1], ny)) * nx + wrap(x + m * E[k][0], nx);
            old[m] = own_t[q[m]] == 0 && own_n[q[m]] == 0;
            if (!old[m]) break;
        }
        if (!old[1]) continue;
        int scheme = scheme0;
        if (scheme == ORC3_A1 && !(old[2] && old[3])) scheme = ORC3_A2;
        if (scheme == ORC3_A2 && !old[2]) scheme = ORC3_A3;
        ++np;
        for (int j = 0; j < 19; ++j) {
            const double f1 = fn[(long)j * N + q[1]];
            double v = f1;
            if (scheme == ORC3_A2) v = 2.0 * f1 - fn[(long)j * N + q[2]];
            if (scheme == ORC3_A1) v = 3.0 * f1 - 3.0 * fn[(long)j * N + q[2]] + fn[(long)j * N + q[3]];
            acc[j] += v;
        }
    }
    *np_out = np;
    if (np > 0)
        for (int j = 0; j < 19; ++j) out[j] = acc[j] / np;
}

static void one_step(orc3_sim* s) {
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    /* collide */
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (s->own[nidx(s, x, y, z)] != 0) continue;
                double fl[19], out[19];
                for (int i = 0; i < 19; ++i) fl[i] = s->f[pidx(s, i, x, y, z)];
                orc3_collide_node(fl, s->tau, s->g, out);
                for (int i = 0; i < 19; ++i) s->ft[pidx(s, i, x, y, z)] = out[i];
            }
    /* pressure inlet and outlet (non-equilibrium extrapolation): the
     * post-collision populations of the planes x = 0 and x = nx - 1 become
     * f_eq(rho_b, u) + (f~ - f_eq(rho, u)) of the fluid node next to them,
     * rho and u its density and momentum over density */
    if (s->pressure)
        for (int side = 0; side < 2; ++side) {
            const int xb = side == 0 ? 0 : nx - 1, xf = side == 0 ? 1 : nx - 2;
            const double rb = side == 0 ? s->rho_in : s->rho_out;
            for (int z = 0; z < nz; ++z)
                for (int y = 0; y < ny; ++y) {
                    if (s->own[nidx(s, xb, y, z)] != 0 || s->own[nidx(s, xf, y, z)] != 0) continue;
                    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
                    for (int i = 0; i < 19; ++i) {
                        const double fi = s->ft[pidx(s, i, xf, y, z)];
                        r += fi;
                        for (int d = 0; d < 3; ++d) j[d] += E[i][d] * fi;
                    }
                    const double u[3] = {j[0] / r, j[1] / r, j[2] / r};
                    double eb[19], ef[19];
                    orc3_feq(rb, u, eb);
                    orc3_feq(r, u, ef);
                    for (int i = 0; i < 19; ++i) s->ft[pidx(s, i, xb, y, z)] = eb[i] + (s->ft[pidx(s, i, xf, y, z)] - ef[i]);
                }
        }
    /* forces on every fluid-solid link */
    double* h = hist_row(s, s->t);
    memset(h, 0, sizeof(double) * (size_t)(s->ns + 1) * 12);
    s->rec_n = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (s->own[nidx(s, x, y, z)] != 0) continue;
                for (int i = 1; i < 19; ++i) {
                    int xb = wrap(x + E[i][0], nx), yb = wrap(y + E[i][1], ny), zb = wrap(z + E[i][2], nz);
                    int o = s->own[nidx(s, xb, yb, zb)];
                    if (o == 0) continue;
                    /* surface point x_f + q e_i: q = 1/2 (half-way), or the link
                     * fraction into a sphere under interpolated bounce-back */
                    const double q = link_q3(s, o, s->t, x, y, z, E[i]);
                    double v[3], r[3];
                    surface_velocity(s, o, s->t, x + q * E[i][0], y + q * E[i][1], z + q * E[i][2], v, r);
                    double a = s->ft[pidx(s, i, x, y, z)];
                    const double m = 6.0 * weight(i) * s->rho0 * (E[i][0] * v[0] + E[i][1] * v[1] + E[i][2] * v[2]);
                    double b = a - m;
                    if (q < 0.5) {
                        const int xq = wrap(x - E[i][0], nx), yq = wrap(y - E[i][1], ny), zq = wrap(z - E[i][2], nz);
                        if (s->own[nidx(s, xq, yq, zq)] == 0)
                            b = 2.0 * q * a + (1.0 - 2.0 * q) * s->ft[pidx(s, i, xq, yq, zq)] - m;
                    } else if (q > 0.5) {
                        b = a / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * s->ft[pidx(s, opposite(i), x, y, z)] -
                            m / (2.0 * q);
                    }
                    double* hs = h + 12 * (o == 255 ? 0 : o);
                    double* rr = NULL;
                    if (s->rec && s->rec_n < s->rec_cap) {
                        rr = s->rec + 11 * s->rec_n++;
                        rr[0] = x;
                        rr[1] = y;
                        rr[2] = z;
                        rr[3] = i;
                        rr[4] = o == 255 ? 0 : o;
                    }
                    for (int sch = 0; sch < 2; ++sch) {
                        double F[3];
                        orc3_link_force(i, a, b, v, sch, F);
                        if (rr)
                            for (int d = 0; d < 3; ++d) rr[5 + 3 * sch + d] = F[d];
                        double* hh = hs + 6 * sch;
                        for (int d = 0; d < 3; ++d) hh[d] += F[d];
                        if (o != 255) {
                            hh[3] += r[1] * F[2] - r[2] * F[1];
                            hh[4] += r[2] * F[0] - r[0] * F[2];
                            hh[5] += r[0] * F[1] - r[1] * F[0];
                        }
                    }
                }
            }
    /* advect with half-way bounce-back */
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (s->own[nidx(s, x, y, z)] != 0) continue;
                for (int i = 0; i < 19; ++i) {
                    int xs = wrap(x - E[i][0], nx), ys = wrap(y - E[i][1], ny), zs = wrap(z - E[i][2], nz);
                    int o = s->own[nidx(s, xs, ys, zs)];
                    double val;
                    if (o == 0) {
                        val = s->ft[pidx(s, i, xs, ys, zs)];
                    } else {
                        int me[3] = {-E[i][0], -E[i][1], -E[i][2]};
                        const double q = link_q3(s, o, s->t, x, y, z, me);
                        double v[3], r[3];
                        surface_velocity(s, o, s->t, x - q * E[i][0], y - q * E[i][1], z - q * E[i][2], v, r);
                        const double m = 6.0 * weight(i) * s->rho0 * (E[i][0] * v[0] + E[i][1] * v[1] + E[i][2] * v[2]);
                        const double fo = s->ft[pidx(s, opposite(i), x, y, z)];
                        val = fo + m;
                        if (q < 0.5) {
                            const int xq = wrap(x + E[i][0], nx), yq = wrap(y + E[i][1], ny), zq = wrap(z + E[i][2], nz);
                            if (s->own[nidx(s, xq, yq, zq)] == 0)
                                val = 2.0 * q * fo + (1.0 - 2.0 * q) * s->ft[pidx(s, opposite(i), xq, yq, zq)] + m;
                        } else if (q > 0.5) {
                            val = fo / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * s->ft[pidx(s, i, x, y, z)] +
                                  m / (2.0 * q);
                        }
                    }
                    s->fn[pidx(s, i, x, y, z)] = val;
                }
            }
    /* free spheres: Newton-Euler step from this step's force and torque */
    for (int k = 0; k < s->ns; ++k) {
        if (!s->free_[k]) continue;
        const double* hk = h + 12 * (k + 1) + 6 * s->dyn_scheme;
        double havg[6];
        if (s->force_avg && s->t >= 1) {
            const double* hp = s->hist + ((s->t - 1) * (s->ns + 1) + (k + 1)) * 12 + 6 * s->dyn_scheme;
            for (int q = 0; q < 6; ++q) havg[q] = 0.5 * (hk[q] + hp[q]);
            hk = havg;
        }
        double* D = s->dyn + 18 * k;
        const double M = s->mass[3 * k], I = s->mass[3 * k + 1], Vol = s->mass[3 * k + 2];
        const double ext = M - s->rho0 * Vol;
        for (int d = 0; d < 3; ++d) {
            D[12 + d] = D[3 + d] + (hk[d] + ext * s->G[d]) / M;
            D[15 + d] = D[6 + d] + hk[3 + d] / I;
            D[9 + d] = D[d] + D[12 + d];
        }
    }
    s->advanced = 1;
    /* moving spheres: geometry of step t + 1, newborn refill */
    int any_moving = 0;
    for (int k = 0; k < s->ns; ++k) any_moving |= s->moving[k];
    if (any_moving) {
        int overlap = 0;
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    s->own_n[nidx(s, x, y, z)] = (unsigned char)classify(s, x, y, z, s->t + 1, &overlap);
        if (overlap) s->err = 1;
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const long n = nidx(s, x, y, z);
                    if (s->own[n] == 0 || s->own_n[n] != 0) continue; /* not newborn */
                    double acc[19];
                    int np = 0;
                    orc3_refill_node(nx, ny, nz, s->fn, s->own, s->own_n, x, y, z, s->refill, &np, acc);
                    double out[19];
                    if (np > 0) {
                        for (int j = 0; j < 19; ++j) out[j] = acc[j];
                    } else {
                        double v[3], r[3];
                        surface_velocity(s, s->own[n], s->t + 1, x, y, z, v, r);
                        orc3_feq(s->rho0, v, out);
                    }
                    for (int j = 0; j < 19; ++j) s->fn[pidx(s, j, x, y, z)] = out[j];
                }
        unsigned char* t2 = s->own;
        s->own = s->own_n;
        s->own_n = t2;
    }
    for (int k = 0; k < s->ns; ++k)
        if (s->free_[k])
            for (int d = 0; d < 9; ++d) s->dyn[18 * k + d] = s->dyn[18 * k + 9 + d];
    s->advanced = 0;
    double* tmp = s->f;
    s->f = s->fn;
    s->fn = tmp;
    s->t += 1;
}

int orc3_set_free(orc3_sim* s, int sphere, double rho_s, const double omega0[3]) {
    if (sphere < 1 || sphere > s->ns || !(rho_s > 0.0) || s->t != 0 || !s->moving[sphere - 1]) return -1;
    const int k = sphere - 1;
    const double* p = s->sp + 10 * k;
    const double r = p[3];
    const double vol = 4.0 / 3.0 * M_PI * r * r * r;
    s->free_[k] = 1;
    s->mass[3 * k] = rho_s * vol;
    s->mass[3 * k + 1] = 0.4 * rho_s * vol * r * r;
    s->mass[3 * k + 2] = vol;
    for (int d = 0; d < 3; ++d) {
        s->dyn[18 * k + d] = p[d];
        s->dyn[18 * k + 3 + d] = p[4 + d];
        s->dyn[18 * k + 6 + d] = omega0[d];
    }
    return 0;
}

void orc3_set_force_average(orc3_sim* s, int on) { s->force_avg = on ? 1 : 0; }

int orc3_set_pressure(orc3_sim* s, double rho_in, double rho_out) {
    for (int k = 0; k < s->ns; ++k)
        if (s->moving[k]) return -1;
    if (!(rho_in > 0.0) || !(rho_out > 0.0) || s->t != 0) return -1;
    s->pressure = 1;
    s->rho_in = rho_in;
    s->rho_out = rho_out;
    return 0;
}

void orc3_set_gravity(orc3_sim* s, const double G[3], int scheme) {
    for (int d = 0; d < 3; ++d) s->G[d] = G[d];
    s->dyn_scheme = scheme == ORC3_CME ? ORC3_CME : ORC3_GME;
}

int orc3_body_state(const orc3_sim* s, int sphere, double out[9]) {
    if (sphere < 1 || sphere > s->ns) return -1;
    double X[3], V[3], Om[3];
    centre(s, sphere - 1, s->t, X);
    motion(s, sphere - 1, s->t, V, Om);
    for (int d = 0; d < 3; ++d) {
        out[d] = X[d];
        out[3 + d] = V[d];
        out[6 + d] = Om[d];
    }
    return 0;
}

int orc3_set_moving(orc3_sim* s, int sphere, int moving, int refill) {
    if (sphere < 1 || sphere > s->ns || refill < ORC3_A1 || refill > ORC3_A3 || s->t != 0) return -1;
    s->moving[sphere - 1] = moving ? 1 : 0;
    s->refill = refill;
    return 0;
}

int orc3_error(const orc3_sim* s) { return s->err; }

void orc3_step(orc3_sim* s, long n) {
    for (long k = 0; k < n; ++k) one_step(s);
}

void orc3_fields(const orc3_sim* s, double* rho, double* u, int* owner) {
    const long N = (long)s->nx * s->ny * s->nz;
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long n = nidx(s, x, y, z);
                int o = s->own[n];
                double r = 0.0, j[3] = {0.0, 0.0, 0.0};
                if (o == 0)
                    for (int i = 0; i < 19; ++i) {
                        double fi = s->f[pidx(s, i, x, y, z)];
                        r += fi;
                        for (int d = 0; d < 3; ++d) j[d] += E[i][d] * fi;
                    }
                if (rho) rho[n] = r;
                if (u)
                    for (int d = 0; d < 3; ++d) u[d * N + n] = o == 0 ? (j[d] + 0.5 * r * s->g[d]) / r : 0.0;
                if (owner) owner[n] = o;
            }
}

int orc3_force(const orc3_sim* s, long step, int solid, int scheme, double out[6]) {
    if (step < 0 || step >= s->t || solid < 0 || solid > s->ns) return -1;
    const double* h = s->hist + (step * (s->ns + 1) + solid) * 12 + 6 * (scheme == ORC3_CME ? 0 : 1);
    for (int d = 0; d < 6; ++d) out[d] = h[d];
    return 0;
}

void orc3_get_f(const orc3_sim* s, double* out) {
    memcpy(out, s->f, sizeof(double) * 19 * (size_t)s->nx * s->ny * s->nz);
}

void orc3_get_ft(const orc3_sim* s, double* out) {
    memcpy(out, s->ft, sizeof(double) * 19 * (size_t)s->nx * s->ny * s->nz);
}

void orc3_set_f(orc3_sim* s, const double* in) {
    memcpy(s->f, in, sizeof(double) * 19 * (size_t)s->nx * s->ny * s->nz);
}

/* Keep the per-link records of each step (up to cap links) from now on. */
void orc3_record_links(orc3_sim* s, long cap) {
    free(s->rec);
    s->rec = cap > 0 ? (double*)calloc((size_t)cap * 11, sizeof(double)) : NULL;
    s->rec_cap = cap > 0 ? cap : 0;
    s->rec_n = 0;
}

/* Link records of the last step, 11 doubles each: x, y, z, i, solid (0 the
 * duct), CME force (3), GME force (3); returns the count copied. */
long orc3_links(const orc3_sim* s, double* out, long max) {
    const long n = s->rec_n < max ? s->rec_n : max;
    if (n > 0) memcpy(out, s->rec, sizeof(double) * 11 * (size_t)n);
    return n;
}
