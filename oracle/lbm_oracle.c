/*
 * lbm_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see the
 * header).  Every loop is a direct statement of the method; nothing is
 * blocked, fused or reordered for speed.  Build with -ffp-contract=off so that
 * no multiply-add is fused: the solid/fluid decision of the rasterisation must
 * be taken with separately rounded products and sums.
 *
 * One time step t -> t+1 on geometry G_t (Sec. II, Sec. III.A-B, Sec. IV.B):
 *   O1 moments       rho = sum f_i, rho*u = sum e_i f_i + rho*g/2
 *   O2 collision     Eq. 2 with the single-relaxation-time (BGK) operator,
 *                    Eq. 8 equilibrium and Guo's forcing term; or, after
 *                    orc_set_mrt, the multiple-relaxation-time operator of
 *                    Sec. IV (relaxation in moment space with the diagonal
 *                    matrix S) with the same equilibrium and forcing
 *   O3 link forces   Eq. 4 (CME) and Eq. 5 (GME) on every fluid-solid link,
 *                    summed per solid (Eq. 6) with torque (Eq. 7)
 *   O4 advection     Eq. 3; a population whose source node is solid is the
 *                    half-way bounce-back of the node's own opposite population
 *                    plus the moving-boundary term 6 w_i rho_w (e_i . v); or,
 *                    after orc_set_ibb, on body links the interpolated
 *                    bounce-back of Sec. IV (linear in the fraction q of the
 *                    link at which the surface lies)
 *   O5 move bodies   positions at t+1 (prescribed, or for free bodies the
 *                    Newton-Euler update from the step's force and torque),
 *                    rasterise G_{t+1}
 *   O6 covered nodes populations dropped
 *   O7 newborn nodes refilled by extrapolation along the participating links
 *                    (A1 second order, A2 linear, A3 neighbour value), averaged
 *   O8 t <- t+1
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9 velocity set in the order given in Sec. III.C. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* ibar: the direction opposite to i. */
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* Weights of Eq. 8 (the D2Q9 set; Eq. 10 reproduces the pressure rho/3 only
 * with these). */
static const double W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

struct orc_sim {
    int nx, ny, walls_y;
    double tau, rho0, gx, gy;
    double wall_vx, wall_vy;
    int refill, rho_w_local;
    int mrt;         /* 0: BGK; 1: MRT with rates s_rate */
    double s_rate[9];
    /* free bodies (Sec. IV): state at step t and the centre at t+1 */
    struct orc_dyn {
        int free_;
        double X, Y, Vx, Vy, Om;   /* centre, velocity, angular velocity at t */
        double Xn, Yn;             /* centre at t+1 (O5) */
        double M, I, A;            /* mass, moment of inertia, area */
    } * dyn;
    double Gx, Gy;   /* gravity acting on free bodies (buoyancy-corrected) */
    int ibb;         /* interpolated bounce-back on body links */
    int dyn_scheme;  /* ORC_CME or ORC_GME force drives them */
    int nb;
    orc_body* body;
    long t;
    double* f;       /* pre-collision f(t), [9][ny][nx] */
    double* ft;      /* post-collision f~(t) */
    double* fn;      /* post-advection f(t+1) */
    int* own;        /* owner map of G_t: 0 fluid, s > 0 body s */
    int* own_next;   /* owner map of G_{t+1} */
    int* oldfluid;   /* fluid in both G_t and G_{t+1} */
    /* force history: [step][nb+1][6] = CME {Fx, Fy, Tz}, GME {Fx, Fy, Tz} */
    long hist_len, hist_cap;
    double* hist;
    /* per-link records of the last step */
    long nlink, link_cap;
    double* link;
};

static long idx(const orc_sim* s, int x, int y) { return (long)y * s->nx + x; }
static long pidx(const orc_sim* s, int i, int x, int y) {
    return ((long)i * s->ny + y) * s->nx + x;
}

static int wrap(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

/* Position of body b at step t. */
static void body_pos(const orc_body* b, long t, double* X, double* Y) {
    if (b->moves) {
        *X = b->cx + (double)t * b->vx;
        *Y = b->cy + (double)t * b->vy;
    } else {
        *X = b->cx;
        *Y = b->cy;
    }
}

/* Whether the point with integer coordinates (x, y) lies inside body b
 * centred at (X, Y).  Disc: dx*dx + dy*dy <= r*r.  Box: |dx| <= a, |dy| <= b. */
static int inside(const orc_body* b, double X, double Y, long x, long y) {
    double dx = (double)x - X;
    double dy = (double)y - Y;
    if (b->kind == ORC_DISC) {
        double d2 = dx * dx;
        d2 = d2 + dy * dy;
        return d2 <= b->a * b->a;
    }
    return fabs(dx) <= b->a && fabs(dy) <= b->b;
}

/* Centre of body k at step t (t = s->t or s->t + 1 for a free body). */
static void body_center(const orc_sim* s, int k, long t, double* X, double* Y) {
    const struct orc_dyn* d = &s->dyn[k];
    if (d->free_) {
        *X = t == s->t ? d->X : d->Xn;
        *Y = t == s->t ? d->Y : d->Yn;
    } else {
        body_pos(&s->body[k], t, X, Y);
    }
}

static double min_image(double d, int n);

/* Velocity of body k's surface at the point (px, py) at step t: V + Omega
 * z x (p - X), minimum image; a prescribed body translates rigidly. */
static void wall_velocity(const orc_sim* s, int k, double px, double py, double* vx, double* vy) {
    const struct orc_dyn* d = &s->dyn[k];
    if (!d->free_) {
        *vx = s->body[k].vx;
        *vy = s->body[k].vy;
        return;
    }
    double rx = min_image(px - d->X, s->nx);
    double ry = s->walls_y ? (py - d->Y) : min_image(py - d->Y, s->ny);
    *vx = d->Vx - d->Om * ry;
    *vy = d->Vy + d->Om * rx;
}

/* Fraction q in (0, 1] of the link from the fluid node (x, y) to (x, y) +
 * (ex, ey) at which the surface of body k, centred at (X, Y), is crossed
 * (the far end is inside the body, the near end outside).  Disc: the smaller
 * root of |P + q e|^2 = r^2; box: the entry parameter of the ray into the
 * slabs |dx| <= a, |dy| <= b.  Minimum image on periodic axes. */
static double link_q_at(const orc_sim* s, int k, double X, double Y, long x, long y, int ex, int ey) {
    const orc_body* b = &s->body[k];
    double px = min_image((double)x - X, s->nx);
    double py = s->walls_y ? ((double)y - Y) : min_image((double)y - Y, s->ny);
    double q;
    if (b->kind == ORC_DISC) {
        double a2 = (double)(ex * ex + ey * ey);
        double b2 = 2.0 * (px * ex + py * ey);
        double c2 = px * px + py * py - b->a * b->a;
        double disc = b2 * b2 - 4.0 * a2 * c2;
        if (disc < 0.0) disc = 0.0;
        q = (-b2 - sqrt(disc)) / (2.0 * a2);
    } else {
        double lo = -1e300;
        const double p[2] = {px, py}, h[2] = {b->a, b->b};
        const int e[2] = {ex, ey};
        for (int d = 0; d < 2; ++d) {
            if (e[d] == 0) continue;
            double t1 = (-h[d] - p[d]) / e[d], t2 = (h[d] - p[d]) / e[d];
            double tmin = t1 < t2 ? t1 : t2;
            if (tmin > lo) lo = tmin;
        }
        q = lo;
    }
    if (q <= 0.0) q = 1e-12;
    if (q > 1.0) q = 1.0;
    return q;
}

/* Rasterise all bodies at step t into own (0 = fluid).  Every integer point
 * of each body's bounding range is tested and mapped to its periodic image. */
static void rasterise(const orc_sim* s, long t, int* own) {
    memset(own, 0, sizeof(int) * (size_t)s->nx * (size_t)s->ny);
    for (int k = 0; k < s->nb; ++k) {
        const orc_body* b = &s->body[k];
        double X, Y;
        body_center(s, k, t, &X, &Y);
        double hx = b->a;
        double hy = (b->kind == ORC_DISC) ? b->a : b->b;
        long x0 = (long)floor(X - hx) - 1, x1 = (long)ceil(X + hx) + 1;
        long y0 = (long)floor(Y - hy) - 1, y1 = (long)ceil(Y + hy) + 1;
        for (long y = y0; y <= y1; ++y) {
            for (long x = x0; x <= x1; ++x) {
                if (!inside(b, X, Y, x, y)) continue;
                int xi = wrap((int)x, s->nx);
                int yi;
                if (s->walls_y) {
                    if (y < 0 || y >= s->ny) continue; /* validated never to happen */
                    yi = (int)y;
                } else {
                    yi = wrap((int)y, s->ny);
                }
                own[idx(s, xi, yi)] = k + 1;
            }
        }
    }
}

/* Neighbour of (x, y) in direction +e_i (sign = +1) or -e_i (sign = -1).
 * Returns 0 and the wrapped node, or 1 if it is a virtual wall node. */
static int neighbour(const orc_sim* s, int x, int y, int i, int sign, int* xo, int* yo) {
    int xn = x + sign * EX[i];
    int yn = y + sign * EY[i];
    *xo = wrap(xn, s->nx);
    if (s->walls_y) {
        if (yn < 0 || yn >= s->ny) return 1;
        *yo = yn;
    } else {
        *yo = wrap(yn, s->ny);
    }
    return 0;
}

void orc_feq(double rho, double ux, double uy, double out[9]) {
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double eu = EX[i] * ux + EY[i] * uy;
        out[i] = rho * W[i] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

/* O1 + O2 for one node. */
void orc_collide_node(const double f[9], double tau, double gx, double gy, double out[9]) {
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) {
        rho += f[i];
        jx += EX[i] * f[i];
        jy += EY[i] * f[i];
    }
    /* Guo et al.: the velocity includes half the body force. */
    double ux = (jx + 0.5 * rho * gx) / rho;
    double uy = (jy + 0.5 * rho * gy) / rho;
    double feq[9];
    orc_feq(rho, ux, uy, feq);
    double pref = 1.0 - 1.0 / (2.0 * tau);
    for (int i = 0; i < 9; ++i) {
        double eu = EX[i] * ux + EY[i] * uy;
        double sx = 3.0 * (EX[i] - ux) + 9.0 * eu * EX[i];
        double sy = 3.0 * (EY[i] - uy) + 9.0 * eu * EY[i];
        double src = pref * W[i] * (sx * rho * gx + sy * rho * gy);
        out[i] = f[i] - (f[i] - feq[i]) / tau + src;
    }
}

/* Moment basis of the D2Q9 multiple-relaxation-time model (Lallemand and
 * Luo): rows rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy over the velocities
 * of Sec. III.C. */
static const double MRT_M[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

/* Inverse of MRT_M by Gauss-Jordan elimination with partial pivoting. */
void orc_mrt_inverse(double inv[81]) {
    double a[9][18];
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 18; ++c) a[r][c] = c < 9 ? MRT_M[r][c] : (c - 9 == r ? 1.0 : 0.0);
    for (int c = 0; c < 9; ++c) {
        int piv = c;
        for (int r = c + 1; r < 9; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        for (int k = 0; k < 18; ++k) {
            double tmp = a[c][k];
            a[c][k] = a[piv][k];
            a[piv][k] = tmp;
        }
        double d = a[c][c];
        for (int k = 0; k < 18; ++k) a[c][k] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == c) continue;
            double m = a[r][c];
            for (int k = 0; k < 18; ++k) a[r][k] -= m * a[c][k];
        }
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) inv[r * 9 + c] = a[r][9 + c];
}

void orc_mrt_matrix(double out[81]) {
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) out[r * 9 + c] = MRT_M[r][c];
}

/* O1 + O2 with the MRT operator: m = M f, m* = m - S (m - M f_eq)
 * + (I - S/2) M F, f* = M^-1 m*, where F_i = w_i [3 (e_i - u) + 9 (e_i.u) e_i]
 * . rho g is Guo's forcing term without its BGK prefactor (the prefactor
 * becomes I - S/2 in moment space) and s[k] is the rate of moment k. */
void orc_collide_node_mrt(const double f[9], const double s[9], double gx, double gy, double out[9]) {
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) {
        rho += f[i];
        jx += EX[i] * f[i];
        jy += EY[i] * f[i];
    }
    double ux = (jx + 0.5 * rho * gx) / rho;
    double uy = (jy + 0.5 * rho * gy) / rho;
    double feq[9], F[9];
    orc_feq(rho, ux, uy, feq);
    for (int i = 0; i < 9; ++i) {
        double eu = EX[i] * ux + EY[i] * uy;
        double sx = 3.0 * (EX[i] - ux) + 9.0 * eu * EX[i];
        double sy = 3.0 * (EY[i] - uy) + 9.0 * eu * EY[i];
        F[i] = W[i] * (sx * rho * gx + sy * rho * gy);
    }
    double m[9], meq[9], mF[9], ms[9];
    for (int k = 0; k < 9; ++k) {
        m[k] = meq[k] = mF[k] = 0.0;
        for (int i = 0; i < 9; ++i) {
            m[k] += MRT_M[k][i] * f[i];
            meq[k] += MRT_M[k][i] * feq[i];
            mF[k] += MRT_M[k][i] * F[i];
        }
        ms[k] = m[k] - s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * s[k]) * mF[k];
    }
    double inv[81];
    orc_mrt_inverse(inv);
    for (int i = 0; i < 9; ++i) {
        out[i] = 0.0;
        for (int k = 0; k < 9; ++k) out[i] += inv[i * 9 + k] * ms[k];
    }
}

void orc_set_mrt(orc_sim* sim, double s_e, double s_eps, double s_q) {
    /* Sec. IV: S = diag(0, s_e, s_eps, 0, s_q, 0, s_q, 1/tau, 1/tau) */
    const double nu = 1.0 / sim->tau;
    const double r[9] = {0.0, s_e, s_eps, 0.0, s_q, 0.0, s_q, nu, nu};
    for (int k = 0; k < 9; ++k) sim->s_rate[k] = r[k];
    sim->mrt = 1;
}

void orc_link_force(int i, double a, double b, double vx, double vy, int scheme, double out[2]) {
    int ib = OPP[i];
    if (scheme == ORC_CME) {
        /* Eq. 4: e_i f~_i(x_f) - e_ibar f~_ibar(x_b) */
        out[0] = EX[i] * a - EX[ib] * b;
        out[1] = EY[i] * a - EY[ib] * b;
    } else {
        /* Eq. 5: (e_i - v) f~_i(x_f) - (e_ibar - v) f~_ibar(x_b) */
        out[0] = (EX[i] - vx) * a - (EX[ib] - vx) * b;
        out[1] = (EY[i] - vy) * a - (EY[ib] - vy) * b;
    }
}

int orc_refill_node(int nx, int ny, int walls_y, const double* fpost, const int* oldfluid,
                    int x, int y, int scheme, double rho0, double vx, double vy, double out[9]) {
    double acc[9] = {0};
    int npart = 0;
    for (int k = 1; k < 9; ++k) {
        /* node positions x + m e_k, m = 1, 2, 3; ok[m] = old-fluid there */
        int ok[4] = {0, 0, 0, 0};
        long at[4] = {0, 0, 0, 0};
        for (int m = 1; m <= 3; ++m) {
            int xm = x + m * EX[k], ym = y + m * EY[k];
            if (walls_y && (ym < 0 || ym >= ny)) break;
            xm = wrap(xm, nx);
            ym = wrap(ym, ny);
            at[m] = (long)ym * nx + xm;
            ok[m] = oldfluid[at[m]] != 0;
            if (!ok[m]) break;
        }
        if (!ok[1]) continue; /* direction k does not participate */
        npart++;
        int use = scheme;
        if (use == ORC_A1 && !(ok[2] && ok[3])) use = ORC_A2;
        if (use == ORC_A2 && !ok[2]) use = ORC_A3;
        for (int j = 0; j < 9; ++j) {
            long plane = (long)j * nx * ny;
            double v1 = fpost[plane + at[1]];
            double val;
            if (use == ORC_A1) {
                /* quadratic through m = 1, 2, 3 evaluated at m = 0 */
                double v2 = fpost[plane + at[2]], v3 = fpost[plane + at[3]];
                val = 3.0 * v1 - 3.0 * v2 + v3;
            } else if (use == ORC_A2) {
                /* line through m = 1, 2 evaluated at m = 0 */
                double v2 = fpost[plane + at[2]];
                val = 2.0 * v1 - v2;
            } else {
                val = v1;
            }
            acc[j] += val;
        }
    }
    if (npart == 0) {
        orc_feq(rho0, vx, vy, out);
        return 0;
    }
    for (int j = 0; j < 9; ++j) out[j] = acc[j] / npart;
    return npart;
}

orc_sim* orc_create(int nx, int ny, int walls_y, double tau, double rho0, double gx, double gy,
                    double u0x, double u0y, double wall_vx, double wall_vy, int refill,
                    int rho_w_local, int n_bodies, const orc_body* bodies) {
    if (nx < 1 || ny < 1 || !(tau > 0.5) || refill < 0 || refill > 2 || n_bodies < 0) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->nx = nx;
    s->ny = ny;
    s->walls_y = walls_y ? 1 : 0;
    s->tau = tau;
    s->rho0 = rho0;
    s->gx = gx;
    s->gy = gy;
    s->wall_vx = wall_vx;
    s->wall_vy = wall_vy;
    s->refill = refill;
    s->rho_w_local = rho_w_local ? 1 : 0;
    s->nb = n_bodies;
    s->body = (orc_body*)calloc((size_t)(n_bodies > 0 ? n_bodies : 1), sizeof(orc_body));
    for (int k = 0; k < n_bodies; ++k) s->body[k] = bodies[k];
    s->dyn = (struct orc_dyn*)calloc((size_t)(n_bodies > 0 ? n_bodies : 1), sizeof(struct orc_dyn));
    size_t n = (size_t)nx * (size_t)ny;
    s->f = (double*)calloc(9 * n, sizeof(double));
    s->ft = (double*)calloc(9 * n, sizeof(double));
    s->fn = (double*)calloc(9 * n, sizeof(double));
    s->own = (int*)calloc(n, sizeof(int));
    s->own_next = (int*)calloc(n, sizeof(int));
    s->oldfluid = (int*)calloc(n, sizeof(int));
    s->t = 0;
    rasterise(s, 0, s->own);
    double feq[9];
    orc_feq(rho0, u0x, u0y, feq);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            if (s->own[idx(s, x, y)] == 0)
                for (int i = 0; i < 9; ++i) s->f[pidx(s, i, x, y)] = feq[i];
    return s;
}

int orc_set_free(orc_sim* s, int body, double rho_s, double omega0) {
    if (body < 1 || body > s->nb || s->t != 0 || !(rho_s > 0.0)) return -1;
    const orc_body* b = &s->body[body - 1];
    if (b->kind != ORC_DISC) return -1;
    struct orc_dyn* d = &s->dyn[body - 1];
    const double pi = 3.14159265358979323846;
    d->free_ = 1;
    d->X = b->cx;
    d->Y = b->cy;
    d->Vx = b->vx;
    d->Vy = b->vy;
    d->Om = omega0;
    d->A = pi * b->a * b->a;
    d->M = rho_s * d->A;
    d->I = 0.5 * d->M * b->a * b->a;
    return 0;
}

void orc_set_ibb(orc_sim* s, int on) { s->ibb = on ? 1 : 0; }

double orc_link_q(const orc_sim* s, int body, long x, long y, int i) {
    if (body < 1 || body > s->nb || i < 1 || i > 8) return -1.0;
    double X, Y;
    body_center(s, body - 1, s->t, &X, &Y);
    return link_q_at(s, body - 1, X, Y, x, y, EX[i], EY[i]);
}

void orc_set_gravity(orc_sim* s, double Gx, double Gy, int scheme) {
    s->Gx = Gx;
    s->Gy = Gy;
    s->dyn_scheme = scheme == ORC_GME ? ORC_GME : ORC_CME;
}

int orc_body_state(const orc_sim* s, int body, double out[5]) {
    if (body < 1 || body > s->nb) return -1;
    double X, Y;
    body_center(s, body - 1, s->t, &X, &Y);
    const struct orc_dyn* d = &s->dyn[body - 1];
    out[0] = X;
    out[1] = Y;
    out[2] = d->free_ ? d->Vx : s->body[body - 1].vx;
    out[3] = d->free_ ? d->Vy : s->body[body - 1].vy;
    out[4] = d->free_ ? d->Om : 0.0;
    return 0;
}

void orc_destroy(orc_sim* s) {
    if (!s) return;
    free(s->dyn);
    free(s->body);
    free(s->f);
    free(s->ft);
    free(s->fn);
    free(s->own);
    free(s->own_next);
    free(s->oldfluid);
    free(s->hist);
    free(s->link);
    free(s);
}

long orc_time(const orc_sim* s) { return s->t; }

static double* hist_row(orc_sim* s, long step) {
    if (step >= s->hist_cap) {
        long cap = s->hist_cap ? s->hist_cap * 2 : 1024;
        while (cap <= step) cap *= 2;
        s->hist = (double*)realloc(s->hist, sizeof(double) * (size_t)cap * (size_t)(s->nb + 1) * 6);
        s->hist_cap = cap;
    }
    return s->hist + (size_t)step * (size_t)(s->nb + 1) * 6;
}

static void push_link(orc_sim* s, const double rec[8]) {
    if (s->nlink == s->link_cap) {
        s->link_cap = s->link_cap ? s->link_cap * 2 : 4096;
        s->link = (double*)realloc(s->link, sizeof(double) * 8 * (size_t)s->link_cap);
    }
    memcpy(s->link + 8 * s->nlink, rec, 8 * sizeof(double));
    s->nlink++;
}

/* Minimum-image difference of a coordinate on a periodic axis of length n. */
static double min_image(double d, int n) {
    while (d > 0.5 * n) d -= n;
    while (d < -0.5 * n) d += n;
    return d;
}

static void one_step(orc_sim* s) {
    const int nx = s->nx, ny = s->ny;
    const long t = s->t;

    /* O1-O2: collide every fluid node of G_t (nodes are independent: the
     * multi-threaded timing build splits the rows over threads). */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (s->own[idx(s, x, y)] != 0) continue;
            double fl[9], out[9];
            for (int i = 0; i < 9; ++i) fl[i] = s->f[pidx(s, i, x, y)];
            if (s->mrt)
                orc_collide_node_mrt(fl, s->s_rate, s->gx, s->gy, out);
            else
                orc_collide_node(fl, s->tau, s->gx, s->gy, out);
            for (int i = 0; i < 9; ++i) s->ft[pidx(s, i, x, y)] = out[i];
        }

    /* O3: forces on every fluid-solid link of G_t, summed per solid in the
     * order (y, x, i), with torque about the body's centre (Eqs. 4-7). */
    double* h = hist_row(s, t);
    memset(h, 0, sizeof(double) * (size_t)(s->nb + 1) * 6);
    s->nlink = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (s->own[idx(s, x, y)] != 0) continue;
            for (int i = 1; i < 9; ++i) {
                int xb, yb, sid;
                double vx, vy;
                if (neighbour(s, x, y, i, +1, &xb, &yb)) {
                    sid = 0;
                    vx = s->wall_vx;
                    vy = s->wall_vy;
                } else {
                    sid = s->own[idx(s, xb, yb)];
                    if (sid == 0) continue;
                }
                /* the link's surface point: the midpoint for half-way bounce-back,
                 * x_f + q e_i for the interpolated one (body links) */
                double q = 0.5;
                if (sid > 0) {
                    if (s->ibb) {
                        double X, Y;
                        body_center(s, sid - 1, t, &X, &Y);
                        q = link_q_at(s, sid - 1, X, Y, x, y, EX[i], EY[i]);
                    }
                    wall_velocity(s, sid - 1, x + q * EX[i], y + q * EY[i], &vx, &vy);
                }
                double rho_w = s->rho0;
                if (s->rho_w_local) {
                    rho_w = 0.0;
                    for (int j = 0; j < 9; ++j) rho_w += s->ft[pidx(s, j, x, y)];
                }
                double a = s->ft[pidx(s, i, x, y)];
                /* population leaving the boundary node towards x_f: HWBB with
                 * the moving-boundary term, or the interpolated bounce-back
                 * (the value O4 streams into x_f) */
                const double m = 6.0 * W[i] * rho_w * (EX[i] * vx + EY[i] * vy);
                double b = a - m;
                if (q != 0.5) {
                    int xq, yq;
                    if (q < 0.5) {
                        /* needs the fluid node behind x_f */
                        if (!neighbour(s, x, y, i, -1, &xq, &yq) && s->own[idx(s, xq, yq)] == 0)
                            b = 2.0 * q * a + (1.0 - 2.0 * q) * s->ft[pidx(s, i, xq, yq)] - m;
                    } else {
                        b = a / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * s->ft[pidx(s, OPP[i], x, y)] -
                            m / (2.0 * q);
                    }
                }
                double fc[2], fg[2];
                orc_link_force(i, a, b, vx, vy, ORC_CME, fc);
                orc_link_force(i, a, b, vx, vy, ORC_GME, fg);
                double tc = 0.0, tg = 0.0;
                if (sid > 0) {
                    double X, Y;
                    body_center(s, sid - 1, t, &X, &Y);
                    /* intersection point S of the link with the surface */
                    double rx = min_image(x + q * EX[i] - X, nx);
                    double ry = s->walls_y ? (y + q * EY[i] - Y) : min_image(y + q * EY[i] - Y, ny);
                    tc = rx * fc[1] - ry * fc[0];
                    tg = rx * fg[1] - ry * fg[0];
                }
                double* hs = h + 6 * sid;
                hs[0] += fc[0];
                hs[1] += fc[1];
                hs[2] += tc;
                hs[3] += fg[0];
                hs[4] += fg[1];
                hs[5] += tg;
                double rec[8] = {x, y, i, sid, fc[0], fc[1], fg[0], fg[1]};
                push_link(s, rec);
            }
        }
    s->hist_len = t + 1;

    /* O4: advection (Eq. 3) with half-way bounce-back on G_t. */
    memset(s->fn, 0, sizeof(double) * 9 * (size_t)nx * (size_t)ny);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (s->own[idx(s, x, y)] != 0) continue;
            for (int i = 0; i < 9; ++i) {
                int xs, ys, sid;
                double vx, vy;
                if (neighbour(s, x, y, i, -1, &xs, &ys)) {
                    sid = 0;
                    vx = s->wall_vx;
                    vy = s->wall_vy;
                } else {
                    sid = s->own[idx(s, xs, ys)];
                    if (sid == 0) {
                        s->fn[pidx(s, i, x, y)] = s->ft[pidx(s, i, xs, ys)];
                        continue;
                    }
                    double q = 0.5;
                    if (s->ibb) {
                        double X, Y;
                        body_center(s, sid - 1, t, &X, &Y);
                        q = link_q_at(s, sid - 1, X, Y, x, y, -EX[i], -EY[i]);
                    }
                    /* boundary velocity at the surface point x - q e_i */
                    wall_velocity(s, sid - 1, x - q * EX[i], y - q * EY[i], &vx, &vy);
                    if (q != 0.5) {
                        double rho_q = s->rho0;
                        if (s->rho_w_local) {
                            rho_q = 0.0;
                            for (int j = 0; j < 9; ++j) rho_q += s->ft[pidx(s, j, x, y)];
                        }
                        const double m = 6.0 * W[i] * rho_q * (EX[i] * vx + EY[i] * vy);
                        const double fo = s->ft[pidx(s, OPP[i], x, y)];
                        double v = fo + m;  /* half-way when the node behind is not fluid */
                        int xq, yq;
                        if (q < 0.5) {
                            if (!neighbour(s, x, y, i, +1, &xq, &yq) && s->own[idx(s, xq, yq)] == 0)
                                v = 2.0 * q * fo + (1.0 - 2.0 * q) * s->ft[pidx(s, OPP[i], xq, yq)] + m;
                        } else {
                            v = fo / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * s->ft[pidx(s, i, x, y)] +
                                m / (2.0 * q);
                        }
                        s->fn[pidx(s, i, x, y)] = v;
                        continue;
                    }
                }
                double rho_w = s->rho0;
                if (s->rho_w_local) {
                    rho_w = 0.0;
                    for (int j = 0; j < 9; ++j) rho_w += s->ft[pidx(s, j, x, y)];
                }
                s->fn[pidx(s, i, x, y)] =
                    s->ft[pidx(s, OPP[i], x, y)] + 6.0 * W[i] * rho_w * (EX[i] * vx + EY[i] * vy);
            }
        }

    /* O5: move bodies.  A free body: M dV/dt = F + (M - rho0 A) G,
     * I dOmega/dt = T with the step's force and torque of the chosen scheme,
     * explicit: V(t+1) = V(t) + (F + (M - rho0 A) G)/M, Omega(t+1) =
     * Omega(t) + T/I, X(t+1) = X(t) + V(t+1).  Then rasterise G_{t+1}. */
    double *nvx = NULL, *nvy = NULL, *nom = NULL;
    if (s->nb > 0) {
        nvx = (double*)calloc((size_t)s->nb * 3, sizeof(double));
        nvy = nvx + s->nb;
        nom = nvx + 2 * s->nb;
    }
    for (int k = 0; k < s->nb; ++k) {
        struct orc_dyn* d = &s->dyn[k];
        if (!d->free_) continue;
        const double* hk = h + 6 * (k + 1) + 3 * s->dyn_scheme;
        const double ext = d->M - s->rho0 * d->A;
        nvx[k] = d->Vx + (hk[0] + ext * s->Gx) / d->M;
        nvy[k] = d->Vy + (hk[1] + ext * s->Gy) / d->M;
        nom[k] = d->Om + hk[2] / d->I;
        d->Xn = d->X + nvx[k];
        d->Yn = d->Y + nvy[k];
    }
    rasterise(s, t + 1, s->own_next);
    for (long n = 0; n < (long)nx * ny; ++n)
        s->oldfluid[n] = (s->own[n] == 0 && s->own_next[n] == 0);

    /* O6-O7: drop covered nodes, refill newborn nodes from old-fluid
     * neighbours' post-advection values. */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long n = idx(s, x, y);
            if (s->own[n] == 0 && s->own_next[n] != 0) {
                for (int i = 0; i < 9; ++i) s->fn[pidx(s, i, x, y)] = 0.0;
            } else if (s->own[n] != 0 && s->own_next[n] == 0) {
                const int k = s->own[n] - 1;
                const orc_body* b = &s->body[k];
                double vx = b->vx, vy = b->vy;
                if (s->dyn[k].free_) {
                    /* the body's surface velocity at the node at t+1 */
                    double rx = min_image(x - s->dyn[k].Xn, nx);
                    double ry = s->walls_y ? (y - s->dyn[k].Yn) : min_image(y - s->dyn[k].Yn, ny);
                    vx = nvx[k] - nom[k] * ry;
                    vy = nvy[k] + nom[k] * rx;
                }
                double out[9];
                orc_refill_node(nx, ny, s->walls_y, s->fn, s->oldfluid, x, y, s->refill, s->rho0, vx, vy,
                                out);
                for (int i = 0; i < 9; ++i) s->fn[pidx(s, i, x, y)] = out[i];
            }
        }

    /* O8 */
    for (int k = 0; k < s->nb; ++k) {
        struct orc_dyn* d = &s->dyn[k];
        if (!d->free_) continue;
        d->X = d->Xn;
        d->Y = d->Yn;
        d->Vx = nvx[k];
        d->Vy = nvy[k];
        d->Om = nom[k];
    }
    free(nvx);
    double* tmp = s->f;
    s->f = s->fn;
    s->fn = tmp;
    int* to = s->own;
    s->own = s->own_next;
    s->own_next = to;
    s->t = t + 1;
}

void orc_step(orc_sim* s, long n) {
    for (long k = 0; k < n; ++k) one_step(s);
}

void orc_fields(const orc_sim* s, double* rho, double* ux, double* uy, int* owner) {
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            long n = idx(s, x, y);
            double r = 0.0, jx = 0.0, jy = 0.0;
            int o = s->own[n];
            if (o == 0) {
                for (int i = 0; i < 9; ++i) {
                    double fi = s->f[pidx(s, i, x, y)];
                    r += fi;
                    jx += EX[i] * fi;
                    jy += EY[i] * fi;
                }
            }
            if (rho) rho[n] = r;
            if (ux) ux[n] = (o == 0) ? (jx + 0.5 * r * s->gx) / r : 0.0;
            if (uy) uy[n] = (o == 0) ? (jy + 0.5 * r * s->gy) / r : 0.0;
            if (owner) owner[n] = o;
        }
}

int orc_force(const orc_sim* s, long step, int solid, int scheme, double out[3]) {
    if (step < 0 || step >= s->hist_len || solid < 0 || solid > s->nb) return -1;
    const double* h = s->hist + ((size_t)step * (size_t)(s->nb + 1) + (size_t)solid) * 6;
    int off = scheme == ORC_CME ? 0 : 3;
    out[0] = h[off];
    out[1] = h[off + 1];
    out[2] = h[off + 2];
    return 0;
}

long orc_links(const orc_sim* s, long max, double* rec) {
    long n = s->nlink < max ? s->nlink : max;
    if (rec && n > 0) memcpy(rec, s->link, sizeof(double) * 8 * (size_t)n);
    return s->nlink;
}

void orc_get_f(const orc_sim* s, double* f) {
    memcpy(f, s->f, sizeof(double) * 9 * (size_t)s->nx * (size_t)s->ny);
}

void orc_set_f(orc_sim* s, const double* f) {
    memcpy(s->f, f, sizeof(double) * 9 * (size_t)s->nx * (size_t)s->ny);
}

void orc_init_fields(orc_sim* s, const double* rho, const double* ux, const double* uy) {
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            long n = idx(s, x, y);
            double feq[9] = {0};
            if (s->own[n] == 0) orc_feq(rho[n], ux[n] - 0.5 * s->gx, uy[n] - 0.5 * s->gy, feq);
            for (int i = 0; i < 9; ++i) s->f[pidx(s, i, x, y)] = feq[i];
        }
}
