// lbm_device.h -- device-side building blocks of the D2Q9 hot path (gfx950).
//
// Lattice: D2Q9 velocity set in the order of Sec. III.C of Wen et al.
// (arXiv:1303.0625); weights 4/9, 1/9, 1/36.  Populations are stored as
// deviations d_i = f_i - w_i rho0 from the rest equilibrium, in one of four
// storage types; collision arithmetic runs in double (double and float
// storage) or float (half and bfloat16 storage, whose nodes next to a solid
// keep FP32 populations).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ---------------------------------------------------------------- lattice
__host__ __device__ constexpr int ex_(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int ey_(int i) {
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
// opposite direction ibar
__host__ __device__ constexpr int opp_(int i) {
    return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
template <typename C>
__host__ __device__ constexpr C w_(int i) {
    return i == 0 ? C(4.0 / 9.0) : (i <= 4 ? C(1.0 / 9.0) : C(1.0 / 36.0));
}
static_assert(opp_(1) == 3 && opp_(2) == 4 && opp_(3) == 1 && opp_(4) == 2, "opp");
static_assert(opp_(5) == 7 && opp_(6) == 8 && opp_(7) == 5 && opp_(8) == 6, "opp");

// ---------------------------------------------------------------- storage
struct bf16_t {
    uint16_t bits;
};

template <typename T>
struct Sto;
// kSplit: the storage type keeps the populations of the nodes next to a solid
// in FP32 instead (see the marker of the 16-bit types below).
template <>
struct Sto<double> {
    using C = double;
    static constexpr bool kSplit = false;
    __device__ static inline double ld(double v) { return v; }
    __device__ static inline double st(double c) { return c; }
    __device__ static inline bool marked(double) { return false; }
    __device__ static inline double mark() { return 0.0; }
};
// FP32 storage collides in double: the moment sums and the equilibrium are
// formed from deviations ~1e-4 whose float partial sums lose digits in a way
// that accumulates over thousands of steps (~1e-5 relative drag drift on the
// driven-cylinder channel, against ~1e-7 with one rounding per stored value).
// Double FMA issues at the non-packed FP32 rate on gfx950, so the
// bandwidth-bound update does not slow down.
template <>
struct Sto<float> {
    using C = double;
    static constexpr bool kSplit = false;
    __device__ static inline double ld(float v) { return (double)v; }
    __device__ static inline float st(double c) { return (float)c; }
    __device__ static inline bool marked(float) { return false; }
    __device__ static inline float mark() { return 0.0f; }
};
// Half and bfloat16 storage: the populations of a fluid node next to a solid
// (or a wall row) are kept in FP32, because the momentum the links exchange
// is formed from them and the slow flow next to the surface does not carry
// their rounding away (in a CPU emulation of the periodic single-cylinder
// run, rounding only these nodes to 16 bits gives the whole drag error of
// 16-bit storage; keeping them in FP32 leaves that of the FP32 arithmetic).
// Such a node's 16-bit slots hold a marker, a signalling-NaN pattern that no
// conversion of a computed value produces (conversions return quiet NaNs),
// and the FP32 value sits in a float array beside the population buffer at
// the same element index.
constexpr uint16_t kMarkF16 = 0x7c01;   // exponent all ones, quiet bit clear
constexpr uint16_t kMarkBF16 = 0x7f81;  // the same for bfloat16
template <>
struct Sto<_Float16> {
    using C = float;
    static constexpr bool kSplit = true;
    __device__ static inline float ld(_Float16 v) { return (float)v; }
    // hardware conversion rounds to nearest even; subnormals are kept
    __device__ static inline _Float16 st(float c) { return (_Float16)c; }
    __device__ static inline bool marked(_Float16 v) { return __builtin_bit_cast(uint16_t, v) == kMarkF16; }
    __device__ static inline _Float16 mark() { return __builtin_bit_cast(_Float16, kMarkF16); }
    // decode h + r and encode h = d - r (one rounding to half)
    __device__ static inline float ld_add(_Float16 h, float r) { return (float)h + r; }
    __device__ static inline _Float16 st_sub(float d, float r) { return (_Float16)(d - r); }
};
template <>
struct Sto<bf16_t> {
    using C = float;
    static constexpr bool kSplit = true;
    __device__ static inline bool marked(bf16_t v) { return v.bits == kMarkBF16; }
    __device__ static inline bf16_t mark() {
        bf16_t r;
        r.bits = kMarkBF16;
        return r;
    }
    __device__ static inline float ld(bf16_t v) { return __uint_as_float(((uint32_t)v.bits) << 16); }
    __device__ static inline float ld_add(bf16_t v, float r) { return ld(v) + r; }
    // the hardware conversion (v_cvt_pk_bf16_f32 on gfx950) rounds to
    // nearest even and returns quiet NaNs
    __device__ static inline bf16_t st(float c) {
        bf16_t r;
        r.bits = __builtin_bit_cast(uint16_t, (__bf16)c);
        return r;
    }
    __device__ static inline bf16_t st_sub(float d, float r) { return st(d - r); }
};

// ---------------------------------------------------------------- collision
// BGK collision with Guo forcing on the deviations d_i (Eq. 2 with the Eq. 8
// equilibrium).  rho = rho0 + sum d_i; rho*u = sum e_i d_i + rho*g/2;
//   d~_i = d_i - omega (d_i - deq_i) + (1 - 1/(2 tau)) w_i [3(e_i - u) + 9 (e_i.u) e_i] . rho g
// with deq_i = w_i [drho + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)].
template <typename C>
struct CollideParams {
    C rho0, omega, gx, gy, pref;  // pref = 1 - 1/(2 tau)
    int mrt;                      // 1: multiple-relaxation-time operator (below)
    C s_e, s_eps, s_q;            // its energy, energy-square and heat-flux rates
};

// 1/x: a correctly rounded division in FP64; in FP32, the arithmetic of the
// 16-bit storages, the hardware reciprocal (within 1 ulp, far below the
// storage's own rounding) instead of the ten-instruction IEEE division.
template <typename C>
__device__ inline C recip(C x) {
    return C(1) / x;
}
template <>
__device__ inline float recip<float>(float x) {
    return __builtin_amdgcn_rcpf(x);
}

// Moments of one node: drho = sum d_i, rho = rho0 + drho, Guo velocity u.
template <typename C>
struct Moments {
    C drho, rho, ux, uy;
};

template <typename C>
__device__ inline Moments<C> moments(const C d[9], const CollideParams<C>& p) {
    Moments<C> m;
    m.drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    m.rho = p.rho0 + m.drho;
    C jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    C jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
    C inv = recip<C>(m.rho);
    m.ux = jx * inv + C(0.5) * p.gx;
    m.uy = jy * inv + C(0.5) * p.gy;
    return m;
}

// Post-collision deviation of direction i from its pre-collision value di.
template <typename C>
__device__ inline C relax_one(int i, C di, const Moments<C>& m, const CollideParams<C>& p) {
    const C w = w_<C>(i);
    const C uu = m.ux * m.ux + m.uy * m.uy;
    const C Fx = m.rho * p.gx, Fy = m.rho * p.gy;
    const C uF = m.ux * Fx + m.uy * Fy;
    const C eu = C(ex_(i)) * m.ux + C(ey_(i)) * m.uy;
    const C eF = C(ex_(i)) * Fx + C(ey_(i)) * Fy;
    const C deq = w * (m.drho + m.rho * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu));
    const C src = p.pref * w * (C(3) * (eF - uF) + C(9) * eu * eF);
    return di - p.omega * (di - deq) + src;
}

// The same collision for all nine directions, written on the opposite pairs
// (i, ibar) with e_ibar = -e_i: the equilibrium and source terms split into
// a part even in e (shared by the pair) and an odd part (sign flipped):
//   d~_i = (1 - omega) d_i + A + B,   d~_ibar = (1 - omega) d_ibar + A - B,
//   A = w z + (e.u) [4.5 omega w rho (e.u) + 9 pref w (e.F)],
//   z = omega (drho - 1.5 rho u.u) - 3 pref u.F,
//   B = 3 omega w rho (e.u) + 3 pref w (e.F),   F = rho g;
// the rest direction keeps (1 - omega) d_0 + w_0 z.  Half the arithmetic of
// nine independent relax_one calls.
template <typename C>
__device__ inline void collide(C d[9], const CollideParams<C>& p, Moments<C>* mo_out = nullptr,
                               const Moments<C>* mo_in = nullptr) {
    // mo_in: the moments of d, when the caller has formed them already
    const Moments<C> m = mo_in ? *mo_in : moments<C>(d, p);
    if (mo_out) *mo_out = m;
    const C om = p.omega, keep = C(1) - p.omega;
    const C Fx = m.rho * p.gx, Fy = m.rho * p.gy;
    const C uu = m.ux * m.ux + m.uy * m.uy;
    const C uF = m.ux * Fx + m.uy * Fy;
    const C z = om * (m.drho - C(1.5) * m.rho * uu) - C(3) * p.pref * uF;
    const C orho = om * m.rho;
    d[0] = keep * d[0] + w_<C>(0) * z;
    auto pair = [&](int i, int j, C eu, C eF, C w) {
        const C t = (C(4.5) * w) * orho * eu + (C(9) * w) * p.pref * eF;
        const C A = w * z + eu * t;
        const C B = (C(3) * w) * orho * eu + (C(3) * w) * p.pref * eF;
        d[i] = keep * d[i] + (A + B);
        d[j] = keep * d[j] + (A - B);
    };
    pair(1, 3, m.ux, Fx, w_<C>(1));
    pair(2, 4, m.uy, Fy, w_<C>(2));
    pair(5, 7, m.ux + m.uy, Fx + Fy, w_<C>(5));
    pair(6, 8, m.uy - m.ux, Fy - Fx, w_<C>(6));
}

// Multiple-relaxation-time collision (Sec. IV) on the deviations, over the
// moments (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy) of the D2Q9 basis
// (Lallemand and Luo) with rates S = diag(0, s_e, s_eps, 0, s_q, 0, s_q,
// omega, omega): m* = m - S (m - m_eq) + (I - S/2) M F.  In this basis the
// Eq. 8 equilibrium has the moments
//   (rho, -2 rho + 3 rho u.u, rho - 3 rho u.u, rho u_x, -rho u_x, rho u_y,
//    -rho u_y, rho (u_x^2 - u_y^2), rho u_x u_y)
// and Guo's source (F = rho g, u the Guo velocity)
//   (0, 6 u.F, -6 u.F, F_x, -F_x, F_y, -F_y, 2 (u_x F_x - u_y F_y),
//    u_x F_y + u_y F_x);
// the rest-state part w rho0 of the deviations has moments rho0 (1, -2, 1, 0..)
// and drops out of m - m_eq.  The rows of M are orthogonal with squared
// norms (9, 36, 36, 6, 12, 6, 12, 4, 4), so M^-1 = M^T diag(1 / norms).
template <typename C>
__device__ inline void collide_mrt(C d[9], const CollideParams<C>& p, Moments<C>* mo_out = nullptr,
                                   const Moments<C>* mo_in = nullptr) {
    const Moments<C> mo = mo_in ? *mo_in : moments<C>(d, p);
    if (mo_out) *mo_out = mo;
    const C drho = mo.drho, rho = mo.rho, ux = mo.ux, uy = mo.uy;
    const C s14 = (d[1] + d[2]) + (d[3] + d[4]);
    const C s58 = (d[5] + d[6]) + (d[7] + d[8]);
    const C e = C(-4) * d[0] - s14 + C(2) * s58;
    const C eps = C(4) * d[0] - C(2) * s14 + s58;
    const C jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    const C jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
    const C qx = C(-2) * (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    const C qy = C(-2) * (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
    const C pxx = (d[1] - d[2]) + (d[3] - d[4]);
    const C pxy = (d[5] - d[6]) + (d[7] - d[8]);
    const C Fx = rho * p.gx, Fy = rho * p.gy;
    const C uu = ux * ux + uy * uy, uF = ux * Fx + uy * Fy;
    const C om = p.omega;
    // relaxed moments (deviation form; rho and j: mass kept, momentum + F)
    const C e1 = e - p.s_e * (e - (C(-2) * drho + C(3) * rho * uu)) + (C(1) - C(0.5) * p.s_e) * (C(6) * uF);
    const C eps1 = eps - p.s_eps * (eps - (drho - C(3) * rho * uu)) - (C(1) - C(0.5) * p.s_eps) * (C(6) * uF);
    const C jx1 = jx + Fx, jy1 = jy + Fy;
    const C qx1 = qx - p.s_q * (qx + rho * ux) - (C(1) - C(0.5) * p.s_q) * Fx;
    const C qy1 = qy - p.s_q * (qy + rho * uy) - (C(1) - C(0.5) * p.s_q) * Fy;
    const C pxx1 = pxx - om * (pxx - rho * (ux * ux - uy * uy)) + (C(1) - C(0.5) * om) * (C(2) * (ux * Fx - uy * Fy));
    const C pxy1 = pxy - om * (pxy - rho * ux * uy) + (C(1) - C(0.5) * om) * (ux * Fy + uy * Fx);
    // back to populations
    const C a = drho * C(1.0 / 9.0), b = e1 * C(1.0 / 36.0), c = eps1 * C(1.0 / 36.0);
    const C jx6 = jx1 * C(1.0 / 6.0), jy6 = jy1 * C(1.0 / 6.0);
    const C qx12 = qx1 * C(1.0 / 12.0), qy12 = qy1 * C(1.0 / 12.0);
    const C p4 = pxx1 * C(0.25), s4 = pxy1 * C(0.25);
    const C ax = a - b - C(2) * c;    // axis directions, even part
    const C dg = a + C(2) * b + c;    // diagonal directions, even part
    const C xo = jx6 - C(2) * qx12, yo = jy6 - C(2) * qy12;  // axis odd parts
    const C xd = jx6 + qx12, yd = jy6 + qy12;                // diagonal odd parts
    d[0] = a - C(4) * b + C(4) * c;
    d[1] = ax + xo + p4;
    d[3] = ax - xo + p4;
    d[2] = ax + yo - p4;
    d[4] = ax - yo - p4;
    d[5] = dg + xd + yd + s4;
    d[7] = dg - xd - yd + s4;
    d[6] = dg - xd + yd - s4;
    d[8] = dg + xd - yd - s4;
}

// The operator the parameters select (used off the streaming path).
template <typename C>
__device__ inline void collide_any(C d[9], const CollideParams<C>& p) {
    if (p.mrt)
        collide_mrt<C>(d, p);
    else
        collide<C>(d, p);
}

// Equilibrium deviation f_eq(rho, u) - w rho0 of Eq. 8, one direction.
template <typename C>
__device__ inline C feq_one(int i, C rho, C rho0, C ux, C uy) {
    const C uu = ux * ux + uy * uy;
    const C eu = C(ex_(i)) * ux + C(ey_(i)) * uy;
    return w_<C>(i) * ((rho - rho0) + rho * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu));
}

// All nine directions.
template <typename C>
__device__ inline void feq_dev(C rho, C rho0, C ux, C uy, C out[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] = feq_one<C>(i, rho, rho0, ux, uy);
}

// ---------------------------------------------------------------- misc
__host__ __device__ inline int wrapi(long v, int n) {
    long r = v % n;
    return (int)(r < 0 ? r + n : r);
}

// Solid record on the device (id 0 is the walls).
struct SolidDev {
    double x0, y0;   // centre at t = 0
    double a, b;     // disc radius / box half-extents
    double vx, vy;   // velocity
    int32_t shape;   // 0 disc, 1 box
    int32_t moves;   // geometry translates
};

// Free discs (particles moving under gravity and the hydrodynamic force):
// state at step t in slot t % 3 (the mover reads t - 1 and t while the next
// step's values go to t + 1).
struct FreeDyn {
    double X[3], Y[3], Vx[3], Vy[3], Om[3];  // centre, velocity, angular velocity
    double M, I, A;                          // mass, moment of inertia, area
    int s;                                   // solid id
    int pad;
};

// Per-solid rotation table, one per step parity: {Omega, X, Y, free} with the
// centre of a free body at that step (Omega = 0 for every other solid).
constexpr int kRot = 4;

// Minimum-image difference on a periodic axis of length n.
__device__ inline double min_image(double d, int n) { return d - (double)n * rint(d / (double)n); }

// Centre of a solid at step t: X = x0 + t*vx with separately rounded product
// and sum (contraction into a fused multiply-add is switched off here and in
// solid_inside), so that the solid/fluid decision of every node is the one a
// plain IEEE double evaluation takes.
__device__ inline void solid_pos(const SolidDev& s, int64_t t, double& X, double& Y) {
#pragma clang fp contract(off)
    if (s.moves) {
        X = s.x0 + (double)t * s.vx;
        Y = s.y0 + (double)t * s.vy;
    } else {
        X = s.x0;
        Y = s.y0;
    }
}

// Whether integer point (x, y) lies inside solid s centred at (X, Y).
__device__ inline bool solid_inside(const SolidDev& s, double X, double Y, long x, long y) {
#pragma clang fp contract(off)
    double dx = (double)x - X;
    double dy = (double)y - Y;
    if (s.shape == 0) {
        double d2 = dx * dx;
        d2 = d2 + dy * dy;
        return d2 <= s.a * s.a;
    }
    return fabs(dx) <= s.a && fabs(dy) <= s.b;
}

// Centre of solid sid at step t: a free body's from the step's rotation
// table {Omega, X, Y, free}, any other from its prescribed motion.
__device__ inline void solid_centre(const SolidDev* __restrict__ sol, const double* __restrict__ rt, int sid,
                                    int64_t t, double& X, double& Y) {
    if (rt != nullptr && rt[kRot * sid + 3] != 0.0) {
        X = rt[kRot * sid + 1];
        Y = rt[kRot * sid + 2];
    } else {
        solid_pos(sol[sid], t, X, Y);
    }
}

// Fraction q of the link from node (x, y) along (ex, ey) at which the link
// enters solid S centred at (X, Y) (interpolated bounce-back, Sec. IV): the
// node lies outside, (x + ex, y + ey) inside, so 0 < q <= 1.  Disc: the
// nearer root of |P + q e| = r with P the node's offset from the centre
// (half-coefficient form); box: the last of the two slab entries.  Offsets
// take the minimum image on periodic axes; rounding is clamped into (0, 1].
__device__ inline double link_fraction(const SolidDev& S, double X, double Y, int x, int y, int ex, int ey,
                                       int nx, int ny, int walls) {
    const double px = min_image((double)x - X, nx);
    const double py = walls ? (double)y - Y : min_image((double)y - Y, ny);
    double q;
    if (S.shape == 0) {
        const double e2 = (double)(ex * ex + ey * ey);
        const double pe = px * ex + py * ey;
        const double c = px * px + py * py - S.a * S.a;
        const double disc = pe * pe - e2 * c;
        q = (-pe - sqrt(disc > 0.0 ? disc : 0.0)) / e2;
    } else {
        q = -1.0e300;
        if (ex != 0) q = fmax(q, fmin((-S.a - px) * ex, (S.a - px) * ex));
        if (ey != 0) q = fmax(q, fmin((-S.b - py) * ey, (S.b - py) * ey));
    }
    if (q <= 0.0) q = 1.0e-12;
    return q > 1.0 ? 1.0 : q;
}

// Population returned by interpolated bounce-back (linear in q) for the
// direction whose link from the fluid node meets the surface at fraction q:
//   q <  1/2:  2q fo + (1 - 2q) fb + m   (fb: the opposite population of the
//              fluid node behind; half-way fo + m when there is none)
//   q >= 1/2:  (fo + m)/(2q) + (1 - 1/(2q)) fi
// fo: the node's own population towards the surface, fi: its own population
// away from it, m: the moving-wall term.  q = 1/2 is half-way bounce-back.
template <typename C>
__device__ inline C ibb_value(double q, C fo, C fi, C fb, bool behind, C m) {
    if (q == 0.5) return fo + m;
    if (q < 0.5) return behind ? C(2.0 * q) * fo + C(1.0 - 2.0 * q) * fb + m : fo + m;
    const double h = 0.5 / q;
    return C(h) * (fo + m) + C(1.0 - h) * fi;
}

// Integer bounding range (with a margin) of solid s centred at (X, Y).
__device__ inline void solid_range(const SolidDev& s, double X, double Y, int margin, long& x0,
                                   long& x1, long& y0, long& y1) {
    double hx = s.a, hy = s.shape == 0 ? s.a : s.b;
    x0 = (long)floor(X - hx) - margin;
    x1 = (long)ceil(X + hx) + margin;
    y0 = (long)floor(Y - hy) - margin;
    y1 = (long)ceil(Y + hy) + margin;
}

// XCD-aware block order: the hardware hands consecutive workgroups to the 8
// XCDs in turn; remap so that each XCD walks a contiguous band of tiles and
// the halo lines shared by neighbouring tiles stay in one L2.
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nb) {
    const uint32_t nxcd = 8;
    uint32_t per = nb / nxcd;
    uint32_t full = per * nxcd;
    if (b >= full) return b;
    return (b % nxcd) * per + b / nxcd;
}

}  // namespace lbm
