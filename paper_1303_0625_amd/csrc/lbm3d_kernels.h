// lbm3d_kernels.h -- HIP kernels of the three-dimensional (D3Q19) momentum-
// exchange step, Sec. IV.D: a duct of solid nodes and spheres whose surfaces
// move rigidly (fixed, translating with newborn refill, or free), half-way
// or interpolated bounce-back with the moving-boundary term, BGK collision
// with Guo forcing, per-link CME (Eq. 4) / GME (Eq. 5) forces with torque
// about each sphere's centre (Eqs. 6-7), and pressure inlet/outlet planes.
//
// State: post-collision deviations d~_i = f~_i - w_i rho0 of every fluid
// node, layout [z][y][19][pitch] (the nineteen population rows of one (y, z)
// line are contiguous), two ping-pong buffers by step parity.  One launch per
// step: force workgroups (512 links each, fixed-order partials), one
// finalizer workgroup per (solid, force or torque component) forming the
// previous step's totals in a fixed order (the first also advances the step
// counter), and from n_lead on the update workgroups (one thread per node, a
// wave = 64 consecutive x of one line).
#pragma once

#include "lbm_device.h"

namespace lbm3 {

using lbm::Sto;

constexpr int kBlock = 256;
constexpr int kChunk = 512;  // links per force workgroup
constexpr int kQ = 19;
constexpr uint8_t kDuct = 255;  // owner value of duct nodes (force slot 0)
// Node flags kept beside the owners: the node is solid, or it is fluid and
// some neighbour x + e_i (equally, some source x - e_i) is solid.
constexpr uint8_t kSolidNode = 2, kNearSolid = 1;

// Velocity set: rest, the axis directions (+x, -x, +y, -y, +z, -z), the
// twelve edge diagonals in opposite pairs; opposite of i is i + 1 for odd
// i, i - 1 for even i > 0.
__device__ constexpr int kE[kQ][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                                      {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                      {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                      {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
__device__ constexpr int opp3(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__device__ constexpr double w3(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

struct Args {
    int nx, ny, nz;
    int pitch;        // elements per population row (multiple of 64)
    int ns;           // spheres (solid slots: 0 duct, 1..ns spheres)
    double rho0, tau;
    double g[3];      // body force (acceleration)
    int nchunks;      // force workgroups
    int64_t hist_cap;
    int duct;         // 0 open, 1 tube, 2 planes
    double R;         // tube radius
    int box;          // edge of a moving sphere's scan box (nodes)
    int refill;       // 0 A1, 1 A2, 2 A3
    int ibb;          // interpolated bounce-back on sphere links
    double rho_in, rho_out;  // pressure planes x = 0 and x = nx - 1
    double omega, cs;        // 1 / tau and 1 - 1 / (2 tau), formed on the host
    // update workgroups per plane K, waves per line W and ny, with the
    // multipliers and shifts of their division (divq)
    uint32_t K, magK, shK, W, magW, shW, magNy, shNy;
};

// n / d for 0 <= n < 2^31 from the round-up multiplier m and shift
// l = ceil(log2 d) of d (Granlund and Montgomery, PLDI 1994).
__device__ inline uint32_t divq(uint32_t n, uint32_t m, uint32_t l) { return (__umulhi(n, m) + n) >> l; }

// Lines (y, z) that the duct makes solid at every x: the tube's outside, the
// two planes.  The squares of the half-integer offsets and their sum are
// exact in double, so the test is the same wherever it is evaluated.
__device__ inline bool duct_solid3(int y, int z, const Args& a) {
#pragma clang fp contract(off)
    if (a.duct == 1) {
        const double dy = (double)y - 0.5 * (a.ny - 1), dz = (double)z - 0.5 * (a.nz - 1);
        return dy * dy + dz * dz > a.R * a.R;
    }
    return a.duct == 2 && (z == 0 || z == a.nz - 1);
}

// Solid table row: X, r, V (3), Omega (3), moves, free; row 0 is the duct.
// One table per step parity: a free sphere's row holds its centre, velocity
// and spin at that step (written by the free-sphere update), every other
// row its initial centre and prescribed motion.
constexpr int kSolidRow = 12;

// Centre of sphere slot s at step t (a translating sphere: X0 + t V,
// product and sum rounded separately; a free sphere: the table's centre).
__device__ inline void centre3(const double* __restrict__ sol, int s, int64_t t, double X[3]) {
#pragma clang fp contract(off)
    const double* S = sol + kSolidRow * s;
    const bool mv = S[10] != 0.0 && S[11] == 0.0;
    for (int d = 0; d < 3; ++d) X[d] = mv ? S[d] + (double)t * S[4 + d] : S[d];
}

__device__ inline double min_image3(double d, int n) { return d - (double)n * floor(d / (double)n + 0.5); }

// Rigid surface velocity of solid slot s at point p at step t (duct at
// rest), and the arm from the centre.
__device__ inline void surface_vel(const double* __restrict__ sol, int s, int64_t t, double px, double py,
                                   double pz, const Args& a, double v[3], double r[3]) {
    if (s == 0) {
        v[0] = v[1] = v[2] = 0.0;
        r[0] = r[1] = r[2] = 0.0;
        return;
    }
    const double* S = sol + kSolidRow * s;
    double X[3];
    centre3(sol, s, t, X);
    r[0] = min_image3(px - X[0], a.nx);
    r[1] = min_image3(py - X[1], a.ny);
    r[2] = min_image3(pz - X[2], a.nz);
    v[0] = S[4] + (S[8] * r[2] - S[9] * r[1]);
    v[1] = S[5] + (S[9] * r[0] - S[7] * r[2]);
    v[2] = S[6] + (S[7] * r[1] - S[8] * r[0]);
}

__device__ inline int wrap3(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Fraction q in (0, 1] of the link from fluid node (., y, z) along e to the
// tube wall: the larger root of |P + q e| = R in the (y, z) plane (the node
// inside, its neighbour outside), P the node's offset from the axis.
__device__ inline double tube_q3(int y, int z, int ey, int ez, const Args& a) {
    const double py = (double)y - 0.5 * (a.ny - 1), pz = (double)z - 0.5 * (a.nz - 1);
    const double e2 = (double)(ey * ey + ez * ez);
    const double pe = py * ey + pz * ez;
    const double c = py * py + pz * pz - a.R * a.R;
    const double disc = pe * pe - e2 * c;
    double q = (-pe + sqrt(disc > 0.0 ? disc : 0.0)) / e2;
    if (q <= 0.0) q = 1.0e-12;
    return q > 1.0 ? 1.0 : q;
}

// Fraction q in (0, 1] of the link from node (x, y, z) along e into sphere
// slot s at step t: the nearer root of |P + q e| = r with P the node's
// minimum-image offset from the centre (half-coefficient form), clamped.
__device__ inline double sphere_q3(const double* __restrict__ sol, int s, int64_t t, int x, int y, int z, int ex,
                                   int ey, int ez, const Args& a) {
    double X[3];
    centre3(sol, s, t, X);
    const double px = min_image3((double)x - X[0], a.nx), py = min_image3((double)y - X[1], a.ny),
                 pz = min_image3((double)z - X[2], a.nz);
    const double r = sol[kSolidRow * s + 3];
    const double e2 = (double)(ex * ex + ey * ey + ez * ez);
    const double pe = px * ex + py * ey + pz * ez;
    const double c = px * px + py * py + pz * pz - r * r;
    const double disc = pe * pe - e2 * c;
    double q = (-pe - sqrt(disc > 0.0 ? disc : 0.0)) / e2;
    if (q <= 0.0) q = 1.0e-12;
    return q > 1.0 ? 1.0 : q;
}

// BGK + Guo on deviations, in FP64: rho = rho0 + sum d, momentum sum e d
// (the weights' first moment vanishes), u = (j + rho g/2)/rho.  With
// eu = e_i . u and eF = e_i . F the post-collision value is
//   (1 - omega) d_i + w_i [C + eu (4.5 omega rho eu + 9 cs eF)]
//                   + w_i [3 omega rho eu + 3 cs eF],
// C = omega (drho - 1.5 rho u^2) - 3 cs u . F: the equilibrium deviation
// w (rho - rho0) + w rho (3 eu + 4.5 eu^2 - 1.5 u^2) relaxed at omega plus
// the Guo source w [3 (e - u) + 9 (e . u) e] . F at cs, grouped by parity
// in e_i so that each opposite pair (i, i + 1) shares the even part and
// takes the odd part with opposite signs.
__device__ inline void collide3(double d[kQ], const Args& a) {
    double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        drho += d[i];
        jx += kE[i][0] * d[i];
        jy += kE[i][1] * d[i];
        jz += kE[i][2] * d[i];
    }
    const double rho = a.rho0 + drho;
    const double Fx = rho * a.g[0], Fy = rho * a.g[1], Fz = rho * a.g[2];
    // one correctly rounded reciprocal instead of three divisions (and the
    // rates from the host: no division per node on the tau of the lattice)
    const double inv = 1.0 / rho;
    const double ux = (jx + 0.5 * Fx) * inv, uy = (jy + 0.5 * Fy) * inv, uz = (jz + 0.5 * Fz) * inv;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double om = a.omega, cs = a.cs, keep = 1.0 - a.omega;
    const double uF = ux * Fx + uy * Fy + uz * Fz;
    const double C = om * (drho - 1.5 * rho * uu) - 3.0 * cs * uF;
    const double P = 4.5 * om * rho, R = 3.0 * om * rho;
    const double Q = 9.0 * cs, S = 3.0 * cs;
    d[0] = keep * d[0] + w3(0) * C;
#pragma unroll
    for (int i = 1; i < kQ; i += 2) {
        const double w = w3(i);
        const double eu = kE[i][0] * ux + kE[i][1] * uy + kE[i][2] * uz;
        const double eF = kE[i][0] * Fx + kE[i][1] * Fy + kE[i][2] * Fz;
        const double ev = w * (C + eu * (P * eu + Q * eF));
        const double od = w * (R * eu + S * eF);
        d[i] = keep * d[i] + (ev + od);
        d[i + 1] = keep * d[i + 1] + (ev - od);
    }
}

struct Ptrs {
    const void* fin;
    void* fout;
    const uint8_t* own;
    const uint8_t* flags;     // per node: kSolidNode, kNearSolid or 0
    const uint32_t* links;    // per link: node << 5 | i
    const int* seg_off;       // per solid slot
    const int* seg_cnt;
    const int* chunk_solid;
    const int* chunk_start;
    const int* solid_chunk0;  // [ns + 2]
    const double* sol;        // [ns + 1][kSolidRow]
    double* partial;          // [2][nchunks][12]
    double* hist;             // [hist_cap][ns + 1][12]
    int64_t* tctr;
};

// Per link (x_f, i) of solid s: a = f~_i(x_f), b = a - 6 w_i rho0 (e_i . v)
// with v at the link midpoint; CME F = e_i (a + b), GME F = (e_i - v) a +
// (e_i + v) b; torque r x F about the sphere's centre.
// IBB: interpolated bounce-back may be on (a.ibb); without it the link code
// (and the kernel's registers) stay those of half-way bounce-back.
template <typename T, bool IBB>
__device__ inline void force_role3(int c, const Ptrs& p, double* __restrict__ partial, const Args& a,
                                   double (*red)[12], int64_t t) {
    const T* f = (const T*)p.fin;
    const int s = p.chunk_solid[c];
    const int start = p.chunk_start[c];
    // a moving sphere's links are found by scanning its box at step t (one
    // node and its 18 directions per thread); other solids walk their list
    const bool box = s > 0 && p.sol[kSolidRow * s + 10] != 0.0;
    int bx0 = 0, by0 = 0, bz0 = 0;
    if (box) {
        double X[3];
        centre3(p.sol, s, t, X);
        const double r0 = p.sol[kSolidRow * s + 3];
        bx0 = (int)floor(X[0] - r0) - 2;
        by0 = (int)floor(X[1] - r0) - 2;
        bz0 = (int)floor(X[2] - r0) - 2;
    }
    const int n = box ? a.box * a.box * a.box : p.seg_cnt[s];
    const int end = start + kChunk < n ? start + kChunk : n;
    const uint32_t* L = p.links + p.seg_off[s];
    double acc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = 0.0;
    for (int k = start + (int)threadIdx.x; k < end; k += kBlock) {
        int x, y, z, i0, i1;
        if (box) {
            const int bx = k % a.box, by = (k / a.box) % a.box, bz = k / (a.box * a.box);
            x = ((bx0 + bx) % a.nx + a.nx) % a.nx;
            y = ((by0 + by) % a.ny + a.ny) % a.ny;
            z = ((bz0 + bz) % a.nz + a.nz) % a.nz;
            if (p.own[((int64_t)z * a.ny + y) * a.pitch + x] != 0) continue;
            i0 = 1;
            i1 = kQ;
        } else {
            const uint32_t code = L[k];
            const uint32_t node = code >> 5;
            x = (int)(node % (uint32_t)a.nx);
            const uint32_t ln = node / (uint32_t)a.nx;  // z * ny + y
            y = (int)(ln % (uint32_t)a.ny);
            z = (int)(ln / (uint32_t)a.ny);
            i0 = (int)(code & 31u);
            i1 = i0 + 1;
        }
        const int64_t line = (int64_t)z * a.ny + y;
        for (int i = i0; i < i1; ++i) {
        if (box) {
            const int xb = wrap3(x + kE[i][0], a.nx), yb = wrap3(y + kE[i][1], a.ny), zb = wrap3(z + kE[i][2], a.nz);
            if (p.own[((int64_t)zb * a.ny + yb) * a.pitch + xb] != s) continue;
        }
        const double ex = kE[i][0], ey = kE[i][1], ez = kE[i][2], w = w3(i);
        // surface point x_f + q e_i (q = 1/2 unless interpolated on a sphere)
        double q = 0.5;
        if constexpr (IBB) {
            if (a.ibb && s > 0) q = sphere_q3(p.sol, s, t, x, y, z, kE[i][0], kE[i][1], kE[i][2], a);
            if (a.ibb && s == 0 && a.duct == 1) q = tube_q3(y, z, kE[i][1], kE[i][2], a);
        }
        double v[3], r[3];
        surface_vel(p.sol, s, t, x + q * ex, y + q * ey, z + q * ez, a, v, r);
        const double av =
            w * a.rho0 + (double)Sto<T>::ld(f[((int64_t)line * kQ + i) * a.pitch + x]);
        const double m = 6.0 * w * a.rho0 * (ex * v[0] + ey * v[1] + ez * v[2]);
        double bv = av - m;
        if (IBB && q < 0.5) {  // the returning population of the interpolated rule
            const int xq = wrap3(x - kE[i][0], a.nx), yq = wrap3(y - kE[i][1], a.ny), zq = wrap3(z - kE[i][2], a.nz);
            const int64_t lq = (int64_t)zq * a.ny + yq;
            if (p.own[lq * a.pitch + xq] == 0)
                bv = 2.0 * q * av + (1.0 - 2.0 * q) * (w * a.rho0 + (double)Sto<T>::ld(f[(lq * kQ + i) * a.pitch + xq])) - m;
        } else if (IBB && q > 0.5) {
            const double fo = w * a.rho0 + (double)Sto<T>::ld(f[((int64_t)line * kQ + opp3(i)) * a.pitch + x]);
            const double h = 0.5 / q;
            bv = h * (av - m) + (1.0 - h) * fo;
        }
        const double e[3] = {ex, ey, ez};
        double Fc[3], Fg[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            Fc[d] = e[d] * av + e[d] * bv;
            Fg[d] = (e[d] - v[d]) * av + (e[d] + v[d]) * bv;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            acc[d] += Fc[d];
            acc[6 + d] += Fg[d];
        }
        if (s > 0) {
            acc[3] += r[1] * Fc[2] - r[2] * Fc[1];
            acc[4] += r[2] * Fc[0] - r[0] * Fc[2];
            acc[5] += r[0] * Fc[1] - r[1] * Fc[0];
            acc[9] += r[1] * Fg[2] - r[2] * Fg[1];
            acc[10] += r[2] * Fg[0] - r[0] * Fg[2];
            acc[11] += r[0] * Fg[1] - r[1] * Fg[0];
        }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        double v = acc[q];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        const int q = threadIdx.x;
        partial[c * 12 + q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    }
}

// Total of component q of solid s at step `step` from the chunk partials
// (one workgroup per (s, q)): thread j sums chunks j, j + 256, ... in order,
// then a fixed shuffle tree per wave and the four waves in order, so the
// result does not depend on scheduling.
__device__ inline void finalize3(const double* __restrict__ partial, const int* __restrict__ solid_chunk0,
                                 double* __restrict__ hist, int64_t step, int pair, const Args& a,
                                 double* red) {
    const int s = pair / 12, q = pair % 12;
    const int c0 = solid_chunk0[s], c1 = solid_chunk0[s + 1];
    double v = 0.0;
    for (int cc = c0 + (int)threadIdx.x; cc < c1; cc += kBlock) v += partial[cc * 12 + q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        hist[((step % a.hist_cap) * (a.ns + 1) + s) * 12 + q] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Update of node (x, line): pull the nineteen populations (all loads issued
// before any is used), replace those whose source is solid by the half-way
// bounce-back of the node's own opposite population plus 6 w_i rho0
// (e_i . v), v the surface velocity at x - e_i/2; collide; store.
// A wave covers 64 consecutive x of one line, so y and z (and every source
// line) are wave-uniform: each access is a scalar line base plus a 32-bit
// lane offset (x - 1, x or x + 1, wrapped).
template <typename T>
__device__ inline const T* at3(const T* base, uint32_t idx) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(T));
}

// PR: pressure planes.  A node of the plane x = 0 (x = nx - 1) whose inner
// neighbour x = 1 (nx - 2) is fluid too computes that neighbour's update
// itself and stores it moved to the plane's density by non-equilibrium
// extrapolation (Guo, Zheng and Shi 2002), the boundary condition applied to
// the post-collision state in the same launch.
template <typename T, bool NT, bool IBB, bool PR>
__device__ inline void update3(int xo, int y, int z, const Ptrs& p, const Args& a, int64_t t) {
    const char* fin = (const char*)p.fin;
    char* fout = (char*)p.fout;
    const uint32_t ny = (uint32_t)a.ny, pitch = (uint32_t)a.pitch;
    // byte strides of a population row and of a line's nineteen rows
    const uint32_t rowB = pitch * (uint32_t)sizeof(T), lineB = (uint32_t)kQ * rowB;
    // wave-uniform: the wrapped neighbour lines, and the line z_s ny + y_s
    // that direction i pulls from
    const uint32_t uy = (uint32_t)y, uz = (uint32_t)z;
    const uint32_t ym = uy == 0 ? ny - 1 : uy - 1, yp = uy + 1 == ny ? 0 : uy + 1;
    const uint32_t zm = uz == 0 ? (uint32_t)a.nz - 1 : uz - 1, zp = uz + 1 == (uint32_t)a.nz ? 0 : uz + 1;
    auto src_line = [&](int i) -> uint32_t {
        const uint32_t ys = kE[i][1] == 1 ? ym : (kE[i][1] == -1 ? yp : uy);
        const uint32_t zs = kE[i][2] == 1 ? zm : (kE[i][2] == -1 ? zp : uz);
        return zs * ny + ys;
    };
    const uint32_t line = uz * ny + uy;
    auto own_at = [&](uint32_t L, uint32_t xs) -> uint32_t { return *at3(p.own + (uint64_t)L * pitch, xs); };
    auto row_in = [&](uint32_t L, int i) -> const T* {
        return (const T*)(fin + (uint64_t)L * lineB + (uint32_t)i * rowB);
    };
    int x = xo;
    bool plane = false;
    if constexpr (PR) {
        if (xo == 0 || xo == a.nx - 1) {
            const int xf = xo == 0 ? 1 : a.nx - 2;
            plane = own_at(line, (uint32_t)xo) == 0 && own_at(line, (uint32_t)xf) == 0;
            if (plane) x = xf;
        }
    }
    const uint32_t ux = (uint32_t)x;
    const uint32_t uxm = (uint32_t)(x == 0 ? a.nx - 1 : x - 1), uxp = (uint32_t)(x == a.nx - 1 ? 0 : x + 1);
    auto src_x = [&](int i) -> uint32_t { return kE[i][0] == 1 ? uxm : (kE[i][0] == -1 ? uxp : ux); };
    // every load is issued whatever the node's flags (a solid node's values
    // are computed on and not stored: a test before the loads would cost a
    // round trip to memory).  Streamed (large) lattices read the owners of
    // the sources only where the flags say that one of them is solid; in a
    // cache-resident lattice the step is latency-bound, so the eighteen
    // owners come with the populations (only their OR is kept through the
    // loads; they are read again, from cache, where a source is solid)
    const uint32_t flag = *at3(p.flags + (uint64_t)line * pitch, ux);
    T raw[kQ];
    uint32_t any = 0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const uint32_t L = src_line(i), xs = src_x(i);
        if (!NT && i > 0) any |= own_at(L, xs);
        const T* ptr = at3(row_in(L, i), xs);
        if constexpr (NT)
            raw[i] = __builtin_nontemporal_load(ptr);
        else
            raw[i] = *ptr;
    }
    double d[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) d[i] = (double)Sto<T>::ld(raw[i]);
    const bool self = (flag & kSolidNode) != 0;
    if (NT ? flag == kNearSolid : (any != 0 && !self)) {
        uint32_t src[kQ];
#pragma unroll
        for (int i = 1; i < kQ; ++i) src[i] = own_at(src_line(i), src_x(i));
        // the node's own values that bounce back: with the interpolated rule
        // (many solid directions per node, each with its own geometry) all of
        // them are loaded together here instead of one round trip per
        // direction; the half-way rule keeps the registers for occupancy
        T mine[kQ];
        if constexpr (IBB) {
#pragma unroll
            for (int i = 1; i < kQ; ++i) mine[i] = *at3(row_in(line, i), ux);
        }
        auto own_val = [&](int i) -> double {
            if constexpr (IBB)
                return (double)Sto<T>::ld(mine[i]);
            else
                return (double)Sto<T>::ld(*at3(row_in(line, i), ux));
        };
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
            if (src[i] == 0) continue;
            const int s = src[i] == kDuct ? 0 : (int)src[i];
            if constexpr (IBB) {
                if (s > 0 || a.duct == 1) {
                    // interpolated bounce-back (spheres and tube): surface
                    // point x - q e_i; the node behind, x + e_i, is the source
                    // of o = opp(i), so d[o] still holds its value when fluid
                    const double q = s > 0 ? sphere_q3(p.sol, s, t, x, y, z, -kE[i][0], -kE[i][1], -kE[i][2], a)
                                           : tube_q3(y, z, -kE[i][1], -kE[i][2], a);
                    double v[3], r[3];
                    surface_vel(p.sol, s, t, x - q * kE[i][0], y - q * kE[i][1], z - q * kE[i][2], a, v, r);
                    const double m = 6.0 * w3(i) * a.rho0 * (kE[i][0] * v[0] + kE[i][1] * v[1] + kE[i][2] * v[2]);
                    const int o = opp3(i);
                    d[i] = lbm::ibb_value<double>(q, own_val(o), own_val(i), d[o], src[o] == 0, m);
                    continue;
                }
            }
            double v[3], r[3];
            surface_vel(p.sol, s, t, x - 0.5 * kE[i][0], y - 0.5 * kE[i][1], z - 0.5 * kE[i][2], a, v, r);
            d[i] = own_val(opp3(i)) + 6.0 * w3(i) * a.rho0 * (kE[i][0] * v[0] + kE[i][1] * v[1] + kE[i][2] * v[2]);
        }
    }
    collide3(d, a);
    if constexpr (PR) {
        if (plane) {
            // the neighbour's stored post-collision state, moments and shift
            double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                d[i] = (double)Sto<T>::ld(Sto<T>::st(d[i]));
                drho += d[i];
                j[0] += kE[i][0] * d[i];
                j[1] += kE[i][1] * d[i];
                j[2] += kE[i][2] * d[i];
            }
            const double rho = a.rho0 + drho;
            const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
            const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            const double dr = (xo == 0 ? a.rho_in : a.rho_out) - rho;
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const double eu = kE[i][0] * u[0] + kE[i][1] * u[1] + kE[i][2] * u[2];
                d[i] += w3(i) * dr * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
            }
        }
    }
    if (self) return;
    const uint32_t uxo = (uint32_t)xo;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        T* ptr = const_cast<T*>(at3((const T*)(fout + (uint64_t)line * lineB + (uint32_t)i * rowB), uxo));
        const T val = Sto<T>::st(d[i]);
        if constexpr (NT)
            __builtin_nontemporal_store(val, ptr);
        else
            *ptr = val;
    }
}

// Workgroups [0, nchunks) force chunks, the next (ns + 1) * 12 the previous
// step's totals (the first also advances the step counter), update
// workgroups from n_lead (a multiple of 8) on.
template <typename T, bool NT, bool IBB, bool PR>
__global__ __launch_bounds__(kBlock) void k3_step(Ptrs p, int parity, int n_lead, Args a) {
    __shared__ double red[kBlock / 64][12];
    const int b = (int)blockIdx.x;
    if (b < n_lead) {
        const int64_t t = p.tctr[parity];
        if (b < a.nchunks) {
            force_role3<T, IBB>(b, p, p.partial + (size_t)(t & 1) * a.nchunks * 12, a, red, t);
        } else if (b < a.nchunks + (a.ns + 1) * 12) {
            const int pair = b - a.nchunks;
            if (t >= 1)
                finalize3(p.partial + (size_t)((t - 1) & 1) * a.nchunks * 12, p.solid_chunk0, p.hist, t - 1, pair,
                          a, &red[0][0]);
            if (pair == 0 && threadIdx.x == 0) p.tctr[parity ^ 1] = t + 1;
        }
        return;
    }
    // XCD-aware order: workgroup b runs on XCD b % 8 (n_lead and the number
    // of update workgroups are multiples of 8 K); each XCD takes a run of K
    // consecutive workgroups, one plane's worth of waves, and the eight XCDs
    // eight consecutive runs at a time, so the lines y +- 1 a node pulls from
    // are in the XCD's own L2 while all XCDs stay in one neighbourhood of
    // planes.  The divisions use multipliers formed on the host.
    const uint32_t u = (uint32_t)(b - n_lead), v = u >> 3;
    const uint32_t grp = divq(v, a.magK, a.shK);
    const uint32_t ub = grp * 8u * a.K + (u & 7u) * a.K + (v - grp * a.K);
    const uint32_t gw = ub * (kBlock / 64) + (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t line = divq(gw, a.magW, a.shW);
    const int x = (int)((gw - line * a.W) << 6) + (int)(threadIdx.x & 63);
    const uint32_t z = divq(line, a.magNy, a.shNy), y = line - z * (uint32_t)a.ny;
    // the duct's solid lines hold no fluid node: the whole wave leaves
    if (z >= (uint32_t)a.nz || duct_solid3((int)y, (int)z, a) || x >= a.nx) return;
    update3<T, NT, IBB, PR>(x, (int)y, (int)z, p, a, p.tctr[parity]);
}

// Owner of node (x, y, z) at step t: the duct, then the spheres (minimum
// image, separately rounded products and sums, ties solid).
__device__ inline uint8_t owner3(const double* __restrict__ sol, int x, int y, int z, int64_t t, const Args& a) {
#pragma clang fp contract(off)
    uint8_t o = duct_solid3(y, z, a) ? kDuct : 0;
    for (int k = 1; k <= a.ns; ++k) {
        double X[3];
        centre3(sol, k, t, X);
        const double dx = min_image3((double)x - X[0], a.nx), dy = min_image3((double)y - X[1], a.ny),
                     dz = min_image3((double)z - X[2], a.nz);
        double d2 = dx * dx;
        d2 = d2 + dy * dy;
        d2 = d2 + dz * dz;
        const double r = sol[kSolidRow * k + 3];
        if (d2 <= r * r) o = (uint8_t)k;
    }
    return o;
}

// Geometry of step t + 1 (moving spheres): the owner of every node.
__global__ __launch_bounds__(kBlock) void k3_raster(const double* __restrict__ sol, uint8_t* __restrict__ own_n,
                                                    int64_t t1, Args a) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= (int64_t)a.nx * a.ny * a.nz) return;
    const int x = (int)(n % a.nx);
    const int64_t line = n / a.nx;
    own_n[line * a.pitch + x] = owner3(sol, x, (int)(line % a.ny), (int)(line / a.ny), t1, a);
}

// Flags of every node from the owners of step t + 1 (moving spheres).
__global__ __launch_bounds__(kBlock) void k3_flags(const uint8_t* __restrict__ own_n, uint8_t* __restrict__ flags_n,
                                                   Args a) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= (int64_t)a.nx * a.ny * a.nz) return;
    const int x = (int)(n % a.nx);
    const int64_t line = n / a.nx;
    const int y = (int)(line % a.ny), z = (int)(line / a.ny);
    uint8_t f = 0;
    if (own_n[line * a.pitch + x] != 0) {
        f = kSolidNode;
    } else {
        for (int i = 1; i < kQ; ++i) {
            const int xb = wrap3(x + kE[i][0], a.nx), yb = wrap3(y + kE[i][1], a.ny), zb = wrap3(z + kE[i][2], a.nz);
            if (own_n[((int64_t)zb * a.ny + yb) * a.pitch + xb] != 0) f = kNearSolid;
        }
    }
    flags_n[line * a.pitch + x] = f;
}

// Post-advection deviation of direction j at node (x, y, z) from step t's
// post-collision populations: streamed from x - e_j, or the half-way
// bounce-back with the moving-wall term when that node is solid at t.
template <typename T>
__device__ inline double pull3(const T* __restrict__ fin, const uint8_t* __restrict__ own_t,
                               const double* __restrict__ sol, int x, int y, int z, int j, int64_t t, const Args& a) {
    const int xs = wrap3(x - kE[j][0], a.nx), ys = wrap3(y - kE[j][1], a.ny), zs = wrap3(z - kE[j][2], a.nz);
    const int64_t ls = (int64_t)zs * a.ny + ys;
    const uint8_t o = own_t[ls * a.pitch + xs];
    if (o == 0) return (double)Sto<T>::ld(fin[(ls * kQ + j) * a.pitch + xs]);
    const int64_t line = (int64_t)z * a.ny + y;
    if (a.ibb && (o != kDuct || a.duct == 1)) {
        const int so = o == kDuct ? 0 : (int)o;
        const double q = so > 0 ? sphere_q3(sol, so, t, x, y, z, -kE[j][0], -kE[j][1], -kE[j][2], a)
                                : tube_q3(y, z, -kE[j][1], -kE[j][2], a);
        double v[3], r[3];
        surface_vel(sol, so, t, x - q * kE[j][0], y - q * kE[j][1], z - q * kE[j][2], a, v, r);
        const double m = 6.0 * w3(j) * a.rho0 * (kE[j][0] * v[0] + kE[j][1] * v[1] + kE[j][2] * v[2]);
        const double fo = (double)Sto<T>::ld(fin[(line * kQ + opp3(j)) * a.pitch + x]);
        const double fi = (double)Sto<T>::ld(fin[(line * kQ + j) * a.pitch + x]);
        const int xb = wrap3(x + kE[j][0], a.nx), yb = wrap3(y + kE[j][1], a.ny), zb = wrap3(z + kE[j][2], a.nz);
        const int64_t lb = (int64_t)zb * a.ny + yb;
        const bool behind = own_t[lb * a.pitch + xb] == 0;
        const double fb = behind ? (double)Sto<T>::ld(fin[(lb * kQ + opp3(j)) * a.pitch + xb]) : 0.0;
        return lbm::ibb_value<double>(q, fo, fi, fb, behind, m);
    }
    double v[3], r[3];
    surface_vel(sol, o == kDuct ? 0 : (int)o, t, x - 0.5 * kE[j][0], y - 0.5 * kE[j][1], z - 0.5 * kE[j][2], a, v, r);
    return (double)Sto<T>::ld(fin[(line * kQ + opp3(j)) * a.pitch + x]) +
           6.0 * w3(j) * a.rho0 * (kE[j][0] * v[0] + kE[j][1] * v[1] + kE[j][2] * v[2]);
}

// Newborn refill (moving sphere `s`, one box node per thread, box around its
// centre at t + 1): a node solid at t and fluid at t + 1 takes the average
// over participating directions k (x + e_k old fluid: fluid at t and t + 1)
// of A1/A2/A3 along k of the post-advection values (falling back A1 -> A2 ->
// A3), or the equilibrium at its surface velocity when none takes part; then
// it is collided and stored with the step's output.
template <typename T>
__global__ __launch_bounds__(kBlock) void k3_refill(Ptrs p, const double* __restrict__ sol_n,
                                                    const uint8_t* __restrict__ own_n, const int* __restrict__ movers,
                                                    int chunks_per_mover, int64_t t, Args a) {
    const int m = (int)blockIdx.x / chunks_per_mover;
    const int k0 = ((int)blockIdx.x % chunks_per_mover) * kBlock + (int)threadIdx.x;
    if (k0 >= a.box * a.box * a.box) return;
    const int s = movers[m];
    double X[3];
    centre3(sol_n, s, t + 1, X);
    const double r0 = p.sol[kSolidRow * s + 3];
    const int x = (((int)floor(X[0] - r0) - 2 + k0 % a.box) % a.nx + a.nx) % a.nx;
    const int y = (((int)floor(X[1] - r0) - 2 + (k0 / a.box) % a.box) % a.ny + a.ny) % a.ny;
    const int z = (((int)floor(X[2] - r0) - 2 + k0 / (a.box * a.box)) % a.nz + a.nz) % a.nz;
    const int64_t line = (int64_t)z * a.ny + y;
    if (p.own[line * a.pitch + x] != s || own_n[line * a.pitch + x] != 0) return;
    const T* fin = (const T*)p.fin;
    double acc[kQ];
#pragma unroll
    for (int j = 0; j < kQ; ++j) acc[j] = 0.0;
    int np = 0;
    for (int k = 1; k < kQ; ++k) {
        int qx[4], qy[4], qz[4];
        bool old[4] = {false, false, false, false};
        for (int mm = 1; mm <= 3; ++mm) {
            qx[mm] = wrap3(x + mm * kE[k][0], a.nx);
            qy[mm] = wrap3(y + mm * kE[k][1], a.ny);
            qz[mm] = wrap3(z + mm * kE[k][2], a.nz);
            // x + m e_k for m <= 3 stays within one period (n >= 4)
            const int64_t q = ((int64_t)qz[mm] * a.ny + qy[mm]) * a.pitch + qx[mm];
            old[mm] = p.own[q] == 0 && own_n[q] == 0;
            if (!old[mm]) break;
        }
        if (!old[1]) continue;
        int scheme = a.refill;
        if (scheme == 0 && !(old[2] && old[3])) scheme = 1;
        if (scheme == 1 && !old[2]) scheme = 2;
        ++np;
        for (int j = 0; j < kQ; ++j) {
            const double f1 = pull3<T>(fin, p.own, p.sol, qx[1], qy[1], qz[1], j, t, a);
            double v = f1;
            if (scheme <= 1) {
                const double f2 = pull3<T>(fin, p.own, p.sol, qx[2], qy[2], qz[2], j, t, a);
                if (scheme == 1) {
                    v = 2.0 * f1 - f2;
                } else {
                    const double f3 = pull3<T>(fin, p.own, p.sol, qx[3], qy[3], qz[3], j, t, a);
                    v = 3.0 * f1 - 3.0 * f2 + f3;
                }
            }
            acc[j] += v;
        }
    }
    double d[kQ];
    if (np > 0) {
        for (int j = 0; j < kQ; ++j) d[j] = acc[j] / np;
    } else {
        double v[3], r[3];
        surface_vel(sol_n, s, t + 1, x, y, z, a, v, r);
        const double uu = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        for (int j = 0; j < kQ; ++j) {
            const double eu = kE[j][0] * v[0] + kE[j][1] * v[1] + kE[j][2] * v[2];
            d[j] = w3(j) * a.rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        }
    }
    collide3(d, a);
    T* fout = (T*)p.fout;
    for (int j = 0; j < kQ; ++j) fout[(line * kQ + j) * a.pitch + x] = Sto<T>::st(d[j]);
}

// Totals of the last step tctr[parity] - 1 after a run of steps, one
// workgroup per (solid, component).
__global__ __launch_bounds__(kBlock) void k3_finalize(const double* __restrict__ partial2,
                                                      const int* __restrict__ solid_chunk0,
                                                      double* __restrict__ hist, const int64_t* __restrict__ tctr,
                                                      int parity, Args a) {
    __shared__ double red[kBlock / 64];
    const int64_t t = tctr[parity];
    if (t < 1) return;
    finalize3(partial2 + (size_t)((t - 1) & 1) * a.nchunks * 12, solid_chunk0, hist, t - 1, (int)blockIdx.x, a,
              red);
}

// Free spheres after step t (one thread per solid slot): the step's force
// and torque of the chosen scheme, summed over the sphere's chunks in order,
// drive the explicit Newton-Euler step V' = V + (F + (M - rho0 Vol) G)/M,
// Omega' = Omega + T/I, X' = X + V' into the next parity's table; every
// other row is copied.  A free sphere that comes within 2 nodes of the duct
// or another sphere, or moves more than half a node, sets bit 1 of err.
struct FreeArgs3 {
    const double* sol_t;
    double* sol_n;
    const double* mass;       // [ns + 1][4]: M, I, Vol
    const double* partial;    // step t's chunk partials
    const double* partial_prev;  // step t - 1's (force average), or nullptr
    const int* solid_chunk0;
    int* err;
    double G[3];
    int scheme;               // 0 CME, 1 GME
};

__global__ __launch_bounds__(kBlock) void k3_free(FreeArgs3 fa, int64_t t, Args a) {
    const int s = (int)threadIdx.x;
    if (s > a.ns) return;
    const double* S = fa.sol_t + kSolidRow * s;
    double* N = fa.sol_n + kSolidRow * s;
    if (s == 0 || S[11] == 0.0) {
        for (int q = 0; q < kSolidRow; ++q) N[q] = S[q];
        return;
    }
    // with the two-step average: the mean of the totals of steps t - 1 and t
    double F[6];
    for (int q = 0; q < 6; ++q) {
        double v = 0.0;
        for (int cc = fa.solid_chunk0[s]; cc < fa.solid_chunk0[s + 1]; ++cc) v += fa.partial[cc * 12 + 6 * fa.scheme + q];
        if (fa.partial_prev) {
            double w = 0.0;
            for (int cc = fa.solid_chunk0[s]; cc < fa.solid_chunk0[s + 1]; ++cc)
                w += fa.partial_prev[cc * 12 + 6 * fa.scheme + q];
            v = 0.5 * (v + w);
        }
        F[q] = v;
    }
    const double M = fa.mass[4 * s], I = fa.mass[4 * s + 1], Vol = fa.mass[4 * s + 2];
    const double ext = M - a.rho0 * Vol;
    for (int q = 0; q < kSolidRow; ++q) N[q] = S[q];
    double speed2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        N[4 + d] = S[4 + d] + (F[d] + ext * fa.G[d]) / M;
        N[7 + d] = S[7 + d] + F[3 + d] / I;
        N[d] = S[d] + N[4 + d];
        speed2 += N[4 + d] * N[4 + d];
    }
    bool bad = speed2 > 0.25;
    const double r = S[3];
    if (a.duct == 1) {
        const double dy = N[1] - 0.5 * (a.ny - 1), dz = N[2] - 0.5 * (a.nz - 1);
        bad |= sqrt(dy * dy + dz * dz) + r > a.R - 2.0;
    } else if (a.duct == 2) {
        bad |= N[2] - r < 2.0 || N[2] + r > a.nz - 3.0;
    }
    for (int j = 1; j <= a.ns; ++j) {
        if (j == s) continue;
        double Y[3];
        centre3(fa.sol_t, j, t, Y);  // the other sphere at step t (good to a node)
        double d2 = 0.0;
        const int n3[3] = {a.nx, a.ny, a.nz};
        for (int d = 0; d < 3; ++d) {
            const double dd = min_image3(N[d] - Y[d], n3[d]);
            d2 += dd * dd;
        }
        bad |= sqrt(d2) < r + fa.sol_t[kSolidRow * j + 3] + 2.0;
    }
    if (bad) atomicOr(fa.err, 1);
}

// Pressure inlet (x = 0, density rho_in) and outlet (x = nx - 1, rho_out)
// by non-equilibrium extrapolation, on the post-collision state: the plane
// takes f_eq(rho_b, u) + (f~ - f_eq(rho, u)) of its fluid neighbour (rho, u:
// the neighbour's density and momentum over density), i.e. in deviations
// d_b = d + w_i (rho_b - rho)(1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u^2).  One
// thread per (line, side); applied to the initial state when the planes are
// set (every step applies the same rule inside the update, PR).
template <typename T>
__global__ __launch_bounds__(kBlock) void k3_pressure(T* __restrict__ f, const uint8_t* __restrict__ own, Args a,
                                                      double rho_in, double rho_out) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t lines = (int64_t)a.ny * a.nz;
    if (k >= 2 * lines) return;
    const int side = (int)(k / lines);
    const int64_t line = k % lines;
    const int xb = side == 0 ? 0 : a.nx - 1, xf = side == 0 ? 1 : a.nx - 2;
    if (own[line * a.pitch + xb] != 0 || own[line * a.pitch + xf] != 0) return;
    double d[kQ];
    double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < kQ; ++i) {
        d[i] = (double)Sto<T>::ld(f[(line * kQ + i) * a.pitch + xf]);
        drho += d[i];
        for (int c = 0; c < 3; ++c) j[c] += kE[i][c] * d[i];
    }
    const double rho = a.rho0 + drho;
    const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double dr = (side == 0 ? rho_in : rho_out) - rho;
    for (int i = 0; i < kQ; ++i) {
        const double eu = kE[i][0] * u[0] + kE[i][1] * u[1] + kE[i][2] * u[2];
        f[(line * kQ + i) * a.pitch + xb] = Sto<T>::st(d[i] + w3(i) * dr * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
    }
}

// f = f_eq(rho0, u0) at every fluid node, collided once; solid nodes zero.
template <typename T>
__global__ __launch_bounds__(kBlock) void k3_init(T* __restrict__ f, const uint8_t* __restrict__ own, Args a,
                                                  double u0x, double u0y, double u0z) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t N = (int64_t)a.ny * a.nz * a.pitch;
    if (n >= N) return;
    const int x = (int)(n % a.pitch);
    const int64_t line = n / a.pitch;
    if (x >= a.nx) return;
    double d[kQ];
    const bool fluid = own[line * a.pitch + x] == 0;
    const double uu = u0x * u0x + u0y * u0y + u0z * u0z;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const double eu = kE[i][0] * u0x + kE[i][1] * u0y + kE[i][2] * u0z;
        d[i] = w3(i) * a.rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
    if (fluid) collide3(d, a);
#pragma unroll
    for (int i = 0; i < kQ; ++i) f[(line * kQ + i) * a.pitch + x] = Sto<T>::st(fluid ? d[i] : 0.0);
}

// rho, Guo velocity (from the post-collision state: u = (sum e f~ - rho g/2)/rho)
// and owner per node, in (z, y, x) order; zeros at solid nodes.
template <typename T>
__global__ __launch_bounds__(kBlock) void k3_fields(const T* __restrict__ f, const uint8_t* __restrict__ own,
                                                    Args a, double* __restrict__ rho_out,
                                                    double* __restrict__ u_out, int32_t* __restrict__ own_out) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t N = (int64_t)a.nx * a.ny * a.nz;
    if (n >= N) return;
    const int x = (int)(n % a.nx);
    const int64_t line = n / a.nx;
    const uint8_t o = own[line * a.pitch + x];
    double r = 0.0, u[3] = {0.0, 0.0, 0.0};
    if (o == 0) {
        double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < kQ; ++i) {
            const double d = (double)Sto<T>::ld(f[(line * kQ + i) * a.pitch + x]);
            drho += d;
            for (int c = 0; c < 3; ++c) j[c] += kE[i][c] * d;
        }
        r = a.rho0 + drho;
        for (int c = 0; c < 3; ++c) u[c] = (j[c] - 0.5 * r * a.g[c]) / r;
    }
    if (rho_out) rho_out[n] = r;
    if (u_out)
        for (int c = 0; c < 3; ++c) u_out[c * N + n] = u[c];
    if (own_out) own_out[n] = o;
}

__global__ void k3_set_counters(int64_t* tctr, int64_t t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        tctr[0] = t;
        tctr[1] = t;
    }
}

}  // namespace lbm3
