// lbm_kernels.h -- HIP kernels of the D2Q9 momentum-exchange hot path.
//
// State convention: the workspace holds the post-collision deviations
// d~_i(x, t) = f~_i(x, t) - w_i rho0 of every fluid node of geometry G_t, SoA
// [9][ny][pitch], in two ping-pong buffers selected by the parity of t.  One
// time step t -> t+1 is one launch of k_fused whose workgroups take one of
// three roles; the roles read only step-t data and write disjoint outputs,
// so they run concurrently:
//   force      Eqs. 4-7 on the link lists of G_t (reads f~(t)), chunked over
//              workgroups, with a fixed-order final sum per solid
//   move       per translating body: owner map of G_{t+1} in its swept box,
//              its link list for G_{t+1} (into the other link buffer), and the
//              refill of its newborn nodes (solid in G_t, fluid in G_{t+1}),
//              extrapolated from old-fluid neighbours' post-advection values
//              and collided
//   step       pull-advection (Eq. 3) with half-way bounce-back on G_t, then
//              collision (Eq. 2), for every node fluid in G_t (a node covered
//              by a body at t+1 is written too and never read again)
#pragma once

#include "lbm_device.h"

namespace lbm {

constexpr int kBlock = 256;
constexpr int kMaxSolids = 254;

// Population layout: element (i, y, x) at i*istride + y*ystride + x.  The
// library uses the row-interleaved layout istride = rowlen, ystride =
// 9*rowlen (the nine population rows of lattice row y are contiguous), which
// keeps the 18 streams of the update kernel within a few DRAM pages.
struct StepArgs {
    int nx, ny;
    int rowlen;        // padded row length in elements (multiple of 64)
    int opitch;        // bytes per owner-map row
    int64_t istride;   // elements between populations i and i+1 of a node
    int64_t ystride;   // elements between rows y and y+1
    int walls;
    double rho0;
    int ibb = 0;       // interpolated bounce-back on body links
    // 16-bit storage: bytes from the start of a population buffer to its
    // float array of FP32 populations of the nodes next to a solid (the same
    // for both buffers; element e of a buffer <-> float element e there),
    // and to its reference table (kSeg floats of the reference equilibrium per
    // kRefNodes-node row segment, nseg segments per row)
    int64_t side_off = 0;
    int64_t ref_off = 0;
    int nseg = 0;
};

// ------------------------------------------------------------------ split storage
// 16-bit storage keeps the FP32 arithmetic's result on two scales.  The
// populations of a node next to a solid are kept in FP32 (their 16-bit
// slots hold the storage type's marker).  Every other node stores, per
// direction, its deviation from a reference equilibrium of its 16-node row
// segment, w_i (drho_s + 3 e_i . u_s) with (drho_s, u_s) the segment's mean
// density deviation and Guo velocity, written by the segment's update beside
// the populations; rounding then acts on the departure from the local flow,
// not on the flow itself (round to nearest even of f_i - w_i rho0 biases the
// momentum of a slowly accelerating flow by ~1e-2 over thousands of steps).
constexpr int kRefShift = 4;            // 16 nodes per reference segment
constexpr int kRefNodes = 1 << kRefShift;
constexpr int kSeg = 9;                 // floats per segment: the nine r_i

template <typename T>
__device__ inline const float* side_of(const T* base, int64_t side_off) {
    return reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + side_off);
}
template <typename T>
__device__ inline float* side_of(T* base, int64_t side_off) {
    return reinterpret_cast<float*>(reinterpret_cast<char*>(base) + side_off);
}
// reference of direction i for node (x, y): table[(y nseg + x / 16) 9 + i]
__device__ inline int64_t ref_index(int nseg, int i, int x, int y) {
    return ((int64_t)y * nseg + (x >> kRefShift)) * kSeg + i;
}

// Deviation f_i - w_i rho0 of direction i at node (x, y) of the population
// buffer base (A: any argument block with istride, ystride, side_off, ref_off
// and nseg).
template <typename T, typename A>
__device__ inline typename Sto<T>::C pop_at(const T* base, const A& a, int i, int x, int y) {
    using C = typename Sto<T>::C;
    const int64_t e = (int64_t)i * a.istride + (int64_t)y * a.ystride + x;
    const T v = base[e];
    if constexpr (Sto<T>::kSplit) {
        if (Sto<T>::marked(v)) return (C)side_of(base, a.side_off)[e];
        return Sto<T>::ld(v) + (C)side_of(base, a.ref_off)[ref_index(a.nseg, i, x, y)];
    }
    return Sto<T>::ld(v);
}

// Store of a node next to a solid (any storage type; 16-bit storage keeps
// it in FP32), direction i at (x, y).
template <typename T, typename A>
__device__ inline void st_near(T* base, const A& a, int i, int x, int y, typename Sto<T>::C v) {
    const int64_t e = (int64_t)i * a.istride + (int64_t)y * a.ystride + x;
    if constexpr (Sto<T>::kSplit) {
        side_of(base, a.side_off)[e] = (float)v;
        base[e] = Sto<T>::mark();
    } else {
        base[e] = Sto<T>::st(v);
    }
}

// Sum of v over the 16 lanes of a DPP row (an aligned quarter of the wave),
// the same in every lane: four rotate-and-add steps within the row, each
// adding two partial sums of the same lanes (every lane of the row must be
// active).
__device__ inline float row16_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));  // ror 8
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xf, 0xf, false));  // ror 4
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x122, 0xf, 0xf, false));  // ror 2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x121, 0xf, 0xf, false));  // ror 1
    return v;
}

// The nine reference deviations w_i (drho + 3 e_i . u) of a segment, written
// per direction so that no product with a zero velocity component is formed
// (the compiler may not drop 0 * u_x, which is not an identity for every
// float): one fused multiply-add per direction.
__device__ inline void ref_eq(float drho, float ux, float uy, float r[9]) {
    const float w0 = w_<float>(0), w1 = w_<float>(1), w5 = w_<float>(5);
    const float a = 3.0f * ux, b = 3.0f * uy, p = a + b, m = b - a;
    const float d1 = w1 * drho, d5 = w5 * drho;
    r[0] = w0 * drho;
    r[1] = __builtin_fmaf(w1, a, d1);
    r[3] = __builtin_fmaf(-w1, a, d1);
    r[2] = __builtin_fmaf(w1, b, d1);
    r[4] = __builtin_fmaf(-w1, b, d1);
    r[5] = __builtin_fmaf(w5, p, d5);
    r[7] = __builtin_fmaf(-w5, p, d5);
    r[6] = __builtin_fmaf(w5, m, d5);
    r[8] = __builtin_fmaf(-w5, m, d5);
}

// A fluid node with a solid neighbour (or a wall row) in the owner map.
__device__ inline bool next_to_solid(const uint8_t* __restrict__ own, const StepArgs& a, int x, int y) {
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        int xs = x + ex_(i), ys = y + ey_(i);
        xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
        if (ys < 0 || ys >= a.ny) {
            if (a.walls) return true;
            ys = ys < 0 ? ys + a.ny : ys - a.ny;
        }
        if (own[(int64_t)ys * a.opitch + xs] != 0) return true;
    }
    return false;
}

// ------------------------------------------------------------------ step
// Streaming memory access: every population is read once and written once per
// step, so both directions bypass cache retention (nontemporal hint).
// NT = false keeps ordinary loads and stores (a working set that fits the
// 256 MB Infinity Cache is better served from it).
template <bool NT, typename T>
__device__ inline T ld_stream(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ inline bf16_t ld_stream(const bf16_t* p) {
    bf16_t r;
    if constexpr (NT) r.bits = __builtin_nontemporal_load(&p->bits);
    else r.bits = p->bits;
    return r;
}
template <bool NT, typename T>
__device__ inline void st_stream(T* p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
template <bool NT>
__device__ inline void st_stream(bf16_t* p, bf16_t v) {
    if constexpr (NT) __builtin_nontemporal_store(v.bits, &p->bits);
    else p->bits = v.bits;
}

// Element idx of a row that starts at a wave-uniform base, with the byte
// offset formed in 32 bits (rows are far below 4 GiB): the load or store
// then takes the scalar base plus a 32-bit vector offset.
template <typename T>
__device__ inline const T* row_at(const T* base, uint32_t idx) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ inline T* row_at(T* base, uint32_t idx) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(T));
}

// One thread per node, each wave 64 consecutive nodes of one row.  The nine
// pull loads of the interior case are issued together with the owner loads;
// only when a source node is solid (or a wall row) are they replaced by the
// per-direction bounce-back values.  bid/nblk: this workgroup's index among
// the update workgroups (remapped so that each XCD walks a contiguous band).
// The body whose link list a boundary workgroup walks: its record, centre
// and spin at the step, loaded once per workgroup (a node's links into
// another body look that one up).
struct BndSolid {
    SolidDev S;
    double X, Y, om;
    int s;
};

// Source rows and columns of node (x, y): x -/+ 1 periodic; y -/+ 1 periodic,
// or, with walls at y, the node's own row where the source row is a wall.
__device__ inline void sources(int x, int y, const StepArgs& a, int& xm, int& xp, int& ym, int& yp, bool& wall_lo,
                               bool& wall_hi) {
    xm = x == 0 ? a.nx - 1 : x - 1;
    xp = x == a.nx - 1 ? 0 : x + 1;
    wall_lo = false;
    wall_hi = false;
    if (a.walls) {
        wall_lo = (y == 0);
        wall_hi = (y == a.ny - 1);
        ym = wall_lo ? y : y - 1;
        yp = wall_hi ? y : y + 1;
    } else {
        ym = y == 0 ? a.ny - 1 : y - 1;
        yp = y == a.ny - 1 ? 0 : y + 1;
    }
}

// ---- 16-bit storage, update role.  A node's update is split into its loads
// (seg16_load) and the rest (seg16_finish), so that a lane can issue the
// loads of a second node before it updates the first.  The nodes of each
// 16-node row segment store against their segment's reference equilibrium,
// which the segment's lanes form together: every lane (also a solid one, or
// one past the row's end with lane_ok false) runs seg16_finish to its
// reference step.
template <typename T>
struct Seg16In {
    T raw[9];        // streamed populations, as stored
    float rr[9];     // reference of each source's segment
    uint32_t self;   // owner of the node
    uint32_t nb;     // OR of the owners of the eight sources
    int x, xr;       // column (clamped into the lattice), the lane's own column
    bool lane_ok;
};

template <typename T, bool NT>
__device__ inline void seg16_load(Seg16In<T>& L, int x, int y, const T* __restrict__ fin,
                                  const uint8_t* __restrict__ own_t, const StepArgs& a, bool lane_ok) {
    L.xr = x;
    L.lane_ok = lane_ok;
    if (!lane_ok) x = a.nx - 1;  // addresses stay in the lattice
    L.x = x;
    int xm, xp, ym, yp;
    bool wall_lo, wall_hi;
    sources(x, y, a, xm, xp, ym, yp, wall_lo, wall_hi);
    // wave-uniform row bases, unsigned 32-bit lane offsets
    const uint32_t ux = (uint32_t)x, uxm = (uint32_t)xm, uxp = (uint32_t)xp;
    const uint8_t* om = own_t + (int64_t)ym * a.opitch;
    const uint8_t* o0 = own_t + (int64_t)y * a.opitch;
    const uint8_t* op = own_t + (int64_t)yp * a.opitch;
    L.self = o0[ux];
    L.nb = (uint32_t)o0[uxm] | o0[uxp] | om[ux] | om[uxm] | om[uxp] | op[ux] | op[uxp] | op[uxm];
    const int64_t P = a.istride;
    const T* r0 = fin + (int64_t)y * a.ystride;
    const T* rm = fin + (int64_t)ym * a.ystride;
    const T* rp = fin + (int64_t)yp * a.ystride;
    L.raw[0] = ld_stream<NT>(row_at(r0, ux));
    L.raw[1] = ld_stream<NT>(row_at(r0 + P, uxm));
    L.raw[2] = ld_stream<NT>(row_at(rm + 2 * P, ux));
    L.raw[3] = ld_stream<NT>(row_at(r0 + 3 * P, uxp));
    L.raw[4] = ld_stream<NT>(row_at(rp + 4 * P, ux));
    L.raw[5] = ld_stream<NT>(row_at(rm + 5 * P, uxm));
    L.raw[6] = ld_stream<NT>(row_at(rm + 6 * P, uxp));
    L.raw[7] = ld_stream<NT>(row_at(rp + 7 * P, uxp));
    L.raw[8] = ld_stream<NT>(row_at(rp + 8 * P, uxm));
    // the reference of each source's segment (a segment's lanes read the same words)
    const float* R = side_of(fin, a.ref_off);
    const float* Rr0 = R + (int64_t)y * a.nseg * kSeg;
    const float* Rrm = R + (int64_t)ym * a.nseg * kSeg;
    const float* Rrp = R + (int64_t)yp * a.nseg * kSeg;
    const uint32_t u0 = (uint32_t)(x >> kRefShift) * kSeg;
    const uint32_t um = (uint32_t)(xm >> kRefShift) * kSeg, uq = (uint32_t)(xp >> kRefShift) * kSeg;
    L.rr[0] = *row_at(Rr0 + 0, u0);
    L.rr[1] = *row_at(Rr0 + 1, um);
    L.rr[2] = *row_at(Rrm + 2, u0);
    L.rr[3] = *row_at(Rr0 + 3, uq);
    L.rr[4] = *row_at(Rrp + 4, u0);
    L.rr[5] = *row_at(Rrm + 5, um);
    L.rr[6] = *row_at(Rrm + 6, uq);
    L.rr[7] = *row_at(Rrp + 7, uq);
    L.rr[8] = *row_at(Rrp + 8, um);
}

// The update of the node whose loads L holds: decode, half-way bounce-back
// (GEO: rigid surface motion of spinning bodies; nodes next to a body are
// left to the boundary role under interpolated bounce-back), collide (BGK,
// or MRT when MRT), the segment's reference, store.
template <typename T, bool NT, bool MRT, bool GEO>
__device__ inline void seg16_finish(const Seg16In<T>& L, int y, const T* __restrict__ fin, T* __restrict__ fout,
                                    const uint8_t* __restrict__ own_t, const double* __restrict__ vtab,
                                    const double* __restrict__ rtab, int64_t t, const StepArgs& a,
                                    const CollideParams<float>& cp) {
    using C = float;
    const int x = L.x, xr = L.xr;
    int xm, xp, ym, yp;
    bool wall_lo, wall_hi;
    sources(x, y, a, xm, xp, ym, yp, wall_lo, wall_hi);
    const bool near = L.nb != 0u || wall_lo || wall_hi;
    // solid at t (a newborn node is refilled by the mover role), past the
    // row's end, or left to the boundary role
    bool live = L.self == 0u && L.lane_ok;
    if constexpr (GEO) live = live && !(a.ibb && L.nb != 0u);
    const int64_t P = a.istride;
    const uint32_t ux = (uint32_t)x;
    // element offsets of the rows y, y - 1, y + 1 (FP32 copies beside the buffer)
    const int64_t e0 = (int64_t)y * a.ystride, em = (int64_t)ym * a.ystride, ep = (int64_t)yp * a.ystride;
    C d[9];
    Moments<C> mo{};
    Moments<C> m0;
    if (live) {
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = Sto<T>::ld_add(L.raw[i], L.rr[i]);
        m0 = moments<C>(d, cp);
    }
    // A source next to a solid holds its FP32 populations in the side array
    // and a marker, a NaN pattern, in its slot: the decoded density sum is
    // NaN exactly then (or for a state that has blown up), so one test finds
    // the nodes that need the side array or the bounce-back
    if (live && (near || __builtin_isnan(m0.drho))) {
        bool mk[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) mk[i] = Sto<T>::marked(L.raw[i]);
        if (mk[0] | mk[1] | mk[2] | mk[3] | mk[4] | mk[5] | mk[6] | mk[7] | mk[8]) {
            const float* sd = side_of(fin, a.side_off);
            if (mk[0]) d[0] = sd[e0 + x];
            if (mk[1]) d[1] = sd[e0 + P + xm];
            if (mk[2]) d[2] = sd[em + 2 * P + x];
            if (mk[3]) d[3] = sd[e0 + 3 * P + xp];
            if (mk[4]) d[4] = sd[ep + 4 * P + x];
            if (mk[5]) d[5] = sd[em + 5 * P + xm];
            if (mk[6]) d[6] = sd[em + 6 * P + xp];
            if (mk[7]) d[7] = sd[ep + 7 * P + xp];
            if (mk[8]) d[8] = sd[ep + 8 * P + xm];
        }
        if (near) {
            // half-way bounce-back for the directions whose source is solid or
            // a wall row: the node's own opposite population plus the
            // moving-wall term; the owners are read again here (cached)
            const uint8_t* om = own_t + (int64_t)ym * a.opitch;
            const uint8_t* o0 = own_t + (int64_t)y * a.opitch;
            const uint8_t* op = own_t + (int64_t)yp * a.opitch;
            const uint32_t src[9] = {0u, o0[xm], om[x], o0[xp], op[x], om[xm], om[xp], op[xp], op[xm]};
            // the node's own population of direction j: FP32 beside the buffer
            // when it was stored next to a solid, else against its segment's
            // reference (a node that a moving body has just come next to)
            const T* r0 = fin + e0;
            const float* Rr0 = side_of(fin, a.ref_off) + (int64_t)y * a.nseg * kSeg;
            const uint32_t u0 = (uint32_t)(x >> kRefShift) * kSeg;
            auto own_pop = [&](int j) -> C {
                const T v = *row_at(r0 + j * P, ux);
                if (Sto<T>::marked(v)) return side_of(fin, a.side_off)[e0 + j * P + x];
                return Sto<T>::ld_add(v, *row_at(Rr0 + j, u0));
            };
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const bool wall = (ey_(i) == 1 && wall_lo) || (ey_(i) == -1 && wall_hi);
                const uint32_t sid = wall ? 0u : src[i];
                if (wall || sid != 0u) {
                    C vx = (C)vtab[2 * sid], vy = (C)vtab[2 * sid + 1];
                    if constexpr (GEO) {
                        const double om_ = rtab[kRot * sid];
                        if (om_ != 0.0) {
                            const double rx = min_image((double)x - 0.5 * ex_(i) - rtab[kRot * sid + 1], a.nx);
                            double ry = (double)y - 0.5 * ey_(i) - rtab[kRot * sid + 2];
                            if (!a.walls) ry = min_image(ry, a.ny);
                            vx = (C)((double)vtab[2 * sid] - om_ * ry);
                            vy = (C)((double)vtab[2 * sid + 1] + om_ * rx);
                        }
                    }
                    d[i] = own_pop(opp_(i)) + C(6) * w_<C>(i) * (C)a.rho0 * (C(ex_(i)) * vx + C(ey_(i)) * vy);
                }
            }
        }
        m0 = moments<C>(d, cp);
    }
    if (live) {
        if constexpr (MRT)
            collide_mrt<C>(d, cp, &mo, &m0);
        else
            collide<C>(d, cp, &mo, &m0);
    }
    // the segment's reference: w_i (drho_s + 3 e_i . u_s) from the means over
    // its live nodes (16 lanes, an aligned quarter of the wave)
    const float sr = row16_sum(live ? mo.drho : 0.0f);
    const float sx = row16_sum(live ? mo.ux : 0.0f);
    const float sy = row16_sum(live ? mo.uy : 0.0f);
    // live lanes of the segment (any reference serves, as long as the table
    // holds the one the stores subtract: the reciprocal need not be exact)
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t grp = (uint32_t)(__ballot(live) >> (lane & ~(uint32_t)(kRefNodes - 1))) & 0xffffu;
    const float inv = grp != 0u ? __builtin_amdgcn_rcpf((float)__builtin_popcount(grp)) : 0.0f;
    float r[9];
    ref_eq(sr * inv, sx * inv, sy * inv, r);
    // lanes 0..8 of the segment record it for the readers of the next step
    // (segments of the padded row only)
    const uint32_t j = (uint32_t)xr & (kRefNodes - 1);
    if (j < (uint32_t)kSeg && ((uint32_t)xr >> kRefShift) < (uint32_t)a.nseg) {
        float rj = r[0];
#pragma unroll
        for (int k = 1; k < 9; ++k) rj = j == (uint32_t)k ? r[k] : rj;
        float* Rw = side_of(fout, a.ref_off) + (int64_t)y * a.nseg * kSeg;
        *row_at(Rw, ((uint32_t)xr >> kRefShift) * kSeg + j) = rj;
    }
    if (!live) return;
    T* w0 = fout + (int64_t)y * a.ystride;
    // one scalar row base, 32-bit offsets i P + x
    if (near) {
        // a node next to a solid keeps its populations in FP32, its slots a marker
        float* sw = side_of(fout, a.side_off) + e0 + x;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            sw[i * P] = d[i];
            st_stream<NT>(row_at(w0, ux + (uint32_t)i * (uint32_t)P), Sto<T>::mark());
        }
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) st_stream<NT>(row_at(w0, ux + (uint32_t)i * (uint32_t)P), Sto<T>::st_sub(d[i], r[i]));
    }
}

template <typename T, bool NT, bool MRT = false, bool GEO = false, bool BND = false>
__device__ inline void step_node(int x, int y, const T* __restrict__ fin, T* __restrict__ fout,
                                 const uint8_t* __restrict__ own_t, const double* __restrict__ vtab,
                                 const double* __restrict__ rtab, const SolidDev* __restrict__ sol, int64_t t,
                                 const StepArgs& a, const CollideParams<typename Sto<T>::C>& cp,
                                 const BndSolid* bs = nullptr, bool lane_ok = true);

template <typename T, bool NT, bool MRT, bool GEO>
__device__ inline void step_role(uint32_t bid, uint32_t nblk, const T* __restrict__ fin,
                                 T* __restrict__ fout, const uint8_t* __restrict__ own_t,
                                 const double* __restrict__ vtab, const double* __restrict__ rtab,
                                 const SolidDev* __restrict__ sol, int64_t t, const StepArgs& a,
                                 const CollideParams<typename Sto<T>::C>& cp) {
    // row and column base are wave-uniform scalars
    const uint32_t b = xcd_remap(bid, nblk);
    const uint32_t wl = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if constexpr (Sto<T>::kSplit) {
        // 16-bit storage: each wave takes 128 consecutive x of a row, two
        // nodes per lane (x and x + 64), and issues the second node's loads
        // before the first node's update, so that a wave keeps both nodes'
        // loads in flight (the 16-bit update is bound by load latency, not
        // by bandwidth)
        const uint32_t wpr = ((uint32_t)a.rowlen + 127u) >> 7;
        const uint32_t gw = b * (kBlock / 64) + wl;
        const int y = (int)(gw / wpr);
        const int x = (int)((gw - (uint32_t)y * wpr) << 7) + (int)(threadIdx.x & 63);
        if (y >= a.ny) return;
        // (the second half of a row's last wave can lie past the padded row,
        // whose length is a multiple of 64: its lanes are not live and write
        // no reference; no branch around it, so that the counters of loads in
        // flight stay exact)
        Seg16In<T> A, B;
        seg16_load<T, NT>(A, x, y, fin, own_t, a, x < a.nx);
        // loads return in issue order: the first node's must be issued first
        // (scheduling barriers keep the two groups apart and ahead of the update)
        __builtin_amdgcn_sched_barrier(0);
        seg16_load<T, NT>(B, x + 64, y, fin, own_t, a, x + 64 < a.nx);
        __builtin_amdgcn_sched_barrier(0);
        seg16_finish<T, NT, MRT, GEO>(A, y, fin, fout, own_t, vtab, rtab, t, a, cp);
        seg16_finish<T, NT, MRT, GEO>(B, y, fin, fout, own_t, vtab, rtab, t, a, cp);
    } else {
        const uint32_t wpr = (uint32_t)a.rowlen >> 6;
        const uint32_t gw = b * (kBlock / 64) + wl;
        const int y = (int)(gw / wpr);
        const int x = (int)((gw - (uint32_t)y * wpr) << 6) + (int)(threadIdx.x & 63);
        if (y >= a.ny || x >= a.nx) return;
        step_node<T, NT, MRT, GEO>(x, y, fin, fout, own_t, vtab, rtab, sol, t, a, cp);
    }
}

// The update of node (x, y): pull, bounce-back, collide (BGK, or MRT when
// MRT), store.  GEO: body links take their surface geometry into account: a
// spinning free body moves at V + Omega z x (p - X) at the surface point p
// of the link.  Under interpolated bounce-back (a.ibb) the nodes next to a
// body are left to the boundary role (BND = true), which updates them with
// the rule of ibb_value and p = x - q e_i; otherwise p is the link midpoint.
// t is the step (centres of moving bodies).
template <typename T, bool NT, bool MRT, bool GEO, bool BND>
__device__ inline void step_node(int x, int y, const T* __restrict__ fin, T* __restrict__ fout,
                                 const uint8_t* __restrict__ own_t, const double* __restrict__ vtab,
                                 const double* __restrict__ rtab, const SolidDev* __restrict__ sol, int64_t t,
                                 const StepArgs& a, const CollideParams<typename Sto<T>::C>& cp,
                                 const BndSolid* bs, bool lane_ok) {
    using C = typename Sto<T>::C;
    if constexpr (Sto<T>::kSplit && !BND) {
        // 16-bit storage outside the boundary role: one node's loads, then its update
        Seg16In<T> L;
        seg16_load<T, NT>(L, x, y, fin, own_t, a, lane_ok);
        seg16_finish<T, NT, MRT, GEO>(L, y, fin, fout, own_t, vtab, rtab, t, a, cp);
        return;
    }
    int xm, xp, ym, yp;
    bool wall_lo, wall_hi;  // source rows y-1 / y+1 are walls
    sources(x, y, a, xm, xp, ym, yp, wall_lo, wall_hi);
    // Row bases are wave-uniform (a wave covers 64 x of one row); the lane
    // offsets are unsigned 32-bit, so every access is a scalar base plus a
    // 32-bit vector offset (no per-lane 64-bit address arithmetic).
    const uint32_t ux = (uint32_t)x, uxm = (uint32_t)xm, uxp = (uint32_t)xp;
    const uint8_t* om = own_t + (int64_t)ym * a.opitch;
    const uint8_t* o0 = own_t + (int64_t)y * a.opitch;
    const uint8_t* op = own_t + (int64_t)yp * a.opitch;
    const uint32_t self = o0[ux];
    // owners of the sources x - e_i
    const uint32_t s1 = o0[uxm], s3 = o0[uxp];
    const uint32_t s2 = om[ux], s5 = om[uxm], s6 = om[uxp];
    const uint32_t s4 = op[ux], s7 = op[uxp], s8 = op[uxm];

    const int64_t P = a.istride;
    const T* r0 = fin + (int64_t)y * a.ystride;
    const T* rm = fin + (int64_t)ym * a.ystride;
    const T* rp = fin + (int64_t)yp * a.ystride;
    T raw[9];
    raw[0] = ld_stream<NT>(row_at(r0, ux));
    raw[1] = ld_stream<NT>(row_at(r0 + P, uxm));
    raw[2] = ld_stream<NT>(row_at(rm + 2 * P, ux));
    raw[3] = ld_stream<NT>(row_at(r0 + 3 * P, uxp));
    raw[4] = ld_stream<NT>(row_at(rp + 4 * P, ux));
    raw[5] = ld_stream<NT>(row_at(rm + 5 * P, uxm));
    raw[6] = ld_stream<NT>(row_at(rm + 6 * P, uxp));
    raw[7] = ld_stream<NT>(row_at(rp + 7 * P, uxp));
    raw[8] = ld_stream<NT>(row_at(rp + 8 * P, uxm));
    // 16-bit storage: the reference of each source's segment, loaded with the
    // populations (a segment's lanes read the same words)
    C rr[9];
    // row bases of the table (wave-uniform) and 32-bit segment offsets
    const float* Rr0 = nullptr;
    uint32_t u0 = 0;
    if constexpr (Sto<T>::kSplit) {
        const float* R = side_of(fin, a.ref_off);
        Rr0 = R + (int64_t)y * a.nseg * kSeg;
        const float* Rrm = R + (int64_t)ym * a.nseg * kSeg;
        const float* Rrp = R + (int64_t)yp * a.nseg * kSeg;
        u0 = (uint32_t)(x >> kRefShift) * kSeg;
        const uint32_t um = (uint32_t)(xm >> kRefShift) * kSeg, uq = (uint32_t)(xp >> kRefShift) * kSeg;
        rr[0] = (C)*row_at(Rr0 + 0, u0);
        rr[1] = (C)*row_at(Rr0 + 1, um);
        rr[2] = (C)*row_at(Rrm + 2, u0);
        rr[3] = (C)*row_at(Rr0 + 3, uq);
        rr[4] = (C)*row_at(Rrp + 4, u0);
        rr[5] = (C)*row_at(Rrm + 5, um);
        rr[6] = (C)*row_at(Rrm + 6, uq);
        rr[7] = (C)*row_at(Rrp + 7, uq);
        rr[8] = (C)*row_at(Rrp + 8, um);
    }
    // boundary role: the node's own populations, which the interpolated rule
    // takes, are loaded with the streamed ones
    T own9[9];
    if constexpr (BND) {
#pragma unroll
        for (int i = 1; i < 9; ++i) own9[i] = ld_stream<NT>(row_at(r0 + i * P, ux));
    }
    const bool near = (s1 | s2 | s3 | s4 | s5 | s6 | s7 | s8) != 0 || wall_lo || wall_hi;
    // solid at t (a newborn node is refilled by the mover role), or left to
    // the boundary role
    bool live = self == 0u;
    if constexpr (GEO && !BND) live = live && !(a.ibb && (s1 | s2 | s3 | s4 | s5 | s6 | s7 | s8) != 0);
    if (!live) return;
    // element offsets of the rows y, y - 1, y + 1 (FP32 copies of 16-bit storage)
    const int64_t e0 = (int64_t)y * a.ystride, em = (int64_t)ym * a.ystride, ep = (int64_t)yp * a.ystride;
    C d[9];
    {
        if constexpr (Sto<T>::kSplit) {
#pragma unroll
            for (int i = 0; i < 9; ++i) d[i] = Sto<T>::ld_add(raw[i], rr[i]);
            // a source next to a solid holds its FP32 populations in the side array
            const bool m0 = Sto<T>::marked(raw[0]), m1 = Sto<T>::marked(raw[1]), m2 = Sto<T>::marked(raw[2]);
            const bool m3 = Sto<T>::marked(raw[3]), m4 = Sto<T>::marked(raw[4]), m5 = Sto<T>::marked(raw[5]);
            const bool m6 = Sto<T>::marked(raw[6]), m7 = Sto<T>::marked(raw[7]), m8 = Sto<T>::marked(raw[8]);
            if (m0 | m1 | m2 | m3 | m4 | m5 | m6 | m7 | m8) {
                const float* sd = side_of(fin, a.side_off);
                if (m0) d[0] = (C)sd[e0 + x];
                if (m1) d[1] = (C)sd[e0 + P + xm];
                if (m2) d[2] = (C)sd[em + 2 * P + x];
                if (m3) d[3] = (C)sd[e0 + 3 * P + xp];
                if (m4) d[4] = (C)sd[ep + 4 * P + x];
                if (m5) d[5] = (C)sd[em + 5 * P + xm];
                if (m6) d[6] = (C)sd[em + 6 * P + xp];
                if (m7) d[7] = (C)sd[ep + 7 * P + xp];
                if (m8) d[8] = (C)sd[ep + 8 * P + xm];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) d[i] = Sto<T>::ld(raw[i]);
        }
        // the node's own population of direction j (bounce-back, interpolated rule)
        auto own_pop = [&](T v, int j) -> C {
            if constexpr (Sto<T>::kSplit) {
                if (Sto<T>::marked(v)) return (C)side_of(fin, a.side_off)[e0 + j * P + x];
                return Sto<T>::ld(v) + (C)*row_at(Rr0 + j, u0);
            }
            return Sto<T>::ld(v);
        };
        if (near) {
            // half-way bounce-back for the directions whose source is solid or a
            // wall row: the node's own opposite population plus the moving-wall
            // term; the loads are independent and issue together
            const uint32_t src[9] = {0u, s1, s2, s3, s4, s5, s6, s7, s8};
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const bool wall = (ey_(i) == 1 && wall_lo) || (ey_(i) == -1 && wall_hi);
                const uint32_t sid = wall ? 0u : src[i];
                if (wall || sid != 0u) {
                    C vx = (C)vtab[2 * sid], vy = (C)vtab[2 * sid + 1];
                    if constexpr (GEO && !BND) {
                        const double om = rtab[kRot * sid];
                        if (om != 0.0) {
                            const double rx = min_image((double)x - 0.5 * ex_(i) - rtab[kRot * sid + 1], a.nx);
                            double ry = (double)y - 0.5 * ey_(i) - rtab[kRot * sid + 2];
                            if (!a.walls) ry = min_image(ry, a.ny);
                            vx = (C)((double)vtab[2 * sid] - om * ry);
                            vy = (C)((double)vtab[2 * sid + 1] + om * rx);
                        }
                    }
                    if constexpr (BND) {
                        if (sid != 0u) {
                            double X = bs->X, Y = bs->Y, om = bs->om;
                            const SolidDev* B = &bs->S;
                            if ((int)sid != bs->s) {
                                solid_centre(sol, rtab, (int)sid, t, X, Y);
                                om = rtab[kRot * sid];
                                B = &sol[sid];
                            }
                            const double q = a.ibb ? link_fraction(*B, X, Y, x, y, -ex_(i), -ey_(i), a.nx, a.ny,
                                                                   a.walls)
                                                   : 0.5;
                            if (om != 0.0) {
                                const double rx = min_image((double)x - q * ex_(i) - X, a.nx);
                                double ry = (double)y - q * ey_(i) - Y;
                                if (!a.walls) ry = min_image(ry, a.ny);
                                vx = (C)((double)vtab[2 * sid] - om * ry);
                                vy = (C)((double)vtab[2 * sid + 1] + om * rx);
                            }
                            const C m = C(6) * w_<C>(i) * (C)a.rho0 * (C(ex_(i)) * vx + C(ey_(i)) * vy);
                            // the node behind, x + e_i, is the source of the
                            // opposite direction o; when it is fluid, d[o] still
                            // holds the value streamed from it (only directions
                            // with a solid or wall source are replaced)
                            const int o = opp_(i);
                            const bool owall = (ey_(o) == 1 && wall_lo) || (ey_(o) == -1 && wall_hi);
                            const bool behind = !owall && src[o] == 0u;
                            d[i] = ibb_value<C>(q, own_pop(own9[o], o), own_pop(own9[i], i), d[o], behind, m);
                            continue;
                        }
                    }
                    d[i] = own_pop(*row_at(r0 + opp_(i) * P, ux), opp_(i)) +
                           C(6) * w_<C>(i) * (C)a.rho0 * (C(ex_(i)) * vx + C(ey_(i)) * vy);
                }
            }
        }
        if constexpr (MRT)
            collide_mrt<C>(d, cp);
        else
            collide<C>(d, cp);
    }
    T* w0 = fout + (int64_t)y * a.ystride;
    if constexpr (Sto<T>::kSplit) {
        // the boundary role's nodes are next to a body: FP32
#pragma unroll
        for (int i = 0; i < 9; ++i) st_near<T>(fout, a, i, x, y, d[i]);
        return;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) st_stream<NT>(row_at(w0 + i * P, ux), Sto<T>::st(d[i]));
}

// ------------------------------------------------------------------ init
// Store of an initial state: a node next to a solid through st_near, every
// other one as its plain deviation (the reference table of the buffer, zeroed
// by ref_zero, holds no reference yet).
template <typename T>
__device__ inline void st_init(T* f, const uint8_t* own, const StepArgs& a, int x, int y,
                               const typename Sto<T>::C d[9]) {
    const bool near = Sto<T>::kSplit && next_to_solid(own, a, x, y);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (near)
            st_near<T>(f, a, i, x, y, d[i]);
        else
            f[(int64_t)i * a.istride + (int64_t)y * a.ystride + x] = Sto<T>::st(d[i]);
    }
}

// 16-bit storage: node (x, y) of a row (x < rowlen) zeroes its share of the
// buffer's reference table.
template <typename T>
__device__ inline void ref_zero(T* f, const StepArgs& a, int x, int y) {
    if constexpr (Sto<T>::kSplit) {
        const int j = x & (kRefNodes - 1);
        if (j < kSeg) side_of(f, a.ref_off)[ref_index(a.nseg, j, x, y)] = 0.0f;
    }
}

// f = f_eq(rho, u) at every fluid node (uniform rho0, u0 when the field
// pointers are NULL; otherwise u - g/2 from the fields so that the Guo
// velocity is u), collided once.  Solid nodes are zeroed.
template <typename T, typename FT>
__global__ __launch_bounds__(kBlock) void k_init(T* __restrict__ f, const uint8_t* __restrict__ own,
                                                 StepArgs a, CollideParams<typename Sto<T>::C> cp,
                                                 double u0x, double u0y, const FT* __restrict__ rho,
                                                 const FT* __restrict__ ux,
                                                 const FT* __restrict__ uy) {
    using C = typename Sto<T>::C;
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int y = (int)(idx / a.rowlen);
    const int x = (int)(idx - (int64_t)y * a.rowlen);
    if (y >= a.ny) return;
    ref_zero<T>(f, a, x, y);
    if (x >= a.nx) return;
    T* w0 = f + (int64_t)y * a.ystride + x;
    if (own[(int64_t)y * a.opitch + x] != 0) {
#pragma unroll
        for (int i = 0; i < 9; ++i) w0[i * a.istride] = Sto<T>::st(C(0));
        return;
    }
    C d[9];
    if (rho == nullptr) {
        feq_dev<C>((C)a.rho0, (C)a.rho0, (C)u0x, (C)u0y, d);
    } else {
        int64_t n = (int64_t)y * a.nx + x;
        feq_dev<C>((C)rho[n], (C)a.rho0, (C)ux[n] - C(0.5) * cp.gx, (C)uy[n] - C(0.5) * cp.gy, d);
    }
    collide_any<C>(d, cp);
    st_init<T>(f, own, a, x, y, d);
}

// f = f_eq(rho0, u_P(y) - g/2), collided once, at every fluid node: the exact
// steady plane-Poiseuille profile of BGK + Guo forcing between half-way walls,
// u_P(y) = g_x / (2 nu) (Y^2 - (y - y_c)^2) + s, Y = ny/2, y_c = (ny - 1)/2,
// s = g_x (16 Lambda - 3) / (24 nu), nu = (tau - 1/2)/3, Lambda = (tau - 1/2)^2
// for BGK and (tau - 1/2)(1/s_q - 1/2) for the MRT operator (the start a
// solve reaches without bodies).  Solid nodes are zeroed.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_poiseuille(T* __restrict__ f, const uint8_t* __restrict__ own,
                                                            StepArgs a, CollideParams<typename Sto<T>::C> cp,
                                                            double gx, double tau) {
    using C = typename Sto<T>::C;
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int y = (int)(idx / a.rowlen);
    const int x = (int)(idx - (int64_t)y * a.rowlen);
    if (y >= a.ny) return;
    ref_zero<T>(f, a, x, y);
    if (x >= a.nx) return;
    T* w0 = f + (int64_t)y * a.ystride + x;
    if (own[(int64_t)y * a.opitch + x] != 0) {
#pragma unroll
        for (int i = 0; i < 9; ++i) w0[i * a.istride] = Sto<T>::st(C(0));
        return;
    }
    const double nu = (tau - 0.5) / 3.0;
    const double Y = 0.5 * a.ny, yc = 0.5 * (a.ny - 1), dy = y - yc;
    // wall slip of the two-rate solution: Lambda = (1/omega - 1/2)(1/s_q - 1/2),
    // (tau - 1/2)^2 for BGK
    const double lam = (tau - 0.5) * (cp.mrt ? 1.0 / (double)cp.s_q - 0.5 : tau - 0.5);
    const double slip = gx * (16.0 * lam - 3.0) / (24.0 * nu);
    const double u = gx / (2.0 * nu) * (Y * Y - dy * dy) + slip;
    C d[9];
    feq_dev<C>((C)a.rho0, (C)a.rho0, (C)(u - 0.5 * gx), (C)(-0.5 * (double)cp.gy), d);
    collide_any<C>(d, cp);
    st_init<T>(f, own, a, x, y, d);
}

// ------------------------------------------------------------------ fields
// rho and the Guo velocity of the pre-collision state f(t), from the stored
// post-collision populations: collision keeps mass and adds rho*g to the
// momentum, so rho*u = sum e_i f~_i - rho*g/2.
template <typename T, typename OT>
__global__ __launch_bounds__(kBlock) void k_fields(const T* __restrict__ f,
                                                   const uint8_t* __restrict__ own, StepArgs a,
                                                   double gx, double gy, OT* __restrict__ rho_o,
                                                   OT* __restrict__ ux_o, OT* __restrict__ uy_o,
                                                   uint8_t* __restrict__ own_o,
                                                   int* __restrict__ errflag) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int y = (int)(idx / a.rowlen);
    const int x = (int)(idx - (int64_t)y * a.rowlen);
    if (y >= a.ny || x >= a.nx) return;
    const int64_t n = (int64_t)y * a.nx + x;
    const uint8_t o = own[(int64_t)y * a.opitch + x];
    double r = 0.0, ux = 0.0, uy = 0.0;
    if (o == 0) {
        double d[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = (double)pop_at(f, a, i, x, y);
        double drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
        r = a.rho0 + drho;
        double jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
        double jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
        ux = jx / r - 0.5 * gx;
        uy = jy / r - 0.5 * gy;
        if (!(r > 0.0) || !isfinite(r) || !isfinite(ux) || !isfinite(uy)) atomicOr(errflag, 2);
    }
    if (rho_o) rho_o[n] = (OT)r;
    if (ux_o) ux_o[n] = (OT)ux;
    if (uy_o) uy_o[n] = (OT)uy;
    if (own_o) own_o[n] = o;
}

// Absolute post-collision populations in double, [9][ny][nx]; 0 at solids.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_populations(const T* __restrict__ f,
                                                        const uint8_t* __restrict__ own,
                                                        StepArgs a, double* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int y = (int)(idx / a.rowlen);
    const int x = (int)(idx - (int64_t)y * a.rowlen);
    if (y >= a.ny || x >= a.nx) return;
    const bool fl = own[(int64_t)y * a.opitch + x] == 0;
    const int64_t nn = (int64_t)a.nx * a.ny;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        double v = fl ? w_<double>(i) * a.rho0 + (double)pop_at(f, a, i, x, y) : 0.0;
        out[i * nn + (int64_t)y * a.nx + x] = v;
    }
}

// ------------------------------------------------------------------ geometry
struct GeomArgs {
    int nx, ny, opitch, walls;
};

// Clear an owner map (fill kernel: graph-safe, no memset node).
__global__ void k_fill_u8(uint8_t* __restrict__ p, int64_t n, uint8_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Rasterise solids list[blockIdx.x] at step t into own (one workgroup per
// solid; the bodies do not overlap, so every node is written by one solid).
__global__ __launch_bounds__(kBlock) void k_raster(uint8_t* __restrict__ own,
                                                   const SolidDev* __restrict__ sol,
                                                   const int* __restrict__ list, int64_t t,
                                                   GeomArgs g) {
    const int s = list[blockIdx.x];
    const SolidDev S = sol[s];
    double X, Y;
    solid_pos(S, t, X, Y);
    long x0, x1, y0, y1;
    solid_range(S, X, Y, 1, x0, x1, y0, y1);
    const long W = x1 - x0 + 1, H = y1 - y0 + 1;
    for (long q = threadIdx.x; q < W * H; q += kBlock) {
        long yy = y0 + q / W, xx = x0 + q % W;
        if (!solid_inside(S, X, Y, xx, yy)) continue;
        if (g.walls && (yy < 0 || yy >= g.ny)) continue;
        own[(int64_t)wrapi(yy, g.ny) * g.opitch + wrapi(xx, g.nx)] = (uint8_t)s;
    }
}

// ------------------------------------------------------------------ links
// Link code: (y*nx + x) << 4 | i, for a fluid node x_f and direction i whose
// neighbour x_f + e_i is solid.
struct LinkArgs {
    int nx, ny, opitch, walls;
};

// Wall links (solid 0): rows 0 and ny-1 are always fluid (bodies keep a gap
// to the walls); row 0 links to the wall through i = 4, 7, 8 and row ny-1
// through i = 2, 5, 6.  Order (y, x, i).
__global__ void k_wall_links(uint32_t* __restrict__ links, int nx, int ny) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * nx) return;
    int top = k >= nx;
    int x = top ? k - nx : k;
    int y = top ? ny - 1 : 0;
    uint32_t node = (uint32_t)y * (uint32_t)nx + (uint32_t)x;
    uint32_t* L = links + 3 * k;
    if (!top) {
        L[0] = node << 4 | 4u;
        L[1] = node << 4 | 7u;
        L[2] = node << 4 | 8u;
    } else {
        L[0] = node << 4 | 2u;
        L[1] = node << 4 | 5u;
        L[2] = node << 4 | 6u;
    }
}

// Block-wide exclusive scan of one int per thread (kBlock threads): an
// inclusive scan inside each wavefront by shuffles, then the wave totals
// through LDS (two barriers; sh needs kBlock / 64 ints).
__device__ inline int block_exclusive_scan(int v, int* sh, int& total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const int tw = sh[w];
        pre += w < wave ? tw : 0;
        tot += tw;
    }
    total = tot;
    __syncthreads();  // sh may be reused by the caller
    return pre + x - v;
}

// Build the link list of solid s from owner map own over its bounding range
// at step t.  Each thread takes a contiguous run of the range's nodes, so the
// scan keeps row-major (y, x, i) order.
__device__ inline void build_links_block(const uint8_t* __restrict__ own, uint32_t* __restrict__ links,
                                         int* __restrict__ seg_cnt, const int* __restrict__ seg_off,
                                         const int* __restrict__ seg_cap, const SolidDev& S, int s,
                                         int64_t t, const LinkArgs& g, int* __restrict__ errflag,
                                         int* sh) {
    double X, Y;
    solid_pos(S, t, X, Y);
    long x0, x1, y0, y1;
    solid_range(S, X, Y, 2, x0, x1, y0, y1);
    if (x1 - x0 + 1 > g.nx) { x0 = 0; x1 = g.nx - 1; }
    if (!g.walls && y1 - y0 + 1 > g.ny) { y0 = 0; y1 = g.ny - 1; }
    if (g.walls) { y0 = y0 < 0 ? 0 : y0; y1 = y1 >= g.ny ? g.ny - 1 : y1; }
    const long W = x1 - x0 + 1, H = y1 - y0 + 1, N = W * H;
    const long chunk = (N + kBlock - 1) / kBlock;
    const long q0 = (long)threadIdx.x * chunk;
    const long q1 = q0 + chunk < N ? q0 + chunk : N;
    auto links_of = [&](long q, uint32_t* out, int base) -> int {
        long yy = y0 + q / W, xx = x0 + q % W;
        int x = wrapi(xx, g.nx), y = wrapi(yy, g.ny);
        if (own[(int64_t)y * g.opitch + x] != 0) return 0;
        int c = 0;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            int yn = y + ey_(i);
            if (g.walls && (yn < 0 || yn >= g.ny)) continue;
            int xn = wrapi(x + ex_(i), g.nx);
            yn = wrapi(yn, g.ny);
            if (own[(int64_t)yn * g.opitch + xn] == s) {
                if (out) out[base + c] = ((uint32_t)y * (uint32_t)g.nx + (uint32_t)x) << 4 | (uint32_t)i;
                ++c;
            }
        }
        return c;
    };
    int cnt = 0;
    for (long q = q0; q < q1; ++q) cnt += links_of(q, nullptr, 0);
    int total;
    int off = block_exclusive_scan(cnt, sh, total);
    const int cap = seg_cap[s];
    uint32_t* L = links + seg_off[s];
    if (total <= cap) {
        for (long q = q0; q < q1; ++q) off += links_of(q, L, off);
    }
    if (threadIdx.x == 0) {
        seg_cnt[s] = total <= cap ? total : 0;
        if (total > cap) atomicOr(errflag, 1);
    }
}

__global__ __launch_bounds__(kBlock) void k_links(const uint8_t* __restrict__ own,
                                                  uint32_t* __restrict__ links,
                                                  int* __restrict__ seg_cnt,
                                                  const int* __restrict__ seg_off,
                                                  const int* __restrict__ seg_cap,
                                                  const SolidDev* __restrict__ sol,
                                                  const int* __restrict__ list, int64_t t,
                                                  LinkArgs g, int* __restrict__ errflag) {
    __shared__ int sh[kBlock];
    const int s = list[blockIdx.x];
    build_links_block(own, links, seg_cnt, seg_off, seg_cap, sol[s], s, t, g, errflag, sh);
}

// ------------------------------------------------------------------ movers
// Two workgroups per translating body s, which run side by side: part 0
// writes G_{t+1} into the second owner map and rebuilds the body's link
// list, part 1 refills the newborn nodes.  Both stage the body's swept range
// from t-1 to t+1, widened by kBoxMargin nodes, in LDS as two byte maps: ot
// (owners of G_t) and on (the second owner map, G_{t-1} on entry, then
// G_{t+1} as both parts rasterise the body at t+1 the same way).  Part 1 may
// stage a node after part 0 has rewritten it; rasterising G_{t+1} over it
// again gives the same value, so neither part depends on the other's
// timing.  Virtual wall rows are marked kWallMark.  Translating
// bodies keep a gap of at least kMoverGap nodes to each other, so no other
// body's workgroups change an owner that these read.
constexpr int kBoxMargin = 5;
constexpr uint8_t kWallMark = 255;
constexpr int kMoverGap = 8;
constexpr int kNewbornBatch = 4;   // newborn nodes refilled together
constexpr int kNewbornMax = 128;   // newborn nodes of one body in one step

struct MoveArgs {
    int nx, ny, opitch, walls;
    int64_t istride, ystride;
    double rho0;
    int refill;     // 0 A1, 1 A2, 2 A3
    int box_bytes;  // capacity of each LDS byte map
    int n_movers;   // translating bodies (mover workgroups: 2 n_movers)
    int ibb = 0;    // interpolated bounce-back on body links
    int64_t side_off = 0;  // 16-bit storage: FP32 side array and reference
    int64_t ref_off = 0;   // table (as in StepArgs)
    int nseg = 0;
};

// Bounding range of the body centred at (Xa, Ya) (step t - 1) and at
// (Xb, Yb) (step t + 1), widened by kBoxMargin.
__device__ inline void swept_box(const SolidDev& S, double Xa, double Ya, double Xb, double Yb, long& x0, long& x1,
                                 long& y0, long& y1) {
    long ax0, ax1, ay0, ay1, bx0, bx1, by0, by1;
    solid_range(S, Xa, Ya, kBoxMargin, ax0, ax1, ay0, ay1);
    solid_range(S, Xb, Yb, kBoxMargin, bx0, bx1, by0, by1);
    x0 = ax0 < bx0 ? ax0 : bx0;
    x1 = ax1 > bx1 ? ax1 : bx1;
    y0 = ay0 < by0 ? ay0 : by0;
    y1 = ay1 > by1 ? ay1 : by1;
}

// Free-body mover arguments (one launch after the step: the step's force
// partials are complete).
struct FreeArgs {
    FreeDyn* dyn;               // [n_free], in the order of the mover list
    const double* partial;      // step t's force partials [nchunks][6]
    const int* solid_chunk0;    // chunk range of each solid
    const double* rtab;         // rotation table of step t
    double* vtab_next;          // velocity table of step t + 1
    double* rtab_next;          // rotation table of step t + 1
    double Gx, Gy, rho0;        // gravity on free bodies, reference density
    int scheme;                 // force that drives them: 0 CME, 1 GME
};

template <typename T>
struct MoveShared {
    using C = typename Sto<T>::C;
    SolidDev body;  // the mover's record (kept here rather than in registers)
    int scan[kBlock];
    int nb_count;
    int nb_list[kNewbornMax];
    int8_t nb_use[kNewbornBatch][8];  // -1: no participation, else 0/1/2
    C nb_val[kNewbornBatch][8][3][9];
    C nb_new[kNewbornBatch][9];
    C nb_mom[kNewbornBatch][4];
};

// Mover role m: part m / n_movers for body movers[m % n_movers]; lds holds
// the two byte maps (2 * box_bytes).  GEO: link geometry in the refill
// stencil (spinning free bodies, interpolated bounce-back).
template <typename T, bool MRT, bool GEO>
__device__ inline void move_role(int m, uint8_t* __restrict__ lds, MoveShared<T>& sm,
                                 const T* __restrict__ fin, T* __restrict__ fout,
                                 const uint8_t* __restrict__ own_t, uint8_t* __restrict__ own_n,
                                 uint32_t* __restrict__ links_n, int* __restrict__ seg_cnt_n,
                                 const int* __restrict__ seg_off, const int* __restrict__ seg_cap,
                                 const SolidDev* __restrict__ sol, const double* __restrict__ vtab,
                                 const double* __restrict__ rt, const int* __restrict__ movers,
                                 const int64_t* __restrict__ tctr, int parity, const MoveArgs& a,
                                 const CollideParams<typename Sto<T>::C>& cp, int* __restrict__ errflag,
                                 const FreeArgs* fr = nullptr) {
    using C = typename Sto<T>::C;
    uint8_t* ot = lds;
    uint8_t* on = lds + a.box_bytes;
    const int part = m / a.n_movers;  // 0: G_{t+1} and links, 1: refill
    // uniform values, issued together (one dependent round trip for the
    // body record, kept in LDS, and its link segment)
    const int s = movers[m - part * a.n_movers];
    const int64_t t = tctr[parity];
    if (threadIdx.x == 0) sm.body = sol[s];
    const int cap = seg_cap[s];
    const int soff = seg_off[s];
    __syncthreads();
    const SolidDev& S = sm.body;
    // centres at t - 1 and t + 1; a free body first takes its Newton-Euler
    // step from the force and torque of step t (summed in chunk order, as
    // the force history is): V' = V + (F + (M - rho0 A) G)/M,
    // Omega' = Omega + T/I, X' = X + V'
    double Xa, Ya, Xn, Yn;
    double Xt = 0.0, Yt = 0.0, Vnx = 0.0, Vny = 0.0, Omn = 0.0;
    if (fr) {
        FreeDyn& D = fr->dyn[m - part * a.n_movers];
        const int k0 = (int)(t % 3), km = (int)((t + 2) % 3), kp = (int)((t + 1) % 3);
        double F[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double v = 0.0;
            for (int cc = fr->solid_chunk0[s]; cc < fr->solid_chunk0[s + 1]; ++cc)
                v += fr->partial[cc * 6 + 3 * fr->scheme + q];
            F[q] = v;
        }
        const double ext = D.M - fr->rho0 * D.A;
        Vnx = D.Vx[k0] + (F[0] + ext * fr->Gx) / D.M;
        Vny = D.Vy[k0] + (F[1] + ext * fr->Gy) / D.M;
        Omn = D.Om[k0] + F[2] / D.I;
        Xa = D.X[km];
        Ya = D.Y[km];
        Xt = D.X[k0];
        Yt = D.Y[k0];
        Xn = Xt + Vnx;
        Yn = Yt + Vny;
        if (part == 0 && threadIdx.x == 0) {
            D.X[kp] = Xn;
            D.Y[kp] = Yn;
            D.Vx[kp] = Vnx;
            D.Vy[kp] = Vny;
            D.Om[kp] = Omn;
            fr->vtab_next[2 * s] = Vnx;
            fr->vtab_next[2 * s + 1] = Vny;
            fr->rtab_next[kRot * s] = Omn;
            fr->rtab_next[kRot * s + 1] = Xn;
            fr->rtab_next[kRot * s + 2] = Yn;
            fr->rtab_next[kRot * s + 3] = 1.0;
            if (fabs(Vnx) + fabs(Vny) > 0.5) atomicOr(errflag, 8);  // outruns its swept box
        }
    } else {
        solid_pos(S, t - 1, Xa, Ya);
        solid_pos(S, t, Xt, Yt);
        solid_pos(S, t + 1, Xn, Yn);
    }
    long x0, x1, y0, y1;
    swept_box(S, Xa, Ya, Xn, Yn, x0, x1, y0, y1);
    const int W = (int)(x1 - x0 + 1), H = (int)(y1 - y0 + 1), N = W * H;
    if (N > a.box_bytes) {  // the host sizes the box for the largest mover
        if (threadIdx.x == 0) atomicOr(errflag, 4);
        return;
    }
    auto gidx = [&](int q, int& gx, int& gy) -> bool {  // box index -> lattice node
        long yy = y0 + q / W, xx = x0 + q % W;
        if (a.walls && (yy < 0 || yy >= a.ny)) return false;
        gx = wrapi(xx, a.nx);
        gy = wrapi(yy, a.ny);
        return true;
    };
    if (threadIdx.x == 0) sm.nb_count = 0;
    // 1. stage the owner maps (part 0 needs only the second one); loads of
    // a round are issued before any store
    constexpr int R = 8;
    for (int q0 = 0; q0 < N; q0 += R * kBlock) {
        uint8_t vt[R], vn[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int q = q0 + r * kBlock + threadIdx.x;
            int gx, gy;
            vt[r] = vn[r] = kWallMark;
            if (q < N && gidx(q, gx, gy)) {
                const int64_t o = (int64_t)gy * a.opitch + gx;
                if (part == 1) vt[r] = own_t[o];
                vn[r] = own_n[o];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int q = q0 + r * kBlock + threadIdx.x;
            if (q < N) {
                ot[q] = vt[r];
                on[q] = vn[r];
            }
        }
    }
    __syncthreads();
    // 2. G_{t+1}: rasterise the body at t+1, clear what it left; collect the
    // newborn nodes (solid at t, fluid at t+1); their order in the list does
    // not affect any value
    for (int q = threadIdx.x; q < N; q += kBlock) {
        const long yy = y0 + q / W, xx = x0 + q % W;
        const uint8_t v = on[q];
        const bool in = solid_inside(S, Xn, Yn, xx, yy);
        // a free body has no validated path: flag it meeting a wall or body
        if (fr && in && (v == kWallMark || (v != 0 && v != s))) atomicOr(errflag, 8);
        if (v == kWallMark) continue;
        const uint8_t nv = in ? (uint8_t)s : (v == s ? (uint8_t)0 : v);
        if (nv != v) {
            on[q] = nv;
            if (part == 0) {
                int gx, gy;
                gidx(q, gx, gy);
                own_n[(int64_t)gy * a.opitch + gx] = nv;
            }
        }
        if (part == 1 && ot[q] == s && nv == 0) {
            const int k = atomicAdd(&sm.nb_count, 1);
            if (k < kNewbornMax) sm.nb_list[k] = q;
        }
    }
    __syncthreads();
    // 3. link list of G_{t+1}, row-major (y, x, i) over the box interior
    if (part == 0) {
        const int chunk = (N + kBlock - 1) / kBlock;
        const int q0 = threadIdx.x * chunk;
        const int q1 = q0 + chunk < N ? q0 + chunk : N;
        auto links_at = [&](int q, uint32_t* out, int base) -> int {
            const int qx = q % W, qy = q / W;
            if (qx == 0 || qy == 0 || qx == W - 1 || qy == H - 1 || on[q] != 0) return 0;
            int c = 0;
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                if (on[q + ey_(i) * W + ex_(i)] == s) {
                    if (out) {
                        int gx, gy;
                        gidx(q, gx, gy);
                        out[base + c] = ((uint32_t)gy * (uint32_t)a.nx + (uint32_t)gx) << 4 | (uint32_t)i;
                    }
                    ++c;
                }
            }
            return c;
        };
        int cnt = 0;
        for (int q = q0; q < q1; ++q) cnt += links_at(q, nullptr, 0);
        int total;
        int off = block_exclusive_scan(cnt, sm.scan, total);
        if (total <= cap) {
            uint32_t* L = links_n + soff;
            for (int q = q0; q < q1; ++q) off += links_at(q, L, off);
        }
        if (threadIdx.x == 0) {
            seg_cnt_n[s] = total <= cap ? total : 0;
            if (total > cap) atomicOr(errflag, 1);
        }
        return;
    }
    // 4. refill the newborn nodes in batches, then collide and store
    const int nborn = sm.nb_count;
    if (nborn > kNewbornMax) {
        if (threadIdx.x == 0) atomicOr(errflag, 4);
        return;
    }
    const C rho0 = (C)a.rho0;
    for (int base = 0; base < nborn; base += kNewbornBatch) {
        const int nbat = nborn - base < kNewbornBatch ? nborn - base : kNewbornBatch;
        // 4a. participation and scheme per (newborn, direction)
        if (threadIdx.x < nbat * 8) {
            const int bb = threadIdx.x / 8, k = threadIdx.x % 8 + 1;
            const int qn = sm.nb_list[base + bb];
            bool ok[4] = {false, false, false, false};
            for (int mm = 1; mm <= 3; ++mm) {
                const int qm = qn + mm * (ey_(k) * W + ex_(k));
                ok[mm] = ot[qm] == 0 && on[qm] == 0;
                if (!ok[mm]) break;
            }
            int use = -1;
            if (ok[1]) {
                use = a.refill;
                if (use == 0 && !(ok[2] && ok[3])) use = 1;
                if (use == 1 && !ok[2]) use = 2;
            }
            sm.nb_use[bb][k - 1] = (int8_t)use;
        }
        __syncthreads();
        // 4b. post-advection values at the stencil nodes, in parallel
        for (int w = threadIdx.x; w < nbat * 216; w += kBlock) {
            const int bb = w / 216, r = w % 216;
            const int k = r / 27 + 1, mm = (r % 27) / 9 + 1, j = r % 9;
            const int use = sm.nb_use[bb][k - 1];
            const int need = use == 0 ? 3 : (use == 1 ? 2 : (use == 2 ? 1 : 0));
            if (mm > need) continue;
            const int qm = sm.nb_list[base + bb] + mm * (ey_(k) * W + ex_(k));
            int gx, gy;
            gidx(qm, gx, gy);
            const int qs = qm - (ey_(j) * W + ex_(j));  // source of population j
            const uint8_t o = ot[qs];
            C v;
            if (j != 0 && o != 0) {
                const int sid = o == kWallMark ? 0 : o;
                C vx = (C)vtab[2 * sid], vy = (C)vtab[2 * sid + 1];
                // surface point gx - q e_j of a body link (q = 1/2 unless
                // interpolated), step t; a spinning free body moves there at
                // V + Omega z x (point - centre)
                const C fo = pop_at(fin, a, opp_(j), gx, gy);
                double q = 0.5;
                C fi = C(0), fb = C(0);
                bool behind = false;
                if (GEO && sid != 0 && (a.ibb || fr)) {
                    if (a.ibb) {
                        // populations the rule may take, loaded before q is
                        // known: the node's own one away from the surface and
                        // the opposite one of the node behind, gx + e_j (in
                        // the box: at most 4 nodes from the newborn node, like
                        // the sources)
                        fi = pop_at(fin, a, j, gx, gy);
                        const int qb = qm + (ey_(j) * W + ex_(j));
                        int bx, by;
                        behind = ot[qb] == 0 && gidx(qb, bx, by);
                        if (behind)
                            fb = pop_at(fin, a, opp_(j), bx, by);
                    }
                    // this body's record and centre are at hand; another
                    // body's come from the tables
                    double X = Xt, Y = Yt;
                    const SolidDev* B = &S;
                    if (sid != s) {
                        solid_centre(sol, rt, sid, t, X, Y);
                        B = &sol[sid];
                    }
                    if (a.ibb) q = link_fraction(*B, X, Y, gx, gy, -ex_(j), -ey_(j), a.nx, a.ny, a.walls);
                    const double om = rt[kRot * sid];
                    if (om != 0.0) {
                        const double rx = min_image((double)gx - q * ex_(j) - X, a.nx);
                        double ry = (double)gy - q * ey_(j) - Y;
                        if (!a.walls) ry = min_image(ry, a.ny);
                        vx = (C)(vtab[2 * sid] - om * ry);
                        vy = (C)(vtab[2 * sid + 1] + om * rx);
                    }
                }
                const C mw = C(6) * w_<C>(j) * rho0 * (C(ex_(j)) * vx + C(ey_(j)) * vy);
                v = q == 0.5 ? fo + mw : ibb_value<C>(q, fo, fi, fb, behind, mw);
            } else {
                int sx, sy;
                gidx(qs, sx, sy);
                v = pop_at(fin, a, j, sx, sy);
            }
            sm.nb_val[bb][k - 1][mm - 1][j] = v;
        }
        __syncthreads();
        // 4c. extrapolate along each participating link, average
        if (threadIdx.x < nbat * 9) {
            const int bb = threadIdx.x / 9, j = threadIdx.x % 9;
            C acc = C(0);
            int np = 0;
            for (int k = 0; k < 8; ++k) {
                const int use = sm.nb_use[bb][k];
                if (use < 0) continue;
                ++np;
                const C v1 = sm.nb_val[bb][k][0][j];
                if (use == 0)
                    acc += C(3) * v1 - C(3) * sm.nb_val[bb][k][1][j] + sm.nb_val[bb][k][2][j];
                else if (use == 1)
                    acc += C(2) * v1 - sm.nb_val[bb][k][1][j];
                else
                    acc += v1;
            }
            // no participant: equilibrium at the body's velocity (a free body:
            // its surface velocity at the node at t + 1)
            C bvx = (C)S.vx, bvy = (C)S.vy;
            if (fr) {
                int nx_, ny_;
                gidx(sm.nb_list[base + bb], nx_, ny_);
                const double rx = min_image((double)nx_ - Xn, a.nx);
                double ry = (double)ny_ - Yn;
                if (!a.walls) ry = min_image(ry, a.ny);
                bvx = (C)(Vnx - Omn * ry);
                bvy = (C)(Vny + Omn * rx);
            }
            sm.nb_new[bb][j] = np > 0 ? acc / C(np) : feq_one<C>(j, rho0, rho0, bvx, bvy);
        }
        __syncthreads();
        // 4d. collide: moments per newborn node, then one direction per thread
        // (MRT: the whole node in one thread, then the stores)
        if constexpr (MRT) {
            if (threadIdx.x < nbat) {
                C dd[9];
#pragma unroll
                for (int j = 0; j < 9; ++j) dd[j] = sm.nb_new[threadIdx.x][j];
                collide_mrt<C>(dd, cp);
#pragma unroll
                for (int j = 0; j < 9; ++j) sm.nb_new[threadIdx.x][j] = dd[j];
            }
            __syncthreads();
            if (threadIdx.x < nbat * 9) {
                const int bb = threadIdx.x / 9, j = threadIdx.x % 9;
                int gx, gy;
                gidx(sm.nb_list[base + bb], gx, gy);
                st_near<T>(fout, a, j, gx, gy, sm.nb_new[bb][j]);
            }
            __syncthreads();
            continue;
        }
        if (threadIdx.x < nbat) {
            const Moments<C> mo = moments<C>(sm.nb_new[threadIdx.x], cp);
            sm.nb_mom[threadIdx.x][0] = mo.drho;
            sm.nb_mom[threadIdx.x][1] = mo.rho;
            sm.nb_mom[threadIdx.x][2] = mo.ux;
            sm.nb_mom[threadIdx.x][3] = mo.uy;
        }
        __syncthreads();
        if (threadIdx.x < nbat * 9) {
            const int bb = threadIdx.x / 9, j = threadIdx.x % 9;
            Moments<C> mo;
            mo.drho = sm.nb_mom[bb][0];
            mo.rho = sm.nb_mom[bb][1];
            mo.ux = sm.nb_mom[bb][2];
            mo.uy = sm.nb_mom[bb][3];
            const C dj = relax_one<C>(j, sm.nb_new[bb][j], mo, cp);
            int gx, gy;
            gidx(sm.nb_list[base + bb], gx, gy);
            st_near<T>(fout, a, j, gx, gy, dj);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ forces
constexpr int kForceChunk = 512;  // links per workgroup

struct ForceArgs {
    int nx, ny, walls;
    int64_t istride, ystride;
    double rho0;
    int64_t hist_cap;
    int nsol;     // bodies + 1
    int nchunks;  // force workgroups
    int opitch = 0;  // bytes per owner-map row
    int ibb = 0;     // interpolated bounce-back on body links
    int64_t side_off = 0;  // 16-bit storage: FP32 side array and reference
    int64_t ref_off = 0;   // table (as in StepArgs)
    int nseg = 0;
};

// One fluid-solid link (x_f, i) of solid s, in FP64 on full populations:
// a = f~_i(x_f) leaves towards the surface, b is the population that
// returns to x_f (the value the update streams there): half-way
// bounce-back a - m, or under interpolated bounce-back the rule of
// ibb_value with q the link fraction; (rx, ry) is the arm from the centre to
// the surface point x_f + q e_i and (vx, vy) the surface velocity there.
struct LinkEval {
    double av, bv, vx, vy, rx, ry;
};

template <typename T, bool GEO>
__device__ inline LinkEval eval_link(const T* __restrict__ f, const uint8_t* __restrict__ own_t,
                                     const SolidDev& S, double X, double Y, double vbx, double vby, double om,
                                     int s, int x, int y, int i, const ForceArgs& a) {
    const double ex = ex_(i), ey = ey_(i), w = w_<double>(i);
    double q = 0.5;
    if constexpr (GEO)
        if (a.ibb && s > 0) q = link_fraction(S, X, Y, x, y, ex_(i), ey_(i), a.nx, a.ny, a.walls);
    LinkEval L;
    L.rx = 0.0;
    L.ry = 0.0;
    if (s > 0) {
        L.rx = min_image(((double)x + q * ex) - X, a.nx);
        L.ry = ((double)y + q * ey) - Y;
        if (!a.walls) L.ry = min_image(L.ry, a.ny);
    }
    L.vx = vbx - om * L.ry;
    L.vy = vby + om * L.rx;
    L.av = w * a.rho0 + (double)pop_at(f, a, i, x, y);
    const double m = 6.0 * w * a.rho0 * (ex * L.vx + ey * L.vy);
    L.bv = L.av - m;
    if constexpr (!GEO) return L;
    if (q < 0.5) {
        // the fluid node behind, x_f - e_i (half-way when it is solid or a wall)
        int xb = x - ex_(i), yb = y - ey_(i);
        xb = xb < 0 ? xb + a.nx : (xb >= a.nx ? xb - a.nx : xb);
        bool ok = true;
        if (a.walls)
            ok = yb >= 0 && yb < a.ny;
        else
            yb = yb < 0 ? yb + a.ny : (yb >= a.ny ? yb - a.ny : yb);
        if (ok && own_t[(int64_t)yb * a.opitch + xb] == 0) {
            const double fb = w * a.rho0 + (double)pop_at(f, a, i, xb, yb);
            L.bv = 2.0 * q * L.av + (1.0 - 2.0 * q) * fb - m;
        }
    } else if (q > 0.5) {
        const double fo = w * a.rho0 + (double)pop_at(f, a, opp_(i), x, y);
        const double h = 0.5 / q;
        L.bv = h * (L.av - m) + (1.0 - h) * fo;
    }
    return L;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Chunked link forces.  Workgroup c takes links [start, start + kForceChunk)
// of solid chunk_solid[c].  Per link (x_f, i) with a = f~_i(x_f) and the
// returning population b of eval_link (half-way: b = a - 6 w_i rho0 (e_i . v)):
//   CME (Eq. 4) F = e_i a - e_ibar b
//   GME (Eq. 5) F = (e_i - v) a - (e_ibar - v) b
//   T_z (Eq. 7) = (x_s - R) x F with x_s = x_f + q e_i (q = 1/2 for half-way
//   bounce-back), R the body centre.
// Each thread sums a fixed strided subset, the wave and workgroup combine in
// a fixed tree into partial[c].  The per-solid totals are formed later, in
// chunk order, by finalize_forces (in the next launch), so no workgroup
// waits on another and the result is independent of scheduling.
struct ForceShared {
    double red[kBlock / 64][6];
};

// GEO: interpolated bounce-back may be on (a.ibb).
template <typename T, bool GEO>
__device__ inline void force_role(int c, ForceShared& fs, const T* __restrict__ f,
                                  const uint8_t* __restrict__ own_t, const uint32_t* __restrict__ links,
                                  const int* __restrict__ seg_cnt, const int* __restrict__ seg_off,
                                  const int* __restrict__ chunk_solid,
                                  const int* __restrict__ chunk_start,
                                  const SolidDev* __restrict__ sol, const double* __restrict__ vt,
                                  const double* __restrict__ rt, double* __restrict__ partial,
                                  int64_t t, const ForceArgs& a) {
    const int s = chunk_solid[c];
    const int start = chunk_start[c];
    const int n = seg_cnt[s];
    const int end = start + kForceChunk < n ? start + kForceChunk : n;
    const uint32_t* L = links + seg_off[s];
    const SolidDev S = sol[s];
    // a free body's velocity, spin and centre come from the step's tables
    const double om = rt ? rt[kRot * s] : 0.0;
    const bool fr = rt && rt[kRot * s + 3] != 0.0;
    double X = 0.0, Y = 0.0;
    if (fr) {
        X = rt[kRot * s + 1];
        Y = rt[kRot * s + 2];
    } else if (s > 0) {
        solid_pos(S, t, X, Y);
    }
    const double vbx = vt[2 * s], vby = vt[2 * s + 1];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int k = start + threadIdx.x; k < end; k += kBlock) {
        const uint32_t code = L[k];
        const int i = (int)(code & 15u);
        const uint32_t node = code >> 4;
        const int y = (int)(node / (uint32_t)a.nx);
        const int x = (int)(node - (uint32_t)y * (uint32_t)a.nx);
        const double ex = ex_(i), ey = ey_(i);
        const LinkEval le = eval_link<T, GEO>(f, own_t, S, X, Y, vbx, vby, om, s, x, y, i, a);
        const double av = le.av, bv = le.bv, vx = le.vx, vy = le.vy, rx = le.rx, ry = le.ry;
        // CME: e_i a - e_ibar b, e_ibar = -e_i
        const double cfx = ex * av + ex * bv;
        const double cfy = ey * av + ey * bv;
        // GME: (e_i - v) a - (e_ibar - v) b
        const double gfx = (ex - vx) * av - (-ex - vx) * bv;
        const double gfy = (ey - vy) * av - (-ey - vy) * bv;
        acc[0] += cfx;
        acc[1] += cfy;
        acc[3] += gfx;
        acc[4] += gfy;
        if (s > 0) {
            acc[2] += rx * cfy - ry * cfx;
            acc[5] += rx * gfy - ry * gfx;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        double v = wave_sum(acc[q]);
        if (lane == 0) fs.red[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int q = threadIdx.x;
        partial[c * 6 + q] = (fs.red[0][q] + fs.red[1][q]) + (fs.red[2][q] + fs.red[3][q]);
    }
}

// Per-solid totals of step `step` from its chunk partials, summed in chunk
// order, into the history ring (one workgroup).
__device__ inline void finalize_forces(const double* __restrict__ partial,
                                       const int* __restrict__ solid_chunk0, double* __restrict__ hist,
                                       int64_t step, const ForceArgs& a) {
    const int64_t slot = step % a.hist_cap;
    for (int r = threadIdx.x; r < a.nsol * 6; r += kBlock) {
        const int sid = r / 6, q = r % 6;
        double v = 0.0;
        for (int cc = solid_chunk0[sid]; cc < solid_chunk0[sid + 1]; ++cc) v += partial[cc * 6 + q];
        hist[(slot * a.nsol + sid) * 6 + q] = v;
    }
}

// Finalize the forces of step tctr[parity] - 1 (after the last launch of a
// batch of steps); partials of step u live in partial[(u & 1)].
__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ partial2,
                                                     const int* __restrict__ solid_chunk0,
                                                     double* __restrict__ hist,
                                                     const int64_t* __restrict__ tctr, int parity,
                                                     ForceArgs a) {
    const int64_t t = tctr[parity];
    if (t < 1) return;
    finalize_forces(partial2 + (size_t)((t - 1) & 1) * a.nchunks * 6, solid_chunk0, hist, t - 1, a);
}

// ------------------------------------------------------------------ fused step
// One launch per time step: workgroups [0, n_force) are force chunks,
// [n_force, n_force + n_move) are translating bodies, workgroup
// n_force + n_move finalizes the previous step's forces and advances the step
// counter, the next n_bnd update the nodes next to bodies under interpolated
// bounce-back, and from n_lead (a multiple of 8, so that update workgroup j sits
// on XCD j % 8) on the fused update.  The roles read only step-t data and write disjoint outputs, so
// the small latency-bound roles run alongside the bandwidth-bound update.
template <typename T>
struct StepPtrs {
    const T* fin;
    T* fout;
    const uint8_t* own_t;
    uint8_t* own_n;
    const uint32_t* links_t;
    const int* seg_cnt_t;
    uint32_t* links_n;
    int* seg_cnt_n;
    const int* seg_off;
    const int* seg_cap;
    const int* chunk_solid;
    const int* chunk_start;
    const int* solid_chunk0;
    const SolidDev* sol;
    const double* vtab;
    const double* rtab;  // rotation table of this step
    const int* movers;
    double* partial;  // [2][nchunks][6], by step parity
    double* hist;
    int64_t* tctr;
    int* errflag;
};

struct RoleCounts {
    int n_force, n_move, n_lead;
    int n_bnd = 0;  // boundary workgroups (interpolated bounce-back, two per force chunk)
};

// Boundary role (interpolated bounce-back): workgroup c takes the links of
// force chunk c; each fluid node next to a body is updated once per link
// list it appears in, by the thread holding its first link there (a node's
// links are contiguous; a node next to two bodies is updated twice with
// identical results).  Wall-only nodes stay with the update role.
template <typename T, bool MRT>
__device__ inline void boundary_role(int wg, const StepPtrs<T>& p, int64_t t, const StepArgs& a,
                                     const CollideParams<typename Sto<T>::C>& cp) {
    // two workgroups per force chunk: one link per thread
    static_assert(kForceChunk == 2 * kBlock, "a force chunk is two workgroups of links");
    const int c = wg >> 1;
    const int s = p.chunk_solid[c];
    if (s == 0) return;
    const int k = p.chunk_start[c] + (wg & 1) * kBlock + (int)threadIdx.x;
    BndSolid bs;
    bs.S = p.sol[s];
    bs.s = s;
    solid_centre(p.sol, p.rtab, s, t, bs.X, bs.Y);
    bs.om = p.rtab[kRot * s];
    const uint32_t* L = p.links_t + p.seg_off[s];
    if (k >= p.seg_cnt_t[s]) return;
    const uint32_t node = L[k] >> 4;
    if (k > 0 && (L[k - 1] >> 4) == node) return;
    const int y = (int)(node / (uint32_t)a.nx);
    const int x = (int)(node - (uint32_t)y * (uint32_t)a.nx);
    step_node<T, false, MRT, true, true>(x, y, p.fin, p.fout, p.own_t, p.vtab, p.rtab, p.sol, t, a, cp, &bs);
}

// Register budget: 64 VGPRs (8 waves per SIMD) keep the bandwidth-bound
// update at full occupancy; the geometry variant allows 128 (4 waves), since
// its boundary and refill roles would otherwise spill, and spill traffic
// lengthens their dependent chains under the update's saturated HBM.
template <typename T, bool NT, bool MRT, bool GEO>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(GEO ? 4 : (Sto<T>::kSplit ? 6 : 8), 8))) void k_fused(
    StepPtrs<T> p, int parity, RoleCounts rc, StepArgs sa, MoveArgs ma, ForceArgs fa,
    CollideParams<typename Sto<T>::C> cp) {
    extern __shared__ __align__(16) uint8_t dyn_lds[];
    __shared__ union Shared {
        ForceShared f;
        MoveShared<T> m;
    } sh;
    const int b = (int)blockIdx.x;
    if (b < rc.n_lead) {
        const int64_t t = p.tctr[parity];
        if (b < rc.n_force) {
            force_role<T, GEO>(b, sh.f, p.fin, p.own_t, p.links_t, p.seg_cnt_t, p.seg_off, p.chunk_solid, p.chunk_start,
                          p.sol, p.vtab, p.rtab, p.partial + (size_t)(t & 1) * fa.nchunks * 6, t, fa);
        } else if (b < rc.n_force + rc.n_move) {
            move_role<T, MRT, GEO>(b - rc.n_force, dyn_lds, sh.m, p.fin, p.fout, p.own_t, p.own_n, p.links_n,
                         p.seg_cnt_n, p.seg_off, p.seg_cap, p.sol, p.vtab, p.rtab, p.movers, p.tctr, parity,
                         ma, cp, p.errflag);
        } else if (b == rc.n_force + rc.n_move) {
            // previous step's totals (its partials are complete: the
            // previous launch has ended); then advance the step counter
            if (t >= 1)
                finalize_forces(p.partial + (size_t)((t - 1) & 1) * fa.nchunks * 6, p.solid_chunk0, p.hist,
                                t - 1, fa);
            if (threadIdx.x == 0) p.tctr[parity ^ 1] = t + 1;
        } else if constexpr (GEO) {
            const int c = b - (rc.n_force + rc.n_move + 1);
            if (c < rc.n_bnd) boundary_role<T, MRT>(c, p, t, sa, cp);
        }
        return;
    }
    const int64_t t = GEO ? p.tctr[parity] : 0;
    step_role<T, NT, MRT, GEO>((uint32_t)(b - rc.n_lead), gridDim.x - (uint32_t)rc.n_lead, p.fin, p.fout,
                               p.own_t, p.vtab, p.rtab, p.sol, t, sa, cp);
}

// Free bodies after the step: two workgroups per body (part 0: Newton-Euler
// step, G_{t+1} and links; part 1: the same step and rasterisation, then the
// newborn refill).  p.movers lists the free bodies.
template <typename T, bool MRT>
__global__ __launch_bounds__(kBlock) void k_free(StepPtrs<T> p, int parity, MoveArgs ma, FreeArgs fa,
                                                 CollideParams<typename Sto<T>::C> cp) {
    extern __shared__ __align__(16) uint8_t dyn_lds[];
    __shared__ MoveShared<T> sm;
    move_role<T, MRT, true>((int)blockIdx.x, dyn_lds, sm, p.fin, p.fout, p.own_t, p.own_n, p.links_n, p.seg_cnt_n,
                      p.seg_off, p.seg_cap, p.sol, p.vtab, p.rtab, p.movers, p.tctr, parity, ma, cp, p.errflag,
                      &fa);
}

// Per-link force records of the current state (test and inspection path).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_link_records(const T* __restrict__ f,
                                                         const uint8_t* __restrict__ own_t,
                                                         const uint32_t* __restrict__ links,
                                                         const int* __restrict__ seg_cnt,
                                                         const int* __restrict__ seg_off,
                                                         const int* __restrict__ rec_off,
                                                         const SolidDev* __restrict__ sol,
                                                         const double* __restrict__ vt,
                                                         const double* __restrict__ rt,
                                                         double* __restrict__ out, int64_t t, ForceArgs a) {
    const int s = blockIdx.x;
    const int n = seg_cnt[s];
    const uint32_t* Lk = links + seg_off[s];
    const double om = rt[kRot * s];
    double X = 0.0, Y = 0.0;
    if (s > 0) solid_centre(sol, rt, s, t, X, Y);
    const SolidDev S = sol[s];
    for (int k = threadIdx.x; k < n; k += kBlock) {
        const uint32_t code = Lk[k];
        const int i = (int)(code & 15u);
        const uint32_t node = code >> 4;
        const int y = (int)(node / (uint32_t)a.nx);
        const int x = (int)(node - (uint32_t)y * (uint32_t)a.nx);
        const double ex = ex_(i), ey = ey_(i);
        const LinkEval le = eval_link<T, true>(f, own_t, S, X, Y, vt[2 * s], vt[2 * s + 1], om, s, x, y, i, a);
        const double av = le.av, bv = le.bv, vx = le.vx, vy = le.vy;
        double* r = out + 8 * (int64_t)(rec_off[s] + k);
        r[0] = x;
        r[1] = y;
        r[2] = i;
        r[3] = s;
        r[4] = ex * av + ex * bv;
        r[5] = ey * av + ey * bv;
        r[6] = (ex - vx) * av - (-ex - vx) * bv;
        r[7] = (ey - vy) * av - (-ey - vy) * bv;
    }
}

// ------------------------------------------------------------------ misc
__global__ void k_set_counters(int64_t* tctr, int64_t t, int* errflag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        tctr[0] = t;
        tctr[1] = t;
        *errflag = 0;
    }
}

}  // namespace lbm
