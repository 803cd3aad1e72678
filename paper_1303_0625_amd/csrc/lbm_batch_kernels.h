// lbm_batch_kernels.h -- many independent lattices of uneven sizes advanced
// together: one launch per time step covers the update tiles of every active
// case (per-case parameters come from a device table), and every check
// interval a monitor evaluates per-case residual and force on the device and
// retires the converged cases (their state freezes).
//
// Residual of case c over its fluid nodes (u the Guo velocity):
//   r = ||u_t - u_{t-k}||_2 / (k ||u_t||_2),
// against the snapshot of the previous check, k steps earlier.
#pragma once

#include "lbm_kernels.h"

namespace lbm {

struct CaseDev {
    StepArgs sa;            // lattice shape and strides
    CollideParams<double> cp64;
    CollideParams<float> cp32;
    ForceArgs fa;           // force arguments (hist unused)
    int64_t f_off[2];       // element offsets of the two population buffers
    int64_t own_off;        // byte offset of the owner map
    int64_t snap_off;       // element offset of the velocity snapshot [2][ny][nx]
    int links_base;         // first link of the case in the global link array
    int solid_base;         // first solid record / vtab entry of the case
    int nsol;               // bodies + 1
    int chunk_first, chunk_count;  // force chunks of the case
    int wpr;                // waves per row (rowlen / 64)
    int nwaves;             // ny * wpr
};

// Update tile: `waves` consecutive waves of one case, starting at wave0.
struct Tile {
    int c;
    int wave0;
};

template <typename T>
__device__ inline const CollideParams<typename Sto<T>::C>& case_cp(const CaseDev& cd);
template <>
__device__ inline const CollideParams<double>& case_cp<double>(const CaseDev& cd) { return cd.cp64; }
template <>
__device__ inline const CollideParams<double>& case_cp<float>(const CaseDev& cd) { return cd.cp64; }
template <>
__device__ inline const CollideParams<float>& case_cp<_Float16>(const CaseDev& cd) { return cd.cp32; }
template <>
__device__ inline const CollideParams<float>& case_cp<bf16_t>(const CaseDev& cd) { return cd.cp32; }

// One time step of every listed tile; a case marked converged is skipped
// (its state stays as it was at retirement).  WAVES waves per workgroup.
template <typename T, bool NT, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_batch_step(const CaseDev* __restrict__ cases,
                                                           const Tile* __restrict__ tiles,
                                                           const int* __restrict__ converged, T* __restrict__ fbase,
                                                           const uint8_t* __restrict__ obase,
                                                           const double* __restrict__ vtab_all, int parity,
                                                           int64_t* __restrict__ tdev) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    if (blockIdx.x == 0 && threadIdx.x == 0 && tdev) tdev[parity ^ 1] = tdev[parity] + 1;
    if (converged[tl.c]) return;
    const CaseDev& cd = cases[tl.c];
    const int w = tl.wave0 + (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= cd.nwaves) return;
    const int y = w / cd.wpr;
    const int x = (w - y * cd.wpr) * 64 + (int)(threadIdx.x & 63);
    if constexpr (!Sto<T>::kSplit) {
        if (x >= cd.sa.nx) return;
    }
    step_node<T, NT>(x, y, fbase + cd.f_off[parity], fbase + cd.f_off[parity ^ 1], obase + cd.own_off,
                     vtab_all + 2 * cd.solid_base, nullptr, nullptr, 0, cd.sa, case_cp<T>(cd), nullptr, x < cd.sa.nx);
}

// Force chunks of every active case at the current state (parity).
struct BatchChunk {
    int c, s, start;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_force(const CaseDev* __restrict__ cases,
                                                        const BatchChunk* __restrict__ chunks,
                                                        const int* __restrict__ converged,
                                                        const T* __restrict__ fbase,
                                                        const uint32_t* __restrict__ links,
                                                        const int* __restrict__ seg_cnt,
                                                        const int* __restrict__ seg_off,
                                                        const SolidDev* __restrict__ sol_all,
                                                        const double* __restrict__ vtab_all,
                                                        double* __restrict__ partial, int parity,
                                                        int64_t t) {
    __shared__ ForceShared fs;
    const BatchChunk ch = chunks[blockIdx.x];
    if (converged[ch.c]) return;
    const CaseDev& cd = cases[ch.c];
    // force_role addresses the case's solids from its own base; chunk tables
    // are per case here, so pass one-element views
    const int cs = ch.s, cstart = ch.start;
    // (half-way bounce-back: the owner map is not consulted)
    force_role<T, false>(0, fs, fbase + cd.f_off[parity], nullptr, links + cd.links_base, seg_cnt + cd.solid_base,
                  seg_off + cd.solid_base, &cs, &cstart, sol_all + cd.solid_base,
                  vtab_all + 2 * cd.solid_base, nullptr, partial + (size_t)blockIdx.x * 6, t, cd.fa);
}

// Per-tile sums of |u - u_snap|^2 and |u|^2 over fluid nodes; the snapshot is
// replaced by u.
template <typename T, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_batch_monitor(const CaseDev* __restrict__ cases,
                                                              const Tile* __restrict__ tiles,
                                                              const int* __restrict__ converged,
                                                              const T* __restrict__ fbase,
                                                              const uint8_t* __restrict__ obase,
                                                              double* __restrict__ snap_base,
                                                              double* __restrict__ mon_partial,
                                                              int parity) {
    __shared__ double red[WAVES][2];
    const Tile tl = tiles[blockIdx.x];
    double dd = 0.0, uu = 0.0;
    if (!converged[tl.c]) {
        const CaseDev& cd = cases[tl.c];
        const int w = tl.wave0 + (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        if (w < cd.nwaves) {
            const int y = w / cd.wpr;
            const int x = (w - y * cd.wpr) * 64 + (int)(threadIdx.x & 63);
            if (x < cd.sa.nx && obase[cd.own_off + (int64_t)y * cd.sa.opitch + x] == 0) {
                const T* f = fbase + cd.f_off[parity];
                double d[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) d[i] = (double)pop_at(f, cd.sa, i, x, y);
                const double drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
                const double r = cd.sa.rho0 + drho;
                const double jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
                const double jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
                // Guo velocity of the pre-collision state: rho u = sum e f~ - rho g / 2
                const double ux = jx / r - 0.5 * cd.cp64.gx;
                const double uy = jy / r - 0.5 * cd.cp64.gy;
                double* sn = snap_base + cd.snap_off + (int64_t)y * cd.sa.nx + x;
                const int64_t plane = (int64_t)cd.sa.nx * cd.sa.ny;
                const double px = sn[0], py = sn[plane];
                dd = (ux - px) * (ux - px) + (uy - py) * (uy - py);
                uu = ux * ux + uy * uy;
                sn[0] = ux;
                sn[plane] = uy;
            }
        }
    }
    dd = wave_sum(dd);
    uu = wave_sum(uu);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[wv][0] = dd;
        red[wv][1] = uu;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double v = 0.0;
        for (int k = 0; k < WAVES; ++k) v += red[k][threadIdx.x];
        mon_partial[(size_t)blockIdx.x * 2 + threadIdx.x] = v;
    }
}

// One thread per case: residual from the tile partials (in tile order), force
// totals per solid from the chunk partials (in chunk order); retire the case
// when a previous snapshot exists and r < tol.
struct CaseResult {
    int converged;
    int have_snap;
    int64_t steps;
    double residual;
};

__global__ void k_batch_finalize(const CaseDev* __restrict__ cases, const int* __restrict__ tile_first,
                                 const int* __restrict__ tile_count, const double* __restrict__ mon_partial,
                                 const BatchChunk* __restrict__ chunks,
                                 const double* __restrict__ force_partial, CaseResult* __restrict__ res,
                                 int* __restrict__ converged, double* __restrict__ forces, int max_nsol,
                                 int n_cases, const int64_t* __restrict__ tdev, int parity, int k_steps,
                                 double tol) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cases) return;
    if (converged[c]) return;
    const CaseDev& cd = cases[c];
    double dd = 0.0, uu = 0.0;
    for (int b = tile_first[c]; b < tile_first[c] + tile_count[c]; ++b) {
        dd += mon_partial[2 * (size_t)b];
        uu += mon_partial[2 * (size_t)b + 1];
    }
    // a state that is not finite (a diverged start) reports NaN and never retires
    const double r = !(isfinite(dd) && isfinite(uu))
                         ? __builtin_nan("")
                         : (uu > 0.0 ? sqrt(dd) / ((double)k_steps * sqrt(uu)) : (dd > 0.0 ? 1.0 : 0.0));
    double* fc = forces + (size_t)c * max_nsol * 6;
    for (int q = 0; q < cd.nsol * 6; ++q) fc[q] = 0.0;
    // chunks of a case are listed solid by solid: chunk order is summation order
    for (int cc = cd.chunk_first; cc < cd.chunk_first + cd.chunk_count; ++cc) {
        const int s = chunks[cc].s;
        for (int q = 0; q < 6; ++q) fc[s * 6 + q] += force_partial[(size_t)cc * 6 + q];
    }
    CaseResult rr = res[c];
    rr.residual = rr.have_snap ? r : -1.0;
    rr.steps = tdev[parity];
    if (rr.have_snap && r < tol) {
        rr.converged = 1;
        converged[c] = 1;
    }
    rr.have_snap = 1;
    res[c] = rr;
}

}  // namespace lbm
