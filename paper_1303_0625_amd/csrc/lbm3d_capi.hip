// lbm3d_capi.hip -- host side of the three-dimensional entry points
// (lbm3d_* in include/lbm.h): validation, the geometry and link lists (fixed
// geometry: built once on the host), workspace layout inside the caller's
// device buffer, and the per-step launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "lbm3d_kernels.h"

using namespace lbm3;

namespace {

thread_local char g_err3[512] = "";

void set_err3(char* buf, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
}

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr size_t kStreamBytes3 = 256ull << 20;  // Infinity Cache: stream above it

struct Layout3 {
    size_t f[2], own[2], flags[2], links, seg_off, seg_cnt, chunk_solid, chunk_start, solid_chunk0, sol[2], partial, hist,
        tctr, movers, mass, err, total;
    int pitch;
    int nchunks;
    int64_t nlinks;
    int box;      // scan-box edge of the moving spheres (0: none moves)
    int nmovers;
};

// Scan-box edge of a moving sphere of radius r: the nodes from
// floor(X - r) - 2 on, far enough to hold every fluid node next to it.
int box_edge(double r) { return 2 * (int)std::ceil(r) + 5; }

}  // namespace

struct lbm3d_ctx {
    lbm3d_grid g;
    int ns = 0;
    int64_t hist_cap = 0;
    int64_t t = 0;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    Layout3 L{};
    char err[512] = "";
    std::vector<double> sol;  // host copy of the solid table (initial state)
    int nfree = 0;
    double G[3] = {0.0, 0.0, 0.0};
    int dyn_scheme = LBM_GME;
    int force_avg = 0;
    int pressure = 0;
    int ibb = 0;
    double rho_in = 1.0, rho_out = 1.0;
    bool prof = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    double prof_ms = 0.0;
    int64_t prof_n = 0;
};

namespace {

lbm_status fail3(lbm3d_ctx* c, hipError_t e, const char* what) {
    set_err3(c ? c->err : g_err3, "%s: %s", what, hipGetErrorString(e));
    return LBM_EDEVICE;
}

#define HIPCHK3(ctx, call)                                  \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return fail3(ctx, e_, #call); \
    } while (0)

// Minimum-image difference on a periodic axis (ties go to +n/2).
double mimg(double d, int n) { return d - (double)n * std::floor(d / (double)n + 0.5); }

// Owner of node (x, y, z): the duct, then the spheres; every product and sum
// rounded separately (no contraction), so that a node on a surface is
// classified as a plain IEEE double evaluation does.  overlap: a node claimed
// twice.
#pragma clang fp contract(off)
int owner_of(const lbm3d_grid& g, const lbm3d_sphere* sp, int ns, int x, int y, int z, bool& overlap) {
    int o = 0;
    if (g.duct == LBM3D_TUBE) {
        const double dy = (double)y - 0.5 * (g.ny - 1), dz = (double)z - 0.5 * (g.nz - 1);
        const double r2 = dy * dy + dz * dz;
        if (r2 > g.R * g.R) o = kDuct;
    } else if (g.duct == LBM3D_PLANES) {
        if (z == 0 || z == g.nz - 1) o = kDuct;
    }
    for (int k = 0; k < ns; ++k) {
        const double dx = mimg((double)x - sp[k].X[0], g.nx);
        const double dy = mimg((double)y - sp[k].X[1], g.ny);
        const double dz = mimg((double)z - sp[k].X[2], g.nz);
        double d2 = dx * dx;
        d2 = d2 + dy * dy;
        d2 = d2 + dz * dz;
        if (d2 <= sp[k].r * sp[k].r) {
            if (o != 0) overlap = true;
            o = k + 1;
        }
    }
    return o;
}

const char* validate(const lbm3d_grid* g, const lbm3d_sphere* sp, int ns) {
    if (g && (g->refill < 0 || g->refill > 2)) return "refill must be LBM_REFILL_A1, A2 or A3";
    if (!g) return "grid is NULL";
    if (g->nx < 4 || g->ny < 4 || g->nz < 4) return "nx, ny, nz must be >= 4";
    if ((int64_t)g->nx * g->ny * g->nz >= (1ll << 27)) return "at most 2^27 nodes (link codes)";
    if (g->dtype != LBM_F64 && g->dtype != LBM_F32) return "dtype must be LBM_F64 or LBM_F32";
    if (!(g->tau > 0.5)) return "tau must exceed 1/2";
    if (!(g->rho0 > 0.0)) return "rho0 must be positive";
    if (g->duct != LBM3D_OPEN && g->duct != LBM3D_TUBE && g->duct != LBM3D_PLANES) return "unknown duct";
    if (g->duct == LBM3D_TUBE && !(g->R >= 2.0)) return "tube radius must be >= 2";
    if (ns < 0 || ns > 200) return "0..200 spheres";
    if (ns > 0 && !sp) return "spheres is NULL";
    for (int k = 0; k < ns; ++k) {
        if (!(sp[k].r >= 1.0)) return "sphere radius must be >= 1";
        double s = 0.0;
        for (int d = 0; d < 3; ++d) s += sp[k].V[d] * sp[k].V[d];
        if (!(std::sqrt(s) < 0.3)) return "sphere surface speed must be below 0.3";
        if (sp[k].moves) {
            const int b = box_edge(sp[k].r);
            if (b > g->nx || b > g->ny || b > g->nz) return "a moving sphere's box (2 ceil(r) + 5) exceeds the lattice";
        }
    }
    return nullptr;
}

// Geometry and link lists on the host; returns an error message or nullptr.
const char* build_geometry(const lbm3d_grid& g, const lbm3d_sphere* sp, int ns, int pitch,
                           std::vector<uint8_t>& own, std::vector<uint8_t>& flags,
                           std::vector<std::vector<uint32_t>>& seg) {
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    own.assign((size_t)ny * nz * pitch, 0);
    bool overlap = false;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                own[((size_t)z * ny + y) * pitch + x] = (uint8_t)owner_of(g, sp, ns, x, y, z, overlap);
    if (overlap) return "a sphere overlaps the duct or another sphere";
    static const int E[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                                 {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                 {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                 {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    seg.assign(ns + 1, {});
    flags.assign(own.size(), 0);
    size_t nfluid = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (own[((size_t)z * ny + y) * pitch + x] != 0) {
                    flags[((size_t)z * ny + y) * pitch + x] = kSolidNode;
                    continue;
                }
                ++nfluid;
                const uint32_t node = (uint32_t)(((int64_t)z * ny + y) * nx + x);
                for (int i = 1; i < 19; ++i) {
                    const int xb = (x + E[i][0] + nx) % nx, yb = (y + E[i][1] + ny) % ny,
                              zb = (z + E[i][2] + nz) % nz;
                    const uint8_t o = own[((size_t)zb * ny + yb) * pitch + xb];
                    if (o == 0) continue;
                    flags[((size_t)z * ny + y) * pitch + x] = kNearSolid;
                    if (o != kDuct && sp[o - 1].moves) continue;  // found by the box scan each step
                    seg[o == kDuct ? 0 : o].push_back(node << 5 | (uint32_t)i);
                }
            }
    if (nfluid == 0) return "no fluid node";
    return nullptr;
}

Layout3 make_layout(const lbm3d_grid& g, const lbm3d_sphere* sp, int ns, int pitch,
                    const std::vector<std::vector<uint32_t>>& seg, int64_t hist_cap) {
    Layout3 L{};
    L.pitch = pitch;
    for (int k = 0; k < ns; ++k)
        if (sp[k].moves) {
            L.box = std::max(L.box, box_edge(sp[k].r));
            ++L.nmovers;
        }
    const size_t es = g.dtype == LBM_F64 ? 8 : 4;
    const size_t fbytes = (size_t)19 * g.ny * g.nz * pitch * es;
    size_t off = 0;
    L.f[0] = off;
    off = al256(off + fbytes);
    // second buffer skewed by 1 MiB off a power-of-two distance
    off = al256(off + (1u << 20));
    L.f[1] = off;
    off = al256(off + fbytes);
    for (int k = 0; k < 2; ++k) {
        L.own[k] = off;
        off = al256(off + (size_t)g.ny * g.nz * pitch);
        L.flags[k] = off;
        off = al256(off + (size_t)g.ny * g.nz * pitch);
    }
    int64_t nl = 0;
    int nch = 0;
    const int64_t box3 = (int64_t)L.box * L.box * L.box;
    for (size_t s = 0; s < seg.size(); ++s) {
        nl += (int64_t)seg[s].size();
        const bool mv = s > 0 && sp[s - 1].moves;
        nch += mv ? (int)((box3 + kChunk - 1) / kChunk) : std::max<int>(1, (int)((seg[s].size() + kChunk - 1) / kChunk));
    }
    L.nlinks = nl;
    L.nchunks = nch;
    L.links = off;
    off = al256(off + 4 * (size_t)std::max<int64_t>(nl, 1));
    L.seg_off = off;
    off = al256(off + 4 * (size_t)(ns + 1));
    L.seg_cnt = off;
    off = al256(off + 4 * (size_t)(ns + 1));
    L.chunk_solid = off;
    off = al256(off + 4 * (size_t)nch);
    L.chunk_start = off;
    off = al256(off + 4 * (size_t)nch);
    L.solid_chunk0 = off;
    off = al256(off + 4 * (size_t)(ns + 2));
    for (int k = 0; k < 2; ++k) {
        L.sol[k] = off;
        off = al256(off + 8 * (size_t)kSolidRow * (ns + 1));
    }
    L.mass = off;
    off = al256(off + 8 * (size_t)4 * (ns + 1));
    L.err = off;
    off = al256(off + 16);
    L.partial = off;
    off = al256(off + 8 * (size_t)2 * nch * 12);
    L.hist = off;
    off = al256(off + 8 * (size_t)hist_cap * (ns + 1) * 12);
    L.tctr = off;
    off = al256(off + 16);
    L.movers = off;
    off = al256(off + 4 * (size_t)std::max(L.nmovers, 1));
    L.total = off;
    return L;
}

template <typename P>
P* at(lbm3d_ctx* c, size_t off) {
    return reinterpret_cast<P*>(c->ws + off);
}

// Round-up multiplier m and shift l = ceil(log2 d) with n / d ==
// (mulhi(n, m) + n) >> l for 0 <= n < 2^31, d >= 1 (Granlund and
// Montgomery, PLDI 1994).
void magic32(uint32_t d, uint32_t& m, uint32_t& l) {
    l = 0;
    while ((1ull << l) < d) ++l;
    m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
}

Args args3(const lbm3d_ctx* c) {
    Args a{};
    a.nx = c->g.nx;
    a.ny = c->g.ny;
    a.nz = c->g.nz;
    a.pitch = c->L.pitch;
    a.ns = c->ns;
    a.rho0 = c->g.rho0;
    a.tau = c->g.tau;
    a.omega = 1.0 / c->g.tau;
    a.cs = 1.0 - 0.5 / c->g.tau;
    for (int d = 0; d < 3; ++d) a.g[d] = c->g.g[d];
    a.nchunks = c->L.nchunks;
    a.hist_cap = c->hist_cap;
    a.duct = c->g.duct;
    a.R = c->g.R;
    a.box = c->L.box;
    a.refill = c->g.refill;
    a.ibb = c->ibb;
    a.rho_in = c->rho_in;
    a.rho_out = c->rho_out;
    // update workgroups per plane and waves per line, with their division
    // multipliers
    a.W = (uint32_t)(c->L.pitch / 64);
    a.K = (uint32_t)((c->g.ny * a.W + kBlock / 64 - 1) / (kBlock / 64));
    magic32(a.K, a.magK, a.shK);
    magic32(a.W, a.magW, a.shW);
    magic32((uint32_t)c->g.ny, a.magNy, a.shNy);
    return a;
}

int pitch_for(int nx) { return (nx + 63) / 64 * 64; }

using StepKernel = void (*)(Ptrs, int, int, Args);

template <typename T, bool NT>
StepKernel step_kernel(bool ibb, bool pressure) {
    if (ibb) return pressure ? k3_step<T, NT, true, true> : k3_step<T, NT, true, false>;
    return pressure ? k3_step<T, NT, false, true> : k3_step<T, NT, false, false>;
}

}  // namespace

extern "C" {

lbm_status lbm3d_workspace_bytes(const lbm3d_grid* g, const lbm3d_sphere* spheres, int32_t n_spheres,
                                 int64_t history_steps, size_t* bytes) {
    if (!bytes) {
        set_err3(g_err3, "bytes is NULL");
        return LBM_EINVAL;
    }
    if (const char* why = validate(g, spheres, n_spheres)) {
        set_err3(g_err3, "%s", why);
        return LBM_EINVAL;
    }
    if (history_steps < 1) {
        set_err3(g_err3, "history_steps must be >= 1");
        return LBM_EINVAL;
    }
    std::vector<uint8_t> own, flags;
    std::vector<std::vector<uint32_t>> seg;
    const int pitch = pitch_for(g->nx);
    if (const char* why = build_geometry(*g, spheres, n_spheres, pitch, own, flags, seg)) {
        set_err3(g_err3, "%s", why);
        return LBM_EGEOM;
    }
    *bytes = make_layout(*g, spheres, n_spheres, pitch, seg, history_steps).total;
    return LBM_OK;
}

lbm_status lbm3d_create(const lbm3d_grid* g, const lbm3d_sphere* spheres, int32_t n_spheres,
                        int64_t history_steps, void* d_workspace, size_t bytes, void* hip_stream,
                        lbm3d_ctx** out) {
    if (!out) {
        set_err3(g_err3, "out is NULL");
        return LBM_EINVAL;
    }
    *out = nullptr;
    if (const char* why = validate(g, spheres, n_spheres)) {
        set_err3(g_err3, "%s", why);
        return LBM_EINVAL;
    }
    if (history_steps < 1) {
        set_err3(g_err3, "history_steps must be >= 1");
        return LBM_EINVAL;
    }
    if (!d_workspace || ((uintptr_t)d_workspace & 255u) != 0) {
        set_err3(g_err3, "workspace must be a non-NULL 256-byte aligned device pointer");
        return LBM_EINVAL;
    }
    const int pitch = pitch_for(g->nx);
    std::vector<uint8_t> own, flags;
    std::vector<std::vector<uint32_t>> seg;
    if (const char* why = build_geometry(*g, spheres, n_spheres, pitch, own, flags, seg)) {
        set_err3(g_err3, "%s", why);
        return LBM_EGEOM;
    }
    Layout3 L = make_layout(*g, spheres, n_spheres, pitch, seg, history_steps);
    if (bytes < L.total) {
        set_err3(g_err3, "workspace holds %zu bytes, %zu needed", bytes, L.total);
        return LBM_ESIZE;
    }
    lbm3d_ctx* c = new (std::nothrow) lbm3d_ctx;
    if (!c) return LBM_EINVAL;
    c->g = *g;
    c->ns = n_spheres;
    c->hist_cap = history_steps;
    c->ws = (char*)d_workspace;
    c->stream = (hipStream_t)hip_stream;
    c->L = L;
    // tables
    std::vector<uint32_t> links;
    std::vector<int> seg_off(n_spheres + 1), seg_cnt(n_spheres + 1), chunk_solid, chunk_start,
        solid_chunk0(n_spheres + 2), movers;
    const int64_t box3 = (int64_t)L.box * L.box * L.box;
    for (int s = 0; s <= n_spheres; ++s) {
        seg_off[s] = (int)links.size();
        seg_cnt[s] = (int)seg[s].size();
        links.insert(links.end(), seg[s].begin(), seg[s].end());
        solid_chunk0[s] = (int)chunk_solid.size();
        const bool mv = s > 0 && spheres[s - 1].moves;
        if (mv) movers.push_back(s);
        const int nchk = mv ? (int)((box3 + kChunk - 1) / kChunk)
                            : std::max<int>(1, (int)((seg[s].size() + kChunk - 1) / kChunk));
        for (int k = 0; k < nchk; ++k) {
            chunk_solid.push_back(s);
            chunk_start.push_back(k * kChunk);
        }
    }
    solid_chunk0[n_spheres + 1] = (int)chunk_solid.size();
    c->sol.assign((size_t)kSolidRow * (n_spheres + 1), 0.0);
    for (int k = 0; k < n_spheres; ++k) {
        double* r = c->sol.data() + kSolidRow * (k + 1);
        for (int d = 0; d < 3; ++d) {
            r[d] = spheres[k].X[d];
            r[4 + d] = spheres[k].V[d];
            r[7 + d] = spheres[k].omega[d];
        }
        r[3] = spheres[k].r;
        r[10] = spheres[k].moves ? 1.0 : 0.0;
    }
    hipError_t e = hipMemsetAsync(c->ws, 0, L.total, c->stream);
    auto up = [&](size_t off, const void* src, size_t n) {
        if (e == hipSuccess && n > 0) e = hipMemcpyAsync(c->ws + off, src, n, hipMemcpyHostToDevice, c->stream);
    };
    up(L.own[0], own.data(), own.size());
    up(L.own[1], own.data(), own.size());
    up(L.flags[0], flags.data(), flags.size());
    up(L.flags[1], flags.data(), flags.size());
    up(L.movers, movers.data(), 4 * movers.size());
    up(L.links, links.data(), 4 * links.size());
    up(L.seg_off, seg_off.data(), 4 * seg_off.size());
    up(L.seg_cnt, seg_cnt.data(), 4 * seg_cnt.size());
    up(L.chunk_solid, chunk_solid.data(), 4 * chunk_solid.size());
    up(L.chunk_start, chunk_start.data(), 4 * chunk_start.size());
    up(L.solid_chunk0, solid_chunk0.data(), 4 * solid_chunk0.size());
    up(L.sol[0], c->sol.data(), 8 * c->sol.size());
    up(L.sol[1], c->sol.data(), 8 * c->sol.size());
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        set_err3(g_err3, "hipMemcpyAsync: %s", hipGetErrorString(e));
        delete c;
        return LBM_EDEVICE;
    }
    const Args a = args3(c);
    const int64_t N = (int64_t)g->ny * g->nz * pitch;
    const unsigned nb = (unsigned)((N + kBlock - 1) / kBlock);
    if (g->dtype == LBM_F64)
        k3_init<double><<<nb, kBlock, 0, c->stream>>>(at<double>(c, L.f[0]), at<uint8_t>(c, L.own[0]), a,
                                                      g->u0[0], g->u0[1], g->u0[2]);
    else
        k3_init<float><<<nb, kBlock, 0, c->stream>>>(at<float>(c, L.f[0]), at<uint8_t>(c, L.own[0]), a, g->u0[0],
                                                     g->u0[1], g->u0[2]);
    k3_set_counters<<<1, 1, 0, c->stream>>>(at<int64_t>(c, L.tctr), 0);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        set_err3(g_err3, "init: %s", hipGetErrorString(e));
        delete c;
        return LBM_EDEVICE;
    }
    *out = c;
    return LBM_OK;
}

// Moving spheres over steps [t0, t1]: each keeps 2 nodes from the duct and
// from every other sphere (so the other solids' link lists stay valid).
static const char* check_paths3(const lbm3d_ctx* c, int64_t t0, int64_t t1) {
    const int ns = c->ns;
    auto centre_at = [&](int k, int64_t t, double X[3]) {
        const double* S = c->sol.data() + kSolidRow * (k + 1);
        for (int d = 0; d < 3; ++d) X[d] = S[10] != 0.0 ? S[d] + (double)t * S[4 + d] : S[d];
    };
    for (int k = 0; k < ns; ++k) {
        const double* S = c->sol.data() + kSolidRow * (k + 1);
        if (S[10] == 0.0 || S[11] != 0.0) continue;  // fixed, or free (checked on the device)
        const double r = S[3];
        for (int64_t t = t0; t <= t1; ++t) {
            double X[3];
            centre_at(k, t, X);
            if (c->g.duct == LBM3D_TUBE) {
                const double dy = X[1] - 0.5 * (c->g.ny - 1), dz = X[2] - 0.5 * (c->g.nz - 1);
                if (std::sqrt(dy * dy + dz * dz) + r > c->g.R - 2.0) return "a moving sphere comes within 2 nodes of the tube";
            } else if (c->g.duct == LBM3D_PLANES) {
                if (X[2] - r < 2.0 || X[2] + r > c->g.nz - 3.0) return "a moving sphere comes within 2 nodes of a plane";
            }
            for (int j = 0; j < ns; ++j) {
                if (j == k || c->sol[kSolidRow * (j + 1) + 11] != 0.0) continue;
                double Y[3];
                centre_at(j, t, Y);
                double d2 = 0.0;
                const int n3[3] = {c->g.nx, c->g.ny, c->g.nz};
                for (int d = 0; d < 3; ++d) {
                    const double dd = mimg(X[d] - Y[d], n3[d]);
                    d2 += dd * dd;
                }
                const double rj = c->sol[kSolidRow * (j + 1) + 3];
                if (std::sqrt(d2) < r + rj + 2.0) return "a moving sphere comes within 2 nodes of another sphere";
            }
        }
    }
    return nullptr;
}

lbm_status lbm3d_step(lbm3d_ctx* c, int64_t n) {
    if (!c || n < 0) return LBM_EINVAL;
    if (n == 0) return LBM_OK;
    if (c->L.nmovers > 0)
        if (const char* why = check_paths3(c, c->t, c->t + n + 1)) {
            set_err3(c->err, "%s", why);
            return LBM_EGEOM;
        }
    const Args a = args3(c);
    const int n_fin = (c->ns + 1) * 12;  // one finalizer workgroup per (solid, component)
    const int n_lead = (c->L.nchunks + n_fin + 7) / 8 * 8;
    const int64_t lines = (int64_t)c->g.ny * c->g.nz;
    // the update workgroups: one wave per 64 nodes of a line, the grid
    // padded to a multiple of 8 K
    const int64_t waves = lines * (c->L.pitch / 64), K8 = 8 * (int64_t)a.K;
    const int64_t n_upd = ((waves + kBlock / 64 - 1) / (kBlock / 64) + K8 - 1) / K8 * K8;
    const unsigned grid = (unsigned)(n_lead + n_upd);
    const size_t es = c->g.dtype == LBM_F64 ? 8 : 4;
    const bool nt = 2 * (size_t)19 * lines * c->L.pitch * es > kStreamBytes3;
    Ptrs p{};
    p.links = at<uint32_t>(c, c->L.links);
    p.seg_off = at<int>(c, c->L.seg_off);
    p.seg_cnt = at<int>(c, c->L.seg_cnt);
    p.chunk_solid = at<int>(c, c->L.chunk_solid);
    p.chunk_start = at<int>(c, c->L.chunk_start);
    p.solid_chunk0 = at<int>(c, c->L.solid_chunk0);

    p.partial = at<double>(c, c->L.partial);
    p.hist = at<double>(c, c->L.hist);
    p.tctr = at<int64_t>(c, c->L.tctr);
    for (int64_t k = 0; k < n; ++k) {
        const int par = (int)(c->t & 1);
        p.fin = c->ws + c->L.f[par];
        p.fout = c->ws + c->L.f[par ^ 1];
        p.own = at<uint8_t>(c, c->L.own[par]);
        p.flags = at<uint8_t>(c, c->L.flags[par]);
        p.sol = at<double>(c, c->L.sol[par]);
        const bool timed = c->prof && c->ev_used + 2 <= c->ev.size();
        if (timed) HIPCHK3(c, hipEventRecord(c->ev[c->ev_used], c->stream));
        {
            // the pressure planes, when set, are part of the step launch
            const bool ibb = c->ibb != 0, pr = c->pressure != 0;
            const StepKernel kern = c->g.dtype == LBM_F64
                                        ? (nt ? step_kernel<double, true>(ibb, pr) : step_kernel<double, false>(ibb, pr))
                                        : (nt ? step_kernel<float, true>(ibb, pr) : step_kernel<float, false>(ibb, pr));
            kern<<<grid, kBlock, 0, c->stream>>>(p, par, n_lead, a);
        }
        double* sol_n = at<double>(c, c->L.sol[par ^ 1]);
        if (c->nfree > 0) {
            // free spheres: Newton-Euler step from this step's forces
            FreeArgs3 fa{};
            fa.sol_t = p.sol;
            fa.sol_n = sol_n;
            fa.mass = at<double>(c, c->L.mass);
            fa.partial = p.partial + (size_t)(c->t & 1) * c->L.nchunks * 12;
            // step t - 1's partials are intact until step t + 1 writes them
            fa.partial_prev = (c->force_avg && c->t >= 1) ? p.partial + (size_t)((c->t - 1) & 1) * c->L.nchunks * 12
                                                           : nullptr;
            fa.solid_chunk0 = p.solid_chunk0;
            fa.err = at<int>(c, c->L.err);
            for (int d = 0; d < 3; ++d) fa.G[d] = c->G[d];
            fa.scheme = c->dyn_scheme == LBM_CME ? 0 : 1;
            k3_free<<<1, kBlock, 0, c->stream>>>(fa, c->t, a);
        }
        if (c->L.nmovers > 0) {
            // geometry of step t + 1, then the newborn refill into the step's output
            uint8_t* own_n = at<uint8_t>(c, c->L.own[par ^ 1]);
            const int64_t N = (int64_t)c->g.nx * c->g.ny * c->g.nz;
            k3_raster<<<(unsigned)((N + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(sol_n, own_n, c->t + 1, a);
            k3_flags<<<(unsigned)((N + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(
                own_n, at<uint8_t>(c, c->L.flags[par ^ 1]), a);
            const int cpm = (int)(((int64_t)c->L.box * c->L.box * c->L.box + kBlock - 1) / kBlock);
            const unsigned nrb = (unsigned)(cpm * c->L.nmovers);
            const int* mv = at<int>(c, c->L.movers);
            if (c->g.dtype == LBM_F64)
                k3_refill<double><<<nrb, kBlock, 0, c->stream>>>(p, sol_n, own_n, mv, cpm, c->t, a);
            else
                k3_refill<float><<<nrb, kBlock, 0, c->stream>>>(p, sol_n, own_n, mv, cpm, c->t, a);
        }
        if (timed) {
            HIPCHK3(c, hipEventRecord(c->ev[c->ev_used + 1], c->stream));
            c->ev_used += 2;
        }
        c->t += 1;
    }
    k3_finalize<<<(unsigned)n_fin, kBlock, 0, c->stream>>>(p.partial, p.solid_chunk0, p.hist, p.tctr,
                                                           (int)(c->t & 1), a);
    HIPCHK3(c, hipGetLastError());
    return LBM_OK;
}

int64_t lbm3d_time(const lbm3d_ctx* c) { return c ? c->t : -1; }

lbm_status lbm3d_force(lbm3d_ctx* c, int32_t solid, int32_t scheme, int64_t step, double out[6]) {
    if (!c || !out || solid < 0 || solid > c->ns || (scheme != LBM_CME && scheme != LBM_GME)) return LBM_EINVAL;
    if (step < 0) step = c->t - 1;
    if (step < 0 || step >= c->t || step < c->t - c->hist_cap) {
        set_err3(c->err, "no force record for step %lld", (long long)step);
        return LBM_ESTATE;
    }
    const size_t off =
        c->L.hist + 8 * (((size_t)(step % c->hist_cap) * (c->ns + 1) + solid) * 12 + 6 * (size_t)scheme);
    HIPCHK3(c, hipMemcpyAsync(out, c->ws + off, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm3d_force_history(lbm3d_ctx* c, int64_t first, int64_t count, double* d_out) {
    if (!c || !d_out || first < 0 || count < 0) return LBM_EINVAL;
    if (first + count > c->t || first < c->t - c->hist_cap) {
        set_err3(c->err, "steps [%lld, %lld) are not in the history", (long long)first, (long long)(first + count));
        return LBM_ESTATE;
    }
    const size_t row = 8 * (size_t)(c->ns + 1) * 12;
    for (int64_t k = 0; k < count; ++k) {
        const size_t src = c->L.hist + row * (size_t)((first + k) % c->hist_cap);
        HIPCHK3(c, hipMemcpyAsync((char*)d_out + row * (size_t)k, c->ws + src, row, hipMemcpyDeviceToDevice,
                                  c->stream));
    }
    return LBM_OK;
}

lbm_status lbm3d_fields(lbm3d_ctx* c, double* d_rho, double* d_u, int32_t* d_owner) {
    if (!c) return LBM_EINVAL;
    const Args a = args3(c);
    const int64_t N = (int64_t)c->g.nx * c->g.ny * c->g.nz;
    const unsigned nb = (unsigned)((N + kBlock - 1) / kBlock);
    const int par = (int)(c->t & 1);
    const uint8_t* own = at<uint8_t>(c, c->L.own[par]);
    if (c->g.dtype == LBM_F64)
        k3_fields<double><<<nb, kBlock, 0, c->stream>>>(at<double>(c, c->L.f[par]), own, a, d_rho, d_u, d_owner);
    else
        k3_fields<float><<<nb, kBlock, 0, c->stream>>>(at<float>(c, c->L.f[par]), own, a, d_rho, d_u, d_owner);
    HIPCHK3(c, hipGetLastError());
    return LBM_OK;
}

int64_t lbm3d_link_count(const lbm3d_ctx* c) { return c ? c->L.nlinks : -1; }

lbm_status lbm3d_set_free(lbm3d_ctx* c, int32_t sphere, double rho_s, const double omega0[3]) {
    if (!c || !omega0) return LBM_EINVAL;
    if (sphere < 1 || sphere > c->ns || !(rho_s > 0.0)) {
        set_err3(c->err, "sphere must be 1..n_spheres and rho_s positive");
        return LBM_EINVAL;
    }
    double* S = c->sol.data() + kSolidRow * sphere;
    if (S[10] == 0.0) {
        set_err3(c->err, "a free sphere must be created with moves = 1");
        return LBM_EINVAL;
    }
    if (c->t != 0) {
        set_err3(c->err, "free spheres are set before the first step");
        return LBM_ESTATE;
    }
    const double r = S[3];
    const double vol = 4.0 / 3.0 * M_PI * r * r * r;
    const double mass[4] = {rho_s * vol, 0.4 * rho_s * vol * r * r, vol, 0.0};
    if (S[11] == 0.0) c->nfree += 1;
    S[11] = 1.0;
    for (int d = 0; d < 3; ++d) S[7 + d] = omega0[d];
    for (int k = 0; k < 2; ++k)
        HIPCHK3(c, hipMemcpyAsync(c->ws + c->L.sol[k] + 8 * (size_t)kSolidRow * sphere, S, 8 * kSolidRow,
                                  hipMemcpyHostToDevice, c->stream));
    HIPCHK3(c, hipMemcpyAsync(c->ws + c->L.mass + 8 * (size_t)4 * sphere, mass, sizeof(mass), hipMemcpyHostToDevice,
                              c->stream));
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm3d_set_gravity(lbm3d_ctx* c, const double G[3], int32_t scheme) {
    if (!c || !G || (scheme != LBM_CME && scheme != LBM_GME)) return LBM_EINVAL;
    for (int d = 0; d < 3; ++d) c->G[d] = G[d];
    c->dyn_scheme = scheme;
    return LBM_OK;
}

lbm_status lbm3d_set_boundary(lbm3d_ctx* c, int32_t rule) {
    if (!c) return LBM_EINVAL;
    if (rule != LBM_HALFWAY && rule != LBM_INTERPOLATED) {
        set_err3(c->err, "rule must be LBM_HALFWAY or LBM_INTERPOLATED");
        return LBM_EINVAL;
    }
    c->ibb = rule == LBM_INTERPOLATED ? 1 : 0;
    return LBM_OK;
}

lbm_status lbm3d_set_pressure(lbm3d_ctx* c, double rho_in, double rho_out) {
    if (!c || !(rho_in > 0.0) || !(rho_out > 0.0)) return LBM_EINVAL;
    if (c->L.nmovers > 0) {
        set_err3(c->err, "pressure boundaries are for fixed spheres only");
        return LBM_EINVAL;
    }
    if (c->t != 0) {
        set_err3(c->err, "pressure boundaries are set before the first step");
        return LBM_ESTATE;
    }
    c->pressure = 1;
    c->rho_in = rho_in;
    c->rho_out = rho_out;
    // the initial post-collision state takes the boundary values too
    const Args a = args3(c);
    const unsigned npb = (unsigned)((2 * (int64_t)c->g.ny * c->g.nz + kBlock - 1) / kBlock);
    if (c->g.dtype == LBM_F64)
        k3_pressure<double><<<npb, kBlock, 0, c->stream>>>(at<double>(c, c->L.f[0]), at<uint8_t>(c, c->L.own[0]), a,
                                                           rho_in, rho_out);
    else
        k3_pressure<float><<<npb, kBlock, 0, c->stream>>>(at<float>(c, c->L.f[0]), at<uint8_t>(c, c->L.own[0]), a,
                                                          rho_in, rho_out);
    HIPCHK3(c, hipGetLastError());
    return LBM_OK;
}

lbm_status lbm3d_set_force_average(lbm3d_ctx* c, int32_t enable) {
    if (!c) return LBM_EINVAL;
    c->force_avg = enable != 0;
    return LBM_OK;
}

lbm_status lbm3d_body_state(lbm3d_ctx* c, int32_t sphere, double out[9]) {
    if (!c || !out || sphere < 1 || sphere > c->ns) return LBM_EINVAL;
    double row[kSolidRow];
    HIPCHK3(c, hipMemcpyAsync(row, c->ws + c->L.sol[c->t & 1] + 8 * (size_t)kSolidRow * sphere, sizeof(row),
                              hipMemcpyDeviceToHost, c->stream));
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    const bool translating = row[10] != 0.0 && row[11] == 0.0;
    for (int d = 0; d < 3; ++d) {
        out[d] = translating ? row[d] + (double)c->t * row[4 + d] : row[d];
        out[3 + d] = row[4 + d];
        out[6 + d] = row[7 + d];
    }
    return LBM_OK;
}

lbm_status lbm3d_status_check(lbm3d_ctx* c) {
    if (!c) return LBM_EINVAL;
    int e = 0;
    HIPCHK3(c, hipMemcpyAsync(&e, c->ws + c->L.err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    if (e != 0) {
        set_err3(c->err, "a free sphere came within 2 nodes of the duct or another sphere, or moved more than half a "
                         "node in a step");
        return LBM_EGEOM;
    }
    return LBM_OK;
}

lbm_status lbm3d_profile(lbm3d_ctx* c, int32_t enable) {
    if (!c) return LBM_EINVAL;
    c->prof = enable != 0;
    c->ev_used = 0;
    c->prof_ms = 0.0;
    c->prof_n = 0;
    if (c->prof && c->ev.empty()) {
        c->ev.resize(2 * 16384);
        for (auto& ev : c->ev) HIPCHK3(c, hipEventCreate(&ev));
    }
    return LBM_OK;
}

lbm_status lbm3d_profile_read(lbm3d_ctx* c, double* step_ms, int64_t* launches) {
    if (!c || !step_ms || !launches) return LBM_EINVAL;
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float ms = 0.f;
        HIPCHK3(c, hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]));
        c->prof_ms += ms;
        c->prof_n += 1;
    }
    c->ev_used = 0;
    *step_ms = c->prof_ms;
    *launches = c->prof_n;
    return LBM_OK;
}

void lbm3d_destroy(lbm3d_ctx* c) {
    if (!c) return;
    for (auto& ev : c->ev) (void)hipEventDestroy(ev);
    delete c;
}

const char* lbm3d_last_error(const lbm3d_ctx* c) { return c ? c->err : g_err3; }

}  // extern "C"
