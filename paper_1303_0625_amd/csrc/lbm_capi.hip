// lbm_capi.hip -- host side of the C ABI declared in include/lbm.h: argument
// validation, workspace layout inside the caller's device buffer, and the
// per-step launch sequence on the caller's stream.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_kernels.h"

using namespace lbm;

// Workspace of contexts created by lbm_create_static, for callers that cannot
// allocate device memory: one array per device, held until the process ends.
// Host code reaches a device's copy only through its address from
// hipGetSymbolAddress (scratch_on), never through the name.
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

thread_local char g_err[512] = "";

void set_err(char* buf, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Working sets above this use nontemporal loads/stores in the update kernel
// (MI355X has a 256 MB Infinity Cache).
constexpr size_t kStreamBytes = 256ull << 20;
// Steps per captured graph of lbm_step (even: a block keeps its parity).
constexpr int kGraphSteps = 32;

size_t dtype_size(int dt) {
    switch (dt) {
        case LBM_F64: return 8;
        case LBM_F32: return 4;
        case LBM_F16: return 2;
        case LBM_BF16: return 2;
        default: return 0;
    }
}

// Workspace layout (byte offsets inside the caller's buffer).
struct Layout {
    int pitch, opitch;
    int64_t plane;
    size_t f[2], own[2], links[2], seg_off, seg_cap, seg_cnt[2], rec_off, sol, vtab, rtab, movers, frees, fdyn,
        all, chunk_solid, chunk_start, solid_chunk0, partial, hist, tctr, err, total;
    int64_t link_total;
    int n_movers;  // bodies whose geometry moves (prescribed or free)
    int nchunks;
    int box_bytes;  // LDS byte map per translating body (mover role)
    size_t fbytes;  // bytes of one population buffer
    size_t pbytes;  // bytes of its populations proper
    // 16-bit storage: bytes from a buffer to its FP32 side array and to its
    // reference table, their sizes, and reference segments per row
    int64_t side_off, ref_off;
    size_t sbytes, rbytes;
    int nseg;
};

// Conservative link capacity of one body: every fluid node adjacent to a
// compact body lies in the ring of its bounding range, each with at most 8
// links.
int body_link_cap(const lbm_solid& s, int nx, int ny) {
    double hx = s.a, hy = s.shape == LBM_DISC ? s.a : s.b;
    long w = std::min<long>(2 * (long)std::ceil(hx) + 5, nx);
    long h = std::min<long>(2 * (long)std::ceil(hy) + 5, ny);
    long ring = 2 * (w + h) + 8;
    return (int)std::min<long>(8 * ring, 8L * w * h);
}

bool make_layout(const lbm_grid& g, const lbm_solid* solids, int n, int64_t hist_steps, Layout& L) {
    const size_t es = dtype_size(g.dtype);
    L.pitch = (g.nx + 63) / 64 * 64;  // padded row length (elements)
    L.opitch = (g.nx + 63) / 64 * 64;
    L.plane = (int64_t)g.ny * L.pitch;  // elements per population (all rows)
    size_t off = 0;
    const size_t fbytes = 9 * (size_t)L.plane * es;
    L.pbytes = fbytes;
    L.fbytes = fbytes;
    L.side_off = 0;
    // The second buffer starts off a large power-of-two distance from the
    // first: reads of row y and writes of row y then fall on different HBM
    // channels (measured on 4096 x 4096: 231.6 us with no offset, 208.4 us
    // with 3 MiB or more).
    const size_t skew = std::min<size_t>(4u << 20, align256(fbytes / 8));
    L.ref_off = 0;
    L.sbytes = L.rbytes = 0;
    L.nseg = L.pitch >> kRefShift;
    if (es == 2) {
        // 16-bit storage: each buffer has its reference table right after it
        // and a float array (nodes next to a solid) at the same distance
        // side_off; the buffers sit one float array apart so that the two
        // float arrays do not overlap
        L.sbytes = 9 * (size_t)L.plane * 4;
        L.rbytes = (size_t)g.ny * L.nseg * kSeg * 4;
        L.ref_off = (int64_t)align256(fbytes);
        L.f[0] = 0;
        L.f[1] = align256(std::max(L.sbytes, (size_t)L.ref_off + L.rbytes)) + skew;
        L.side_off = (int64_t)align256(L.f[1] + (size_t)L.ref_off + L.rbytes);
        off = align256(L.f[1] + (size_t)L.side_off + L.sbytes);
    } else {
        for (int k = 0; k < 2; ++k) {
            L.f[k] = off;
            off = align256(off + fbytes) + (k == 0 ? skew : 0);
        }
    }
    L.n_movers = 0;
    for (int k = 0; k < n; ++k) L.n_movers += solids[k].moves ? 1 : 0;
    for (int k = 0; k < 2; ++k) {
        L.own[k] = off;
        off = align256(off + (size_t)g.ny * L.opitch);
    }
    int64_t tot = g.walls_y ? 6LL * g.nx : 0;
    int nch = std::max<int64_t>(1, (tot + kForceChunk - 1) / kForceChunk);
    L.box_bytes = 16;
    for (int k = 0; k < n; ++k) {
        int cap = body_link_cap(solids[k], g.nx, g.ny);
        tot += cap;
        nch += std::max(1, (cap + kForceChunk - 1) / kForceChunk);
        if (solids[k].moves) {
            double hx = solids[k].a, hy = solids[k].shape == LBM_DISC ? solids[k].a : solids[k].b;
            int w = (int)std::ceil(2 * hx + 0.6) + 2 * kBoxMargin + 4;
            int h = (int)std::ceil(2 * hy + 0.6) + 2 * kBoxMargin + 4;
            L.box_bytes = std::max(L.box_bytes, (w * h + 15) / 16 * 16);
        }
    }
    L.link_total = tot;
    L.nchunks = nch;
    for (int k = 0; k < 2; ++k) {
        L.links[k] = off;
        off = align256(off + 4 * (size_t)std::max<int64_t>(tot, 1));
    }
    const size_t ns = (size_t)n + 1;
    L.seg_off = off; off = align256(off + 4 * ns);
    L.seg_cap = off; off = align256(off + 4 * ns);
    for (int k = 0; k < 2; ++k) {
        L.seg_cnt[k] = off;
        off = align256(off + 4 * ns);
    }
    L.chunk_solid = off; off = align256(off + 4 * (size_t)nch);
    L.chunk_start = off; off = align256(off + 4 * (size_t)nch);
    L.solid_chunk0 = off; off = align256(off + 4 * (ns + 1));
    L.partial = off; off = align256(off + 2 * 48 * (size_t)nch);
    L.rec_off = off; off = align256(off + 4 * ns);
    L.sol = off; off = align256(off + sizeof(SolidDev) * ns);
    // per-solid velocity {vx, vy} and rotation {Omega, X, Y, free} tables, one per step parity
    L.vtab = off; off = align256(off + 2 * 16 * ns);
    L.rtab = off; off = align256(off + 2 * 8 * kRot * ns);
    L.movers = off; off = align256(off + 4 * (size_t)std::max(L.n_movers, 1));
    L.frees = off; off = align256(off + 4 * (size_t)std::max(L.n_movers, 1));
    L.fdyn = off; off = align256(off + sizeof(FreeDyn) * (size_t)std::max(L.n_movers, 1));
    L.all = off; off = align256(off + 4 * ns);
    L.hist = off; off = align256(off + 48 * ns * (size_t)hist_steps);
    L.tctr = off; off = align256(off + 16);
    L.err = off; off = align256(off + 4);
    L.total = off;
    return true;
}

// Distance between the surfaces of two bodies, with bounding boxes for any box
// shape (conservative) and the minimum image on periodic axes.
double body_gap(const lbm_solid& p, double px, double py, const lbm_solid& q, double qx,
                double qy, const lbm_grid& g) {
    double dx = std::fabs(px - qx);
    dx = std::fmod(dx, (double)g.nx);
    dx = std::min(dx, g.nx - dx);
    double dy = std::fabs(py - qy);
    if (!g.walls_y) {
        dy = std::fmod(dy, (double)g.ny);
        dy = std::min(dy, g.ny - dy);
    }
    if (p.shape == LBM_DISC && q.shape == LBM_DISC) return std::hypot(dx, dy) - p.a - q.a;
    double phx = p.a, phy = p.shape == LBM_DISC ? p.a : p.b;
    double qhx = q.a, qhy = q.shape == LBM_DISC ? q.a : q.b;
    return std::max(dx - phx - qhx, dy - phy - qhy);
}

const char* validate(const lbm_grid* g, double tau, const lbm_solid* s, int n, char* buf) {
    if (!g) return "grid is NULL";
    if (g->nx < 4 || g->ny < 4) return "nx and ny must be >= 4";
    if ((int64_t)g->nx * g->ny >= (1LL << 28)) return "nx*ny must be < 2^28";
    if (!(tau > 0.5)) return "tau must be > 1/2";
    if (dtype_size(g->dtype) == 0) return "unknown dtype";
    if (g->refill < 0 || g->refill > 2) return "unknown refill scheme";
    if (g->rho_w_local != 0) return "rho_w_local is not supported (must be 0)";
    if (!(g->rho0 > 0.0) || !std::isfinite(g->rho0)) return "rho0 must be > 0";
    if (!std::isfinite(g->gx) || !std::isfinite(g->gy)) return "body force must be finite";
    if (std::hypot(g->u0x, g->u0y) >= 0.3) return "|u0| must be < 0.3";
    if (std::hypot(g->wall_vx, g->wall_vy) >= 0.3) return "|wall velocity| must be < 0.3";
    if (n < 0 || n > kMaxSolids) return "n_solids must be in [0, 254]";
    if (n > 0 && !s) return "solids is NULL";
    for (int k = 0; k < n; ++k) {
        const lbm_solid& b = s[k];
        if (b.shape != LBM_DISC && b.shape != LBM_BOX) return "unknown solid shape";
        if (!std::isfinite(b.cx) || !std::isfinite(b.cy)) return "solid centre must be finite";
        if (b.shape == LBM_DISC && !(b.a > 0.0)) return "disc radius must be > 0";
        if (b.shape == LBM_BOX && !(b.a >= 0.0 && b.b >= 0.0)) return "box half-extents must be >= 0";
        if (std::hypot(b.vx, b.vy) >= 0.3) return "|solid velocity| must be < 0.3";
        double hx = b.a, hy = b.shape == LBM_DISC ? b.a : b.b;
        bool full_x = b.shape == LBM_BOX && 2 * hx + 1 >= g->nx;
        if (!full_x && 2 * hx + 6 >= g->nx) return "solid too wide for the lattice";
        if (b.moves && full_x) return "a translating solid must not span the lattice";
        if (g->walls_y) {
            if (b.cy - hy < 2.0 || b.cy + hy > g->ny - 3.0)
                return "solids must keep a gap of 2 nodes to the walls";
        } else if (2 * hy + 6 >= g->ny && !(b.shape == LBM_BOX && 2 * hy + 1 >= g->ny && !b.moves)) {
            return "solid too tall for the lattice";
        }
    }
    for (int p = 0; p < n; ++p)
        for (int q = p + 1; q < n; ++q) {
            const double need = (s[p].moves && s[q].moves) ? (double)kMoverGap : 2.0;
            if (body_gap(s[p], s[p].cx, s[p].cy, s[q], s[q].cx, s[q].cy, *g) < need) {
                snprintf(buf, 512, "solids %d and %d are closer than %g nodes", p + 1, q + 1, need);
                return buf;
            }
        }
    return nullptr;
}

}  // namespace

struct lbm_ctx {
    lbm_grid g;
    double tau;
    std::vector<lbm_solid> solids;
    int n;
    int64_t hist_cap;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    Layout L;
    int64_t t;
    std::vector<int> movers_h, frees_h;  // prescribed and free translating bodies
    std::vector<char> is_free;           // by solid id
    double Gx = 0.0, Gy = 0.0;           // gravity on free bodies
    int dyn_scheme = LBM_GME;            // force that drives them
    int mrt = 0;                        // collision operator: 0 BGK, 1 MRT
    int ibb = 0;                        // interpolated bounce-back on body links
    double mrt_s[3] = {0.0, 0.0, 0.0};  // MRT rates s_e, s_eps, s_q
    int64_t hist_first = 0;  // first step whose force record is held
    std::vector<int> seg_off, seg_cap;
    int64_t link_cap_total;
    char err[512];
    // blocks of kGraphSteps steps replayed as HIP graphs, one per start
    // parity (every kernel argument is fixed by the parity; the step counter
    // lives on the device), captured on a stream of the context's own
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    // the force totals of the last step are summed when first read (every
    // earlier step's are summed by the launch after it)
    bool fin_pending = false;
    // device whose static scratch holds the workspace (lbm_create_static), or -1
    int static_dev = -1;
    // instrumentation: event pairs around the lattice-update kernel
    bool prof = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    double prof_ms = 0.0;
    int64_t prof_n = 0;
};

namespace {

template <typename T>
T* wsp(lbm_ctx* c, size_t off) {
    return reinterpret_cast<T*>(c->ws + off);
}

StepArgs step_args(const lbm_ctx* c) {
    StepArgs a;
    a.nx = c->g.nx;
    a.ny = c->g.ny;
    a.rowlen = c->L.pitch;
    a.opitch = c->L.opitch;
    a.istride = c->L.pitch;
    a.ystride = 9 * (int64_t)c->L.pitch;
    a.walls = c->g.walls_y;
    a.rho0 = c->g.rho0;
    a.ibb = c->ibb;
    a.side_off = c->L.side_off;
    a.ref_off = c->L.ref_off;
    a.nseg = c->L.nseg;
    return a;
}

template <typename C>
CollideParams<C> collide_params(const lbm_ctx* c) {
    CollideParams<C> p{};
    p.rho0 = (C)c->g.rho0;
    p.omega = (C)(1.0 / c->tau);
    p.gx = (C)c->g.gx;
    p.gy = (C)c->g.gy;
    p.pref = (C)(1.0 - 1.0 / (2.0 * c->tau));
    p.mrt = c->mrt;
    p.s_e = (C)c->mrt_s[0];
    p.s_eps = (C)c->mrt_s[1];
    p.s_q = (C)c->mrt_s[2];
    return p;
}

ForceArgs force_args(const lbm_ctx* c) {
    ForceArgs a;
    a.nx = c->g.nx;
    a.ny = c->g.ny;
    a.walls = c->g.walls_y;
    a.istride = c->L.pitch;
    a.ystride = 9 * (int64_t)c->L.pitch;
    a.rho0 = c->g.rho0;
    a.hist_cap = c->hist_cap;
    a.nsol = c->n + 1;
    a.nchunks = c->L.nchunks;
    a.opitch = c->L.opitch;
    a.ibb = c->ibb;
    a.side_off = c->L.side_off;
    a.ref_off = c->L.ref_off;
    a.nseg = c->L.nseg;
    return a;
}

lbm_status hip_fail(lbm_ctx* c, hipError_t e, const char* what) {
    set_err(c ? c->err : g_err, "%s: %s", what, hipGetErrorString(e));
    return LBM_EDEVICE;
}

#define HIPCHK(ctx, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

int64_t node_blocks(const lbm_ctx* c) {
    return ((int64_t)c->g.ny * c->L.pitch + kBlock - 1) / kBlock;
}

// Update workgroups of the step launch: one node per lane, or two per lane
// (128 consecutive x per wave) with 16-bit storage.
template <typename T>
int64_t update_blocks(const lbm_ctx* c) {
    if constexpr (Sto<T>::kSplit)
        return ((int64_t)c->g.ny * ((c->L.pitch + 127) / 128) + kBlock / 64 - 1) / (kBlock / 64);
    return node_blocks(c);
}

// The two owner maps; with no translating body both views are the same map.
uint8_t* own_ptr(lbm_ctx* c, int k) {
    if (c->L.n_movers == 0) k = 0;
    return wsp<uint8_t>(c, c->L.own[k]);
}

// Enqueue one time step at parity p = t & 1 for storage type T: a single
// launch whose workgroups compute the forces on G_t, move the translating
// bodies (G_{t+1}, links, refill) and run the fused update.
template <typename T>
lbm_status enqueue_step(lbm_ctx* c) {
    using C = typename Sto<T>::C;
    const int p = (int)(c->t & 1);
    StepPtrs<T> sp;
    sp.fin = wsp<T>(c, c->L.f[p]);
    sp.fout = wsp<T>(c, c->L.f[p ^ 1]);
    sp.own_t = own_ptr(c, p);
    sp.own_n = own_ptr(c, p ^ 1);
    sp.links_t = wsp<uint32_t>(c, c->L.links[p]);
    sp.seg_cnt_t = wsp<int>(c, c->L.seg_cnt[p]);
    sp.links_n = wsp<uint32_t>(c, c->L.links[p ^ 1]);
    sp.seg_cnt_n = wsp<int>(c, c->L.seg_cnt[p ^ 1]);
    sp.seg_off = wsp<int>(c, c->L.seg_off);
    sp.seg_cap = wsp<int>(c, c->L.seg_cap);
    sp.chunk_solid = wsp<int>(c, c->L.chunk_solid);
    sp.chunk_start = wsp<int>(c, c->L.chunk_start);
    sp.solid_chunk0 = wsp<int>(c, c->L.solid_chunk0);
    sp.sol = wsp<SolidDev>(c, c->L.sol);
    const int ns = c->n + 1;
    sp.vtab = wsp<double>(c, c->L.vtab) + (size_t)p * 2 * ns;
    sp.rtab = wsp<double>(c, c->L.rtab) + (size_t)p * kRot * ns;
    sp.movers = wsp<int>(c, c->L.movers);
    sp.partial = wsp<double>(c, c->L.partial);
    sp.hist = wsp<double>(c, c->L.hist);
    sp.tctr = wsp<int64_t>(c, c->L.tctr);
    sp.errflag = wsp<int>(c, c->L.err);
    const int n_presc = (int)c->movers_h.size(), n_free = (int)c->frees_h.size();
    RoleCounts rc;
    rc.n_force = c->L.nchunks;
    rc.n_move = 2 * n_presc;  // geometry and refill workgroup per prescribed mover
    rc.n_bnd = c->ibb ? 2 * c->L.nchunks : 0;  // boundary role: two per link chunk
    rc.n_lead = (rc.n_force + rc.n_move + 1 + rc.n_bnd + 7) / 8 * 8;
    MoveArgs ma{c->g.nx, c->g.ny, c->L.opitch, c->g.walls_y, (int64_t)c->L.pitch,
                9 * (int64_t)c->L.pitch, c->g.rho0, c->g.refill, c->L.box_bytes, n_presc};
    ma.ibb = c->ibb;
    ma.side_off = c->L.side_off;
    ma.ref_off = c->L.ref_off;
    ma.nseg = c->L.nseg;
    StepArgs sa = step_args(c);
    ForceArgs fa = force_args(c);
    CollideParams<C> cp = collide_params<C>(c);
    const dim3 grid((unsigned)(rc.n_lead + update_blocks<T>(c)));
    const size_t lds = n_presc > 0 ? 2 * (size_t)c->L.box_bytes : 0;
    // both population buffers larger than the Infinity Cache: stream them
    const bool nt = 2 * c->L.pbytes > kStreamBytes;
    using KF = decltype(&k_fused<T, true, true, true>);
    KF kern;
    // per-link surface geometry: spinning free bodies or interpolated bounce-back
    if (n_free > 0 || c->ibb)
        kern = c->mrt ? (nt ? k_fused<T, true, true, true> : k_fused<T, false, true, true>)
                      : (nt ? k_fused<T, true, false, true> : k_fused<T, false, false, true>);
    else
        kern = c->mrt ? (nt ? k_fused<T, true, true, false> : k_fused<T, false, true, false>)
                      : (nt ? k_fused<T, true, false, false> : k_fused<T, false, false, false>);
    const bool timed = c->prof && c->ev_used + 2 <= c->ev.size();
    if (timed) {
        hipExtLaunchKernelGGL(kern, grid, dim3(kBlock), lds, c->stream, c->ev[c->ev_used],
                              c->ev[c->ev_used + 1], 0, sp, p, rc, sa, ma, fa, cp);
        c->ev_used += 2;
    } else {
        kern<<<grid, kBlock, lds, c->stream>>>(sp, p, rc, sa, ma, fa, cp);
    }
    if (n_free > 0) {
        // free bodies: Newton-Euler step from this step's forces, then their
        // G_{t+1}, links and refill (after the update: its partials are done)
        StepPtrs<T> fp = sp;
        fp.movers = wsp<int>(c, c->L.frees);
        MoveArgs fm = ma;
        fm.n_movers = n_free;
        FreeArgs fr;
        fr.dyn = wsp<FreeDyn>(c, c->L.fdyn);
        fr.partial = sp.partial + (size_t)p * fa.nchunks * 6;
        fr.solid_chunk0 = sp.solid_chunk0;
        fr.rtab = sp.rtab;
        fr.vtab_next = wsp<double>(c, c->L.vtab) + (size_t)(p ^ 1) * 2 * ns;
        fr.rtab_next = wsp<double>(c, c->L.rtab) + (size_t)(p ^ 1) * kRot * ns;
        fr.Gx = c->Gx;
        fr.Gy = c->Gy;
        fr.rho0 = c->g.rho0;
        fr.scheme = c->dyn_scheme == LBM_CME ? 0 : 1;
        auto kf = c->mrt ? k_free<T, true> : k_free<T, false>;
        kf<<<2 * n_free, kBlock, 2 * (size_t)c->L.box_bytes, c->stream>>>(fp, p, fm, fr, cp);
    }
    c->t += 1;
    return LBM_OK;
}

lbm_status dispatch_step(lbm_ctx* c) {
    switch (c->g.dtype) {
        case LBM_F64: return enqueue_step<double>(c);
        case LBM_F32: return enqueue_step<float>(c);
        case LBM_F16: return enqueue_step<_Float16>(c);
        default: return enqueue_step<bf16_t>(c);
    }
}

template <typename T, typename FT>
void enqueue_init(lbm_ctx* c, const FT* rho, const FT* ux, const FT* uy) {
    using C = typename Sto<T>::C;
    const int p = (int)(c->t & 1);
    k_init<T, FT><<<(unsigned)node_blocks(c), kBlock, 0, c->stream>>>(
        wsp<T>(c, c->L.f[p]), own_ptr(c, p), step_args(c), collide_params<C>(c), c->g.u0x,
        c->g.u0y, rho, ux, uy);
}

template <typename T>
void enqueue_init_poiseuille(lbm_ctx* c) {
    using C = typename Sto<T>::C;
    const int p = (int)(c->t & 1);
    k_init_poiseuille<T><<<(unsigned)node_blocks(c), kBlock, 0, c->stream>>>(
        wsp<T>(c, c->L.f[p]), own_ptr(c, p), step_args(c), collide_params<C>(c), c->g.gx, c->tau);
}

template <typename FT>
void dispatch_init(lbm_ctx* c, const FT* rho, const FT* ux, const FT* uy) {
    switch (c->g.dtype) {
        case LBM_F64: enqueue_init<double, FT>(c, rho, ux, uy); break;
        case LBM_F32: enqueue_init<float, FT>(c, rho, ux, uy); break;
        case LBM_F16: enqueue_init<_Float16, FT>(c, rho, ux, uy); break;
        default: enqueue_init<bf16_t, FT>(c, rho, ux, uy); break;
    }
}

// Host-side check that translating bodies keep their gaps over steps
// [t0, t1]: sampled so that relative displacement between samples is <= 0.1.
const char* check_paths(const lbm_ctx* c, int64_t t0, int64_t t1, char* buf) {
    const auto& S = c->solids;
    const lbm_grid& g = c->g;
    for (int p = 0; p < c->n; ++p) {
        if (!S[p].moves || c->is_free[p + 1]) continue;  // free bodies are checked on the device
        double hy = S[p].shape == LBM_DISC ? S[p].a : S[p].b;
        if (g.walls_y && S[p].vy != 0.0) {
            for (int64_t t : {t0, t1}) {
                double y = S[p].cy + (double)t * S[p].vy;
                if (y - hy < 2.0 || y + hy > g.ny - 3.0) {
                    snprintf(buf, 512, "solid %d reaches the walls before step %lld", p + 1, (long long)t1);
                    return buf;
                }
            }
        }
        for (int q = 0; q < c->n; ++q) {
            if (q == p || (S[q].moves && q < p) || c->is_free[q + 1]) continue;
            double rvx = S[p].vx - (S[q].moves ? S[q].vx : 0.0);
            double rvy = S[p].vy - (S[q].moves ? S[q].vy : 0.0);
            double rv = std::hypot(rvx, rvy);
            int64_t dt = rv > 0 ? std::max<int64_t>(1, (int64_t)(0.1 / rv)) : (t1 - t0 + 1);
            for (int64_t t = t0;; t += dt) {
                if (t > t1) t = t1;
                double px = S[p].cx + (double)t * S[p].vx, py = S[p].cy + (double)t * S[p].vy;
                double qx = S[q].moves ? S[q].cx + (double)t * S[q].vx : S[q].cx;
                double qy = S[q].moves ? S[q].cy + (double)t * S[q].vy : S[q].cy;
                const double need = S[q].moves ? (double)kMoverGap : 2.0;
                if (body_gap(S[p], px, py, S[q], qx, qy, g) < need) {
                    snprintf(buf, 512, "solids %d and %d come closer than %g nodes at step %lld", p + 1,
                             q + 1, need, (long long)t);
                    return buf;
                }
                if (t == t1) break;
            }
        }
    }
    return nullptr;
}

lbm_status read_err(lbm_ctx* c) {
    int e = 0;
    HIPCHK(c, hipMemcpyAsync(&e, wsp<int>(c, c->L.err), sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (e & 1) {
        set_err(c->err, "a link list overflowed its capacity");
        return LBM_EGEOM;
    }
    if (e & 2) {
        set_err(c->err, "non-finite or non-positive density detected");
        return LBM_ENUMERIC;
    }
    if (e & 8) {
        set_err(c->err, "a free body met a wall or another body, or moved more than half a node in a step");
        return LBM_EGEOM;
    }
    return LBM_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                     // guards the two tables below
void* g_scratch_ptr[kMaxDevices] = {};      // device address of each device's scratch
bool g_scratch_held[kMaxDevices] = {};      // a context lives in it

// Forget the captured step graphs (a setter changed what the launches take).
void drop_graphs(lbm_ctx* c) {
    for (auto& g : c->gexec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

// Capture kGraphSteps steps starting at parity p into c->gexec[p].
lbm_status capture_block(lbm_ctx* c, int p) {
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    const int64_t tsave = c->t;
    c->t = p;  // only the parity of t enters the launches
    c->stream = c->cap_stream;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    lbm_status rs = LBM_OK;
    if (e == hipSuccess)
        for (int k = 0; k < kGraphSteps && rs == LBM_OK; ++k) rs = dispatch_step(c);
    hipGraph_t g = nullptr;
    hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(c->cap_stream, &g) : e;
    c->stream = user;
    c->t = tsave;
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
    if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
    if (rs != LBM_OK) {
        (void)hipGraphDestroy(g);
        return rs;
    }
    e = hipGraphInstantiate(&c->gexec[p], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->gexec[p] = nullptr;
        return hip_fail(c, e, "hipGraphInstantiate");
    }
    return LBM_OK;
}

// Sum the last step's force totals if a reader needs them.
void finalize_pending(lbm_ctx* c) {
    if (!c->fin_pending) return;
    k_finalize<<<1, kBlock, 0, c->stream>>>(wsp<double>(c, c->L.partial), wsp<int>(c, c->L.solid_chunk0),
                                            wsp<double>(c, c->L.hist), wsp<int64_t>(c, c->L.tctr),
                                            (int)(c->t & 1), force_args(c));
    c->fin_pending = false;
}

}  // namespace

extern "C" {

int32_t lbm_abi_version(void) { return LBM_ABI_VERSION; }

lbm_status lbm_workspace_bytes(const lbm_grid* grid, const lbm_solid* solids, int32_t n_solids,
                               int64_t history_steps, size_t* bytes) {
    char buf[512];
    if (!bytes) {
        set_err(g_err, "bytes is NULL");
        return LBM_EINVAL;
    }
    const char* why = validate(grid, 0.75, solids, n_solids, buf);
    if (why) {
        set_err(g_err, "%s", why);
        return strstr(why, "closer") || strstr(why, "gap") ? LBM_EGEOM : LBM_EINVAL;
    }
    if (history_steps < 1) {
        set_err(g_err, "history_steps must be >= 1");
        return LBM_EINVAL;
    }
    Layout L;
    make_layout(*grid, solids, n_solids, history_steps, L);
    *bytes = L.total;
    return LBM_OK;
}

lbm_status lbm_create(const lbm_grid* grid, double tau, const lbm_solid* solids, int32_t n_solids,
                      int64_t history_steps, void* d_workspace, size_t bytes, void* hip_stream,
                      lbm_ctx** out) {
    char buf[512];
    if (!out) {
        set_err(g_err, "out is NULL");
        return LBM_EINVAL;
    }
    *out = nullptr;
    const char* why = validate(grid, tau, solids, n_solids, buf);
    if (why) {
        set_err(g_err, "%s", why);
        return strstr(why, "closer") || strstr(why, "gap") ? LBM_EGEOM : LBM_EINVAL;
    }
    if (history_steps < 1) {
        set_err(g_err, "history_steps must be >= 1");
        return LBM_EINVAL;
    }
    if (!d_workspace || ((uintptr_t)d_workspace & 255) != 0) {
        set_err(g_err, "workspace must be a non-NULL 256-byte aligned device pointer");
        return LBM_EINVAL;
    }
    Layout L;
    make_layout(*grid, solids, n_solids, history_steps, L);
    if (bytes < L.total) {
        set_err(g_err, "workspace too small: %zu < %zu bytes", bytes, L.total);
        return LBM_ESIZE;
    }
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) {
        set_err(g_err, "out of host memory");
        return LBM_EINVAL;
    }
    c->g = *grid;
    c->tau = tau;
    c->solids.assign(solids, solids + n_solids);
    c->n = n_solids;
    c->hist_cap = history_steps;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)d_workspace;
    c->ws_bytes = bytes;
    c->L = L;
    c->t = 0;
    c->err[0] = 0;

    // host tables
    const int ns = n_solids + 1;
    std::vector<SolidDev> sol(ns);
    std::vector<double> vtab(2 * ns);
    sol[0] = SolidDev{0, 0, 0, 0, grid->wall_vx, grid->wall_vy, 0, 0};
    vtab[0] = grid->wall_vx;
    vtab[1] = grid->wall_vy;
    std::vector<int> movers, all;
    for (int k = 0; k < n_solids; ++k) {
        const lbm_solid& b = solids[k];
        sol[k + 1] = SolidDev{b.cx, b.cy, b.a, b.b, b.vx, b.vy, b.shape, b.moves ? 1 : 0};
        vtab[2 * (k + 1)] = b.vx;
        vtab[2 * (k + 1) + 1] = b.vy;
        all.push_back(k + 1);
        if (b.moves) movers.push_back(k + 1);
    }
    c->seg_off.resize(ns);
    c->seg_cap.resize(ns);
    std::vector<int> seg_cnt(ns, 0), rec_off(ns, 0);
    int off = 0;
    c->seg_cap[0] = grid->walls_y ? 6 * grid->nx : 0;
    c->seg_off[0] = 0;
    seg_cnt[0] = c->seg_cap[0];
    off = c->seg_cap[0];
    for (int k = 0; k < n_solids; ++k) {
        c->seg_off[k + 1] = off;
        c->seg_cap[k + 1] = body_link_cap(solids[k], grid->nx, grid->ny);
        off += c->seg_cap[k + 1];
    }
    c->link_cap_total = off;
    // force chunks: each solid's segment split into kForceChunk-link pieces
    // (at least one per solid, so the final reduction always runs)
    std::vector<int> chunk_solid, chunk_start, solid_chunk0(ns + 1, 0);
    for (int sdx = 0; sdx < ns; ++sdx) {
        solid_chunk0[sdx] = (int)chunk_solid.size();
        const int nchk = std::max(1, (c->seg_cap[sdx] + kForceChunk - 1) / kForceChunk);
        for (int k = 0; k < nchk; ++k) {
            chunk_solid.push_back(sdx);
            chunk_start.push_back(k * kForceChunk);
        }
    }
    solid_chunk0[ns] = (int)chunk_solid.size();
    if ((int)chunk_solid.size() != L.nchunks) {
        set_err(g_err, "internal: chunk count mismatch");
        delete c;
        return LBM_EINVAL;
    }

    hipStream_t st = c->stream;
    auto up = [&](size_t dst, const void* src, size_t n) {
        return hipMemcpyAsync(c->ws + dst, src, n, hipMemcpyHostToDevice, st);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(L.sol, sol.data(), sizeof(SolidDev) * ns);
    if (e == hipSuccess) e = up(L.vtab, vtab.data(), sizeof(double) * 2 * ns);
    if (e == hipSuccess) e = up(L.vtab + sizeof(double) * 2 * ns, vtab.data(), sizeof(double) * 2 * ns);
    std::vector<double> rtab((size_t)2 * kRot * ns, 0.0);
    if (e == hipSuccess) e = up(L.rtab, rtab.data(), sizeof(double) * rtab.size());
    if (e == hipSuccess) e = up(L.seg_off, c->seg_off.data(), sizeof(int) * ns);
    if (e == hipSuccess) e = up(L.seg_cap, c->seg_cap.data(), sizeof(int) * ns);
    if (e == hipSuccess) e = up(L.seg_cnt[0], seg_cnt.data(), sizeof(int) * ns);
    if (e == hipSuccess) e = up(L.chunk_solid, chunk_solid.data(), sizeof(int) * chunk_solid.size());
    if (e == hipSuccess) e = up(L.chunk_start, chunk_start.data(), sizeof(int) * chunk_start.size());
    if (e == hipSuccess) e = up(L.solid_chunk0, solid_chunk0.data(), sizeof(int) * solid_chunk0.size());
    if (e == hipSuccess && !movers.empty()) e = up(L.movers, movers.data(), sizeof(int) * movers.size());
    c->movers_h = movers;
    c->is_free.assign(ns, 0);
    if (e == hipSuccess && !all.empty()) e = up(L.all, all.data(), sizeof(int) * all.size());
    // the uploads read pageable host vectors: finish them before they go away
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_err(g_err, "upload failed: %s", hipGetErrorString(e));
        delete c;
        return LBM_EDEVICE;
    }

    const int64_t own_bytes = (int64_t)grid->ny * L.opitch;
    k_set_counters<<<1, 1, 0, st>>>(wsp<int64_t>(c, L.tctr), 0, wsp<int>(c, L.err));
    k_fill_u8<<<(unsigned)((own_bytes + 255) / 256), 256, 0, st>>>(wsp<uint8_t>(c, L.own[0]), own_bytes, 0);
    GeomArgs ga{grid->nx, grid->ny, L.opitch, grid->walls_y};
    if (n_solids > 0)
        k_raster<<<n_solids, kBlock, 0, st>>>(wsp<uint8_t>(c, L.own[0]), wsp<SolidDev>(c, L.sol),
                                              wsp<int>(c, L.all), 0, ga);
    if (!movers.empty())
        e = hipMemcpyAsync(c->ws + L.own[1], c->ws + L.own[0], (size_t)own_bytes,
                           hipMemcpyDeviceToDevice, st);
    if (grid->walls_y)
        k_wall_links<<<(2 * grid->nx + 255) / 256, 256, 0, st>>>(wsp<uint32_t>(c, L.links[0]), grid->nx,
                                                                 grid->ny);
    LinkArgs la{grid->nx, grid->ny, L.opitch, grid->walls_y};
    if (n_solids > 0)
        k_links<<<n_solids, kBlock, 0, st>>>(wsp<uint8_t>(c, L.own[0]), wsp<uint32_t>(c, L.links[0]),
                                             wsp<int>(c, L.seg_cnt[0]), wsp<int>(c, L.seg_off),
                                             wsp<int>(c, L.seg_cap), wsp<SolidDev>(c, L.sol),
                                             wsp<int>(c, L.all), 0, la, wsp<int>(c, L.err));
    // both link buffers start as the lists of G_0 (translating bodies rewrite
    // theirs in the other buffer every step)
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + L.links[1], c->ws + L.links[0],
                           4 * (size_t)std::max<int64_t>(c->link_cap_total, 1), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + L.seg_cnt[1], c->ws + L.seg_cnt[0], 4 * (size_t)ns,
                           hipMemcpyDeviceToDevice, st);
    dispatch_init<double>(c, nullptr, nullptr, nullptr);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_err(g_err, "initialisation failed: %s", hipGetErrorString(e));
        delete c;
        return LBM_EDEVICE;
    }
    lbm_status rs = read_err(c);
    if (rs != LBM_OK) {
        set_err(g_err, "%s", c->err);
        delete c;
        return rs;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_create_static(const lbm_grid* grid, double tau, const lbm_solid* solids, int32_t n_solids,
                             int64_t history_steps, void* hip_stream, lbm_ctx** out) {
    if (!out) {
        set_err(g_err, "out is NULL");
        return LBM_EINVAL;
    }
    *out = nullptr;
    size_t need = 0;
    lbm_status rs = lbm_workspace_bytes(grid, solids, n_solids, history_steps, &need);
    if (rs != LBM_OK) return rs;
    if (need > kScratchBytes) {
        set_err(g_err, "this configuration needs %zu bytes of workspace; the static scratch holds %zu", need,
                kScratchBytes);
        return LBM_ESIZE;
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_err(g_err, "no usable current device (%s)", hipGetErrorString(e));
        return LBM_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_held[dev]) {
        set_err(g_err, "the static scratch of device %d is held by another context; destroy that one first", dev);
        return LBM_ESTATE;
    }
    if (!g_scratch_ptr[dev]) {  // first use on this device, which is current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_err(g_err, "hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
            return LBM_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    rs = lbm_create(grid, tau, solids, n_solids, history_steps, g_scratch_ptr[dev], kScratchBytes, hip_stream, out);
    if (rs == LBM_OK) {
        (*out)->static_dev = dev;
        g_scratch_held[dev] = true;
    }
    return rs;
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
    if (!c) return LBM_EINVAL;
    if (n < 0) {
        set_err(c->err, "n must be >= 0");
        return LBM_EINVAL;
    }
    if (n == 0) return LBM_OK;
    if (c->L.n_movers > 0) {
        char buf[512];
        const char* why = check_paths(c, c->t, c->t + n + 1, buf);
        if (why) {
            set_err(c->err, "%s", why);
            return LBM_EGEOM;
        }
    }
    c->fin_pending = false;  // the first launch sums the previous step's totals
    int64_t k = 0;
    // whole blocks as graph replays (not while timing single launches, and
    // not for a context that must not allocate: instantiating a graph may)
    while (!c->prof && c->static_dev < 0 && n - k >= kGraphSteps) {
        const int p = (int)(c->t & 1);
        if (!c->gexec[p]) {
            lbm_status rs = capture_block(c, p);
            if (rs != LBM_OK) return rs;
        }
        HIPCHK(c, hipGraphLaunch(c->gexec[p], c->stream));
        c->t += kGraphSteps;
        k += kGraphSteps;
    }
    for (; k < n; ++k) {
        lbm_status s = dispatch_step(c);
        if (s != LBM_OK) return s;
    }
    c->fin_pending = true;
    HIPCHK(c, hipGetLastError());
    return LBM_OK;
}

int64_t lbm_time(const lbm_ctx* c) { return c ? c->t : -1; }

lbm_status lbm_force(lbm_ctx* c, int32_t solid_id, int32_t scheme, double out[3]) {
    if (!c || !out) return LBM_EINVAL;
    if (solid_id < 0 || solid_id > c->n) {
        set_err(c->err, "solid_id %d out of range [0, %d]", solid_id, c->n);
        return LBM_EINVAL;
    }
    if (scheme != LBM_CME && scheme != LBM_GME) {
        set_err(c->err, "unknown scheme %d", scheme);
        return LBM_EINVAL;
    }
    if (c->t == 0 || c->t - 1 < c->hist_first) {
        set_err(c->err, "no step has been taken yet (since create or load)");
        return LBM_ESTATE;
    }
    finalize_pending(c);
    double rec[6];
    const int64_t slot = (c->t - 1) % c->hist_cap;
    const double* src = wsp<double>(c, c->L.hist) + (slot * (c->n + 1) + solid_id) * 6;
    HIPCHK(c, hipMemcpyAsync(rec, src, sizeof(rec), hipMemcpyDeviceToHost, c->stream));
    lbm_status rs = read_err(c);  // synchronises the stream
    if (rs != LBM_OK) return rs;
    const int o = scheme == LBM_CME ? 0 : 3;
    out[0] = rec[o];
    out[1] = rec[o + 1];
    out[2] = rec[o + 2];
    return LBM_OK;
}

lbm_status lbm_force_history(lbm_ctx* c, int64_t first, int64_t count, double* d_out) {
    if (!c || !d_out) return LBM_EINVAL;
    if (first < c->hist_first || count < 0 || first + count > c->t || first < c->t - c->hist_cap) {
        set_err(c->err, "steps [%lld, %lld) are not held by the history ring (t = %lld, capacity %lld)",
                (long long)first, (long long)(first + count), (long long)c->t, (long long)c->hist_cap);
        return LBM_EINVAL;
    }
    finalize_pending(c);
    const size_t row = (size_t)(c->n + 1) * 6 * sizeof(double);
    const char* base = c->ws + c->L.hist;
    int64_t k = 0;
    while (k < count) {
        int64_t slot = (first + k) % c->hist_cap;
        int64_t run = std::min<int64_t>(count - k, c->hist_cap - slot);
        HIPCHK(c, hipMemcpyAsync((char*)d_out + k * row, base + slot * row, run * row,
                                 hipMemcpyDeviceToDevice, c->stream));
        k += run;
    }
    return LBM_OK;
}

lbm_status lbm_fields(lbm_ctx* c, void* d_rho, void* d_ux, void* d_uy, int32_t out_dtype,
                      uint8_t* d_owner) {
    if (!c) return LBM_EINVAL;
    if (out_dtype != LBM_F64 && out_dtype != LBM_F32) {
        set_err(c->err, "fields are written as LBM_F64 or LBM_F32");
        return LBM_EINVAL;
    }
    const int p = (int)(c->t & 1);
    StepArgs sa = step_args(c);
    const uint8_t* own = own_ptr(c, p);
    int* errf = wsp<int>(c, c->L.err);
    const unsigned nb = (unsigned)node_blocks(c);
#define FIELDS_T(T)                                                                              \
    if (out_dtype == LBM_F64)                                                                    \
        k_fields<T, double><<<nb, kBlock, 0, c->stream>>>(wsp<T>(c, c->L.f[p]), own, sa, c->g.gx,  \
                                                          c->g.gy, (double*)d_rho, (double*)d_ux, \
                                                          (double*)d_uy, d_owner, errf);          \
    else                                                                                         \
        k_fields<T, float><<<nb, kBlock, 0, c->stream>>>(wsp<T>(c, c->L.f[p]), own, sa, c->g.gx,   \
                                                         c->g.gy, (float*)d_rho, (float*)d_ux,    \
                                                         (float*)d_uy, d_owner, errf);
    switch (c->g.dtype) {
        case LBM_F64: FIELDS_T(double) break;
        case LBM_F32: FIELDS_T(float) break;
        case LBM_F16: FIELDS_T(_Float16) break;
        default: FIELDS_T(bf16_t) break;
    }
#undef FIELDS_T
    HIPCHK(c, hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_init_fields(lbm_ctx* c, const void* d_rho, const void* d_ux, const void* d_uy,
                           int32_t in_dtype) {
    if (!c) return LBM_EINVAL;
    if (!d_rho || !d_ux || !d_uy) {
        set_err(c->err, "field pointers must not be NULL");
        return LBM_EINVAL;
    }
    if (in_dtype == LBM_F64)
        dispatch_init<double>(c, (const double*)d_rho, (const double*)d_ux, (const double*)d_uy);
    else if (in_dtype == LBM_F32)
        dispatch_init<float>(c, (const float*)d_rho, (const float*)d_ux, (const float*)d_uy);
    else {
        set_err(c->err, "fields are read as LBM_F64 or LBM_F32");
        return LBM_EINVAL;
    }
    HIPCHK(c, hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_set_boundary(lbm_ctx* c, int32_t rule) {
    if (!c) return LBM_EINVAL;
    if (rule != LBM_HALFWAY && rule != LBM_INTERPOLATED) {
        set_err(c->err, "rule must be LBM_HALFWAY or LBM_INTERPOLATED");
        return LBM_EINVAL;
    }
    c->ibb = rule == LBM_INTERPOLATED ? 1 : 0;
    drop_graphs(c);
    return LBM_OK;
}

lbm_status lbm_set_collision(lbm_ctx* c, int32_t model, const double* rates) {
    if (!c) return LBM_EINVAL;
    if (model != LBM_BGK && model != LBM_MRT) {
        set_err(c->err, "model must be LBM_BGK or LBM_MRT");
        return LBM_EINVAL;
    }
    if (model == LBM_MRT) {
        if (!rates) return LBM_EINVAL;
        for (int k = 0; k < 3; ++k)
            if (!(rates[k] > 0.0 && rates[k] < 2.0)) {
                set_err(c->err, "MRT rates must lie in (0, 2)");
                return LBM_EINVAL;
            }
    }
    if (c->t != 0) {
        set_err(c->err, "the collision operator is chosen before the first step");
        return LBM_ESTATE;
    }
    c->mrt = model == LBM_MRT ? 1 : 0;
    for (int k = 0; k < 3; ++k) c->mrt_s[k] = c->mrt ? rates[k] : 0.0;
    drop_graphs(c);
    // the start state is f_eq(rho0, u0) collided once with the chosen operator
    dispatch_init<double>(c, nullptr, nullptr, nullptr);
    HIPCHK(c, hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_set_free_body(lbm_ctx* c, int32_t solid_id, double rho_s, double omega0) {
    if (!c) return LBM_EINVAL;
    if (c->t != 0) {
        set_err(c->err, "free bodies are declared before the first step");
        return LBM_ESTATE;
    }
    if (solid_id < 1 || solid_id > c->n || !(rho_s > 0.0) || !std::isfinite(omega0)) {
        set_err(c->err, "solid_id must name a body and rho_s must be > 0");
        return LBM_EINVAL;
    }
    const lbm_solid& b = c->solids[solid_id - 1];
    if (b.shape != LBM_DISC || !b.moves) {
        set_err(c->err, "a free body must be a disc created with moves = 1");
        return LBM_EINVAL;
    }
    if (c->is_free[solid_id]) return LBM_OK;
    // the body leaves the prescribed movers and joins the free ones
    std::vector<int> presc;
    for (int s : c->movers_h)
        if (s != solid_id) presc.push_back(s);
    std::vector<int> frees = c->frees_h;
    frees.push_back(solid_id);
    const double pi = 3.14159265358979323846;
    FreeDyn d{};
    for (int k = 0; k < 3; ++k) {
        d.X[k] = b.cx;
        d.Y[k] = b.cy;
        d.Vx[k] = b.vx;
        d.Vy[k] = b.vy;
        d.Om[k] = omega0;
    }
    d.A = pi * b.a * b.a;
    d.M = rho_s * d.A;
    d.I = 0.5 * d.M * b.a * b.a;
    d.s = solid_id;
    const double rot[kRot] = {omega0, b.cx, b.cy, 1.0};
    const int ns = c->n + 1;
    hipStream_t st = c->stream;
    HIPCHK(c, hipStreamSynchronize(st));
    if (!presc.empty())
        HIPCHK(c, hipMemcpy(c->ws + c->L.movers, presc.data(), sizeof(int) * presc.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ws + c->L.frees, frees.data(), sizeof(int) * frees.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ws + c->L.fdyn + sizeof(FreeDyn) * (frees.size() - 1), &d, sizeof(FreeDyn),
                        hipMemcpyHostToDevice));
    for (int k = 0; k < 2; ++k)
        HIPCHK(c, hipMemcpy(c->ws + c->L.rtab + sizeof(double) * ((size_t)k * kRot * ns + (size_t)kRot * solid_id),
                            rot, sizeof(rot), hipMemcpyHostToDevice));
    c->movers_h = presc;
    c->frees_h = frees;
    drop_graphs(c);
    c->is_free[solid_id] = 1;
    return LBM_OK;
}

lbm_status lbm_set_gravity(lbm_ctx* c, double gx, double gy, int32_t scheme) {
    if (!c || !std::isfinite(gx) || !std::isfinite(gy) || (scheme != LBM_CME && scheme != LBM_GME))
        return LBM_EINVAL;
    c->Gx = gx;
    c->Gy = gy;
    c->dyn_scheme = scheme;
    drop_graphs(c);
    return LBM_OK;
}

lbm_status lbm_body_state(lbm_ctx* c, int32_t solid_id, double out[5]) {
    if (!c || !out || solid_id < 1 || solid_id > c->n) return LBM_EINVAL;
    lbm_status rs = read_err(c);
    if (rs != LBM_OK) return rs;
    const lbm_solid& b = c->solids[solid_id - 1];
    if (c->is_free[solid_id]) {
        size_t f = 0;
        while (c->frees_h[f] != solid_id) ++f;
        FreeDyn d;
        HIPCHK(c, hipMemcpy(&d, c->ws + c->L.fdyn + sizeof(FreeDyn) * f, sizeof(FreeDyn), hipMemcpyDeviceToHost));
        const int k = (int)(c->t % 3);
        out[0] = d.X[k];
        out[1] = d.Y[k];
        out[2] = d.Vx[k];
        out[3] = d.Vy[k];
        out[4] = d.Om[k];
        return LBM_OK;
    }
    const double tt = b.moves ? (double)c->t : 0.0;
    out[0] = b.cx + tt * b.vx;
    out[1] = b.cy + tt * b.vy;
    out[2] = b.vx;
    out[3] = b.vy;
    out[4] = 0.0;
    return LBM_OK;
}

lbm_status lbm_init_poiseuille(lbm_ctx* c) {
    if (!c) return LBM_EINVAL;
    if (!c->g.walls_y) {
        set_err(c->err, "the Poiseuille start needs walls at y (walls_y = 1)");
        return LBM_ESTATE;
    }
    switch (c->g.dtype) {
        case LBM_F64: enqueue_init_poiseuille<double>(c); break;
        case LBM_F32: enqueue_init_poiseuille<float>(c); break;
        case LBM_F16: enqueue_init_poiseuille<_Float16>(c); break;
        default: enqueue_init_poiseuille<bf16_t>(c); break;
    }
    HIPCHK(c, hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_populations(lbm_ctx* c, double* d_out) {
    if (!c || !d_out) return LBM_EINVAL;
    const int p = (int)(c->t & 1);
    StepArgs sa = step_args(c);
    const unsigned nb = (unsigned)node_blocks(c);
    const uint8_t* own = own_ptr(c, p);
    switch (c->g.dtype) {
        case LBM_F64: k_populations<double><<<nb, kBlock, 0, c->stream>>>(wsp<double>(c, c->L.f[p]), own, sa, d_out); break;
        case LBM_F32: k_populations<float><<<nb, kBlock, 0, c->stream>>>(wsp<float>(c, c->L.f[p]), own, sa, d_out); break;
        case LBM_F16: k_populations<_Float16><<<nb, kBlock, 0, c->stream>>>(wsp<_Float16>(c, c->L.f[p]), own, sa, d_out); break;
        default: k_populations<bf16_t><<<nb, kBlock, 0, c->stream>>>(wsp<bf16_t>(c, c->L.f[p]), own, sa, d_out); break;
    }
    HIPCHK(c, hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_link_forces(lbm_ctx* c, double* d_out, int64_t max, int64_t* n) {
    if (!c || !n) return LBM_EINVAL;
    const int ns = c->n + 1;
    std::vector<int> cnt(ns), roff(ns);
    const int pc = (int)(c->t & 1);
    HIPCHK(c, hipMemcpyAsync(cnt.data(), wsp<int>(c, c->L.seg_cnt[pc]), sizeof(int) * ns,
                             hipMemcpyDeviceToHost, c->stream));
    lbm_status rs = read_err(c);
    if (rs != LBM_OK) return rs;
    int64_t tot = 0;
    for (int s = 0; s < ns; ++s) {
        roff[s] = (int)tot;
        tot += cnt[s];
    }
    *n = tot;
    if (tot > max || (!d_out && tot > 0)) {
        set_err(c->err, "output holds %lld records, %lld needed", (long long)max, (long long)tot);
        return LBM_ESIZE;
    }
    if (tot == 0) return LBM_OK;
    HIPCHK(c, hipMemcpyAsync(wsp<int>(c, c->L.rec_off), roff.data(), sizeof(int) * ns,
                             hipMemcpyHostToDevice, c->stream));
    const int p = (int)(c->t & 1);
    ForceArgs fa = force_args(c);
    const uint32_t* links = wsp<uint32_t>(c, c->L.links[p]);
    const int* sc = wsp<int>(c, c->L.seg_cnt[p]);
    const int* so = wsp<int>(c, c->L.seg_off);
    const int* ro = wsp<int>(c, c->L.rec_off);
    const SolidDev* sol = wsp<SolidDev>(c, c->L.sol);
    const double* vt = wsp<double>(c, c->L.vtab) + (size_t)p * 2 * (c->n + 1);
    const double* rt = wsp<double>(c, c->L.rtab) + (size_t)p * kRot * (c->n + 1);
    const uint8_t* own = own_ptr(c, p);
    switch (c->g.dtype) {
        case LBM_F64: k_link_records<double><<<ns, kBlock, 0, c->stream>>>(wsp<double>(c, c->L.f[p]), own, links, sc, so, ro, sol, vt, rt, d_out, c->t, fa); break;
        case LBM_F32: k_link_records<float><<<ns, kBlock, 0, c->stream>>>(wsp<float>(c, c->L.f[p]), own, links, sc, so, ro, sol, vt, rt, d_out, c->t, fa); break;
        case LBM_F16: k_link_records<_Float16><<<ns, kBlock, 0, c->stream>>>(wsp<_Float16>(c, c->L.f[p]), own, links, sc, so, ro, sol, vt, rt, d_out, c->t, fa); break;
        default: k_link_records<bf16_t><<<ns, kBlock, 0, c->stream>>>(wsp<bf16_t>(c, c->L.f[p]), own, links, sc, so, ro, sol, vt, rt, d_out, c->t, fa); break;
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// Bytes of the state of one step: populations and, for 16-bit storage, the
// FP32 side array and the reference table.
size_t ckpt_pop_bytes(const lbm_ctx* c) { return c->L.pbytes + c->L.sbytes + c->L.rbytes; }

lbm_status lbm_checkpoint_bytes(const lbm_ctx* c, size_t* bytes) {
    if (!c || !bytes) return LBM_EINVAL;
    // populations (current buffer and, for 16-bit storage, its FP32 side
    // array), both owner maps, links + counts, counters
    *bytes = 64 + ckpt_pop_bytes(c) + 2 * (c->L.own[1] - c->L.own[0]) +
             4 * (size_t)std::max<int64_t>(c->link_cap_total, 1) + 4 * (size_t)(c->n + 1);
    return LBM_OK;
}

lbm_status lbm_save(lbm_ctx* c, void* d_dst, size_t bytes) {
    if (!c || !d_dst) return LBM_EINVAL;
    if (!c->frees_h.empty()) {
        set_err(c->err, "checkpoints do not hold the state of free bodies");
        return LBM_ESTATE;
    }
    size_t need;
    lbm_checkpoint_bytes(c, &need);
    if (bytes < need) {
        set_err(c->err, "checkpoint buffer too small: %zu < %zu", bytes, need);
        return LBM_ESIZE;
    }
    char* d = (char*)d_dst;
    int64_t hdr[8] = {0x6c626d63, (int64_t)LBM_ABI_VERSION, c->t, c->g.nx, c->g.ny, c->g.dtype, c->n, 0};
    const int p = (int)(c->t & 1);
    const size_t fb = c->L.pbytes, sb = c->L.sbytes, rb = c->L.rbytes;
    const size_t ob = c->L.own[1] - c->L.own[0];
    HIPCHK(c, hipMemcpyAsync(d, hdr, 64, hipMemcpyHostToDevice, c->stream));
    size_t o = 64;
    HIPCHK(c, hipMemcpyAsync(d + o, c->ws + c->L.f[p], fb, hipMemcpyDeviceToDevice, c->stream));
    o += fb;
    if (sb) HIPCHK(c, hipMemcpyAsync(d + o, c->ws + c->L.f[p] + c->L.side_off, sb, hipMemcpyDeviceToDevice, c->stream));
    o += sb;
    if (rb) HIPCHK(c, hipMemcpyAsync(d + o, c->ws + c->L.f[p] + c->L.ref_off, rb, hipMemcpyDeviceToDevice, c->stream));
    o += rb;
    HIPCHK(c, hipMemcpyAsync(d + o, own_ptr(c, p), ob, hipMemcpyDeviceToDevice, c->stream));
    o += ob;
    HIPCHK(c, hipMemcpyAsync(d + o, own_ptr(c, p ^ 1), ob, hipMemcpyDeviceToDevice, c->stream));
    o += ob;
    const size_t lb = 4 * (size_t)std::max<int64_t>(c->link_cap_total, 1);
    HIPCHK(c, hipMemcpyAsync(d + o, c->ws + c->L.links[p], lb, hipMemcpyDeviceToDevice, c->stream));
    o += lb;
    HIPCHK(c, hipMemcpyAsync(d + o, c->ws + c->L.seg_cnt[p], 4 * (size_t)(c->n + 1), hipMemcpyDeviceToDevice, c->stream));
    return read_err(c);
}

lbm_status lbm_load(lbm_ctx* c, const void* d_src, size_t bytes) {
    if (c && !c->frees_h.empty()) {
        set_err(c->err, "checkpoints do not hold the state of free bodies");
        return LBM_ESTATE;
    }
    if (!c || !d_src) return LBM_EINVAL;
    size_t need;
    lbm_checkpoint_bytes(c, &need);
    if (bytes < need) {
        set_err(c->err, "checkpoint buffer too small: %zu < %zu", bytes, need);
        return LBM_ESIZE;
    }
    const char* s = (const char*)d_src;
    int64_t hdr[8];
    HIPCHK(c, hipMemcpyAsync(hdr, s, 64, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (hdr[0] != 0x6c626d63 || hdr[1] != LBM_ABI_VERSION || hdr[3] != c->g.nx || hdr[4] != c->g.ny ||
        hdr[5] != c->g.dtype || hdr[6] != c->n || hdr[2] < 0) {
        set_err(c->err, "checkpoint does not match this context");
        return LBM_EINVAL;
    }
    c->t = hdr[2];
    const int p = (int)(c->t & 1);
    const size_t fb = c->L.pbytes, sb = c->L.sbytes, rb = c->L.rbytes;
    const size_t ob = c->L.own[1] - c->L.own[0];
    size_t o = 64;
    HIPCHK(c, hipMemcpyAsync(c->ws + c->L.f[p], s + o, fb, hipMemcpyDeviceToDevice, c->stream));
    o += fb;
    if (sb) HIPCHK(c, hipMemcpyAsync(c->ws + c->L.f[p] + c->L.side_off, s + o, sb, hipMemcpyDeviceToDevice, c->stream));
    o += sb;
    if (rb) HIPCHK(c, hipMemcpyAsync(c->ws + c->L.f[p] + c->L.ref_off, s + o, rb, hipMemcpyDeviceToDevice, c->stream));
    o += rb;
    HIPCHK(c, hipMemcpyAsync(own_ptr(c, p), s + o, ob, hipMemcpyDeviceToDevice, c->stream));
    o += ob;
    if (c->L.n_movers > 0)
        HIPCHK(c, hipMemcpyAsync(own_ptr(c, p ^ 1), s + o, ob, hipMemcpyDeviceToDevice, c->stream));
    o += ob;
    const size_t lb = 4 * (size_t)std::max<int64_t>(c->link_cap_total, 1);
    HIPCHK(c, hipMemcpyAsync(c->ws + c->L.links[p], s + o, lb, hipMemcpyDeviceToDevice, c->stream));
    o += lb;
    HIPCHK(c, hipMemcpyAsync(c->ws + c->L.seg_cnt[p], s + o, 4 * (size_t)(c->n + 1), hipMemcpyDeviceToDevice, c->stream));
    k_set_counters<<<1, 1, 0, c->stream>>>(wsp<int64_t>(c, c->L.tctr), c->t, wsp<int>(c, c->L.err));
    c->hist_first = c->t;  // force records before the checkpoint are not restored
    c->fin_pending = false;
    HIPCHK(c, hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_profile(lbm_ctx* c, int32_t enable) {
    if (!c) return LBM_EINVAL;
    c->prof = enable != 0;
    c->ev_used = 0;
    c->prof_ms = 0.0;
    c->prof_n = 0;
    if (c->prof && c->ev.empty()) {
        c->ev.resize(2 * 65536);
        for (auto& e : c->ev) HIPCHK(c, hipEventCreate(&e));
    }
    return LBM_OK;
}

lbm_status lbm_profile_read(lbm_ctx* c, double* update_ms, int64_t* launches) {
    if (!c || !update_ms || !launches) return LBM_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]));
        c->prof_ms += ms;
        c->prof_n += 1;
    }
    c->ev_used = 0;
    *update_ms = c->prof_ms;
    *launches = c->prof_n;
    return LBM_OK;
}

lbm_status lbm_status_check(lbm_ctx* c) {
    if (!c) return LBM_EINVAL;
    return read_err(c);
}

void lbm_destroy(lbm_ctx* c) {
    if (!c) return;
    drop_graphs(c);
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        g_scratch_held[c->static_dev] = false;
    }
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    delete c;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err : g_err; }

}  // extern "C"

#include "lbm_batch_capi.h"
