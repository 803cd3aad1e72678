// lbm_batch_capi.h -- host side of the batched C ABI (lbm_batch_* in
// include/lbm.h).  Included at the end of lbm_capi.hip: it shares that
// translation unit's validation and layout helpers.
#pragma once

#include <chrono>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "lbm_batch_kernels.h"

struct lbm_batch {
    int n = 0;
    int dtype = 0;
    hipStream_t user_stream = nullptr;
    hipStream_t run_stream = nullptr;  // graphs are captured and replayed here
    char* ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<lbm_grid> grids;
    std::vector<double> taus;
    std::vector<std::vector<lbm_solid>> solids;
    std::vector<CaseDev> cd;
    std::vector<BatchChunk> chunks;
    int max_nsol = 1;
    int n_tiles_max = 0;
    // layout (byte offsets)
    size_t o_cases, o_tiles, o_conv, o_f, o_side, o_own, o_snap, o_links, o_segcnt, o_segoff, o_segcap, o_sol,
        o_vtab, o_chunks, o_fpart, o_mpart, o_res, o_forces, o_tdev, o_tfirst, o_tcount, o_list, o_err;
    // current tiling
    int waves = 4;
    int nt = 1;
    int n_tiles = 0;
    std::vector<int> conv_h;  // host copy of the converged flags (at the last sync)
    int64_t t = 0;
    int64_t last_snap_t = -1;
    // captured interval
    hipGraphExec_t gexec = nullptr;
    int64_t graph_k = 0;
    double graph_tol = 0.0;
    bool use_graph = true;
    char err[512];
};

namespace {

template <typename T>
T* bws(lbm_batch* b, size_t off) {
    return reinterpret_cast<T*>(b->ws + off);
}

lbm_status bfail(lbm_batch* b, hipError_t e, const char* what) {
    set_err(b ? b->err : g_err, "%s: %s", what, hipGetErrorString(e));
    return LBM_EDEVICE;
}

#define BCHK(b, call)                                     \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return bfail(b, e_, #call); \
    } while (0)

struct BatchLayout {
    size_t total;
    std::vector<CaseDev> cd;
    std::vector<BatchChunk> chunks;
    std::vector<int> seg_off, seg_cap, solid_base;
    int max_nsol;
    int n_tiles_max;
    size_t o_cases, o_tiles, o_conv, o_f, o_side, o_own, o_snap, o_links, o_segcnt, o_segoff, o_segcap, o_sol,
        o_vtab, o_chunks, o_fpart, o_mpart, o_res, o_forces, o_tdev, o_tfirst, o_tcount, o_list, o_err;
};

const char* batch_layout(const lbm_grid* grids, const double* taus, const lbm_solid* solids,
                         const int32_t* n_solids, int n, BatchLayout& B, char* buf) {
    if (n < 1) return "n_cases must be >= 1";
    if (!grids || !taus || !n_solids) return "grids, taus and n_solids must not be NULL";
    const size_t es = dtype_size(grids[0].dtype);
    int64_t elem_off = 0, own_off = 0, snap_off = 0, side_el = 0;
    int links = 0, sbase = 0;
    B.max_nsol = 1;
    B.n_tiles_max = 0;
    B.cd.assign(n, CaseDev{});
    const lbm_solid* sp = solids;
    for (int c = 0; c < n; ++c) {
        const lbm_grid& g = grids[c];
        if (g.dtype != grids[0].dtype) return "all cases must share one dtype";
        const char* why = validate(&g, taus[c], sp, n_solids[c], buf);
        if (why) {
            snprintf(buf, 512, "case %d: %s", c, why);
            return buf;
        }
        for (int k = 0; k < n_solids[c]; ++k)
            if (sp[k].moves) return "batched cases have fixed geometry (moves = 0)";
        CaseDev& d = B.cd[c];
        const int pitch = (g.nx + 63) / 64 * 64;
        d.sa.nx = g.nx;
        d.sa.ny = g.ny;
        d.sa.rowlen = pitch;
        d.sa.opitch = pitch;
        d.sa.istride = pitch;
        d.sa.ystride = 9 * (int64_t)pitch;
        d.sa.walls = g.walls_y;
        d.sa.rho0 = g.rho0;
        d.cp64 = CollideParams<double>{g.rho0, 1.0 / taus[c], g.gx, g.gy, 1.0 - 1.0 / (2.0 * taus[c])};
        d.cp32 = CollideParams<float>{(float)g.rho0, (float)(1.0 / taus[c]), (float)g.gx, (float)g.gy,
                                      (float)(1.0 - 1.0 / (2.0 * taus[c]))};
        d.fa.nx = g.nx;
        d.fa.ny = g.ny;
        d.fa.walls = g.walls_y;
        d.fa.istride = pitch;
        d.fa.ystride = 9 * (int64_t)pitch;
        d.fa.rho0 = g.rho0;
        d.fa.hist_cap = 1;
        d.fa.nsol = n_solids[c] + 1;
        d.fa.nchunks = 0;
        const int64_t fel = 9 * (int64_t)g.ny * pitch;
        elem_off = (elem_off + 127) / 128 * 128;  // 256-byte aligned rows for every storage size
        d.f_off[0] = elem_off;
        d.sa.nseg = pitch >> kRefShift;
        d.fa.nseg = d.sa.nseg;
        if (es == 2) {
            // 16-bit storage: each buffer has its reference table right after
            // it; the two buffers sit at least one FP32 side array apart, so
            // that side arrays at one common distance from them do not overlap
            const int64_t ref_el = (fel + 127) / 128 * 128;               // byte offset 2 ref_el
            const int64_t rb_el = (int64_t)g.ny * d.sa.nseg * kSeg * 2;   // reference table (floats)
            d.sa.ref_off = 2 * ref_el;
            d.fa.ref_off = d.sa.ref_off;
            d.f_off[1] = elem_off + (std::max(2 * fel, ref_el + rb_el) + 127) / 128 * 128;
            elem_off = d.f_off[1] + ref_el + rb_el;
            d.sa.side_off = side_el;  // element offset in the side region for now
            side_el += 2 * (d.f_off[1] - d.f_off[0]);
        } else {
            d.f_off[1] = elem_off + (fel + 63) / 64 * 64;
            elem_off = d.f_off[1] + fel;
        }
        d.own_off = own_off;
        own_off += (int64_t)g.ny * pitch;
        d.snap_off = snap_off;
        snap_off += 2 * (int64_t)g.nx * g.ny;
        d.links_base = links;
        d.solid_base = sbase;
        d.nsol = n_solids[c] + 1;
        B.max_nsol = std::max(B.max_nsol, d.nsol);
        d.wpr = pitch / 64;
        d.nwaves = g.ny * d.wpr;
        B.n_tiles_max += d.nwaves;  // one wave per tile at the finest tiling
        // links and chunks: walls, then bodies
        int local = 0;
        d.chunk_first = (int)B.chunks.size();
        for (int s = 0; s < d.nsol; ++s) {
            const int cap = s == 0 ? (g.walls_y ? 6 * g.nx : 0) : body_link_cap(sp[s - 1], g.nx, g.ny);
            B.seg_off.push_back(local);
            B.seg_cap.push_back(cap);
            for (int k = 0; k < std::max(1, (cap + kForceChunk - 1) / kForceChunk); ++k)
                B.chunks.push_back(BatchChunk{c, s, k * kForceChunk});
            local += cap;
        }
        d.chunk_count = (int)B.chunks.size() - d.chunk_first;
        links += std::max(local, 1);
        sbase += d.nsol;
        sp += n_solids[c];
    }
    size_t off = 0;
    auto take = [&](size_t& o, size_t bytes) {
        o = off;
        off = align256(off + std::max<size_t>(bytes, 4));
    };
    take(B.o_cases, sizeof(CaseDev) * n);
    take(B.o_tiles, sizeof(Tile) * B.n_tiles_max);
    take(B.o_conv, 4 * (size_t)n);
    take(B.o_f, es * (size_t)elem_off);
    take(B.o_side, es * (size_t)side_el);
    if (es == 2)
        for (auto& d : B.cd) {
            // bytes from a case's population buffer to its FP32 side array
            d.sa.side_off = (int64_t)B.o_side + 2 * d.sa.side_off - (int64_t)(B.o_f + 2 * (size_t)d.f_off[0]);
            d.fa.side_off = d.sa.side_off;
        }
    take(B.o_own, (size_t)own_off);
    take(B.o_snap, 8 * (size_t)snap_off);
    take(B.o_links, 4 * (size_t)links);
    take(B.o_segcnt, 4 * (size_t)sbase);
    take(B.o_segoff, 4 * (size_t)sbase);
    take(B.o_segcap, 4 * (size_t)sbase);
    take(B.o_sol, sizeof(SolidDev) * sbase);
    take(B.o_vtab, 16 * (size_t)sbase);
    take(B.o_chunks, sizeof(BatchChunk) * B.chunks.size());
    take(B.o_fpart, 48 * B.chunks.size());
    take(B.o_mpart, 16 * (size_t)B.n_tiles_max);
    take(B.o_res, sizeof(CaseResult) * n);
    take(B.o_forces, 48 * (size_t)n * B.max_nsol);
    take(B.o_tdev, 16);
    take(B.o_tfirst, 4 * (size_t)n);
    take(B.o_tcount, 4 * (size_t)n);
    take(B.o_list, 4 * (size_t)B.max_nsol);
    take(B.o_err, 4);
    B.total = off;
    return nullptr;
}

// Tiles of the cases not yet converged, case by case; returns the count.
int build_tiles(lbm_batch* b, std::vector<Tile>& tiles, std::vector<int>& first, std::vector<int>& count) {
    tiles.clear();
    first.assign(b->n, 0);
    count.assign(b->n, 0);
    for (int c = 0; c < b->n; ++c) {
        first[c] = (int)tiles.size();
        if (b->conv_h[c]) continue;
        for (int w = 0; w < b->cd[c].nwaves; w += b->waves) tiles.push_back(Tile{c, w});
        count[c] = (int)tiles.size() - first[c];
    }
    return (int)tiles.size();
}

lbm_status upload_tiles(lbm_batch* b) {
    std::vector<Tile> tiles;
    std::vector<int> first, count;
    b->n_tiles = build_tiles(b, tiles, first, count);
    if (b->n_tiles > 0)
        BCHK(b, hipMemcpyAsync(b->ws + b->o_tiles, tiles.data(), sizeof(Tile) * tiles.size(),
                               hipMemcpyHostToDevice, b->run_stream));
    BCHK(b, hipMemcpyAsync(b->ws + b->o_tfirst, first.data(), 4 * (size_t)b->n, hipMemcpyHostToDevice,
                           b->run_stream));
    BCHK(b, hipMemcpyAsync(b->ws + b->o_tcount, count.data(), 4 * (size_t)b->n, hipMemcpyHostToDevice,
                           b->run_stream));
    BCHK(b, hipStreamSynchronize(b->run_stream));  // host vectors go out of scope
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    return LBM_OK;
}

template <typename T, bool NT, int W>
void launch_batch_step(lbm_batch* b, hipStream_t st) {
    const int p = (int)(b->t & 1);
    k_batch_step<T, NT, W><<<b->n_tiles, W * 64, 0, st>>>(
        bws<CaseDev>(b, b->o_cases), bws<Tile>(b, b->o_tiles), bws<int>(b, b->o_conv), bws<T>(b, b->o_f),
        bws<uint8_t>(b, b->o_own), bws<double>(b, b->o_vtab), p, bws<int64_t>(b, b->o_tdev));
}

template <typename T, bool NT>
void batch_step_w(lbm_batch* b, hipStream_t st) {
    switch (b->waves) {
        case 1: launch_batch_step<T, NT, 1>(b, st); break;
        case 2: launch_batch_step<T, NT, 2>(b, st); break;
        case 8: launch_batch_step<T, NT, 8>(b, st); break;
        default: launch_batch_step<T, NT, 4>(b, st); break;
    }
}

template <typename T>
void batch_step_t(lbm_batch* b, hipStream_t st) {
    if (b->nt)
        batch_step_w<T, true>(b, st);
    else
        batch_step_w<T, false>(b, st);
}

void batch_step_one(lbm_batch* b, hipStream_t st) {
    if (b->n_tiles > 0) {
        switch (b->dtype) {
            case LBM_F64: batch_step_t<double>(b, st); break;
            case LBM_F32: batch_step_t<float>(b, st); break;
            case LBM_F16: batch_step_t<_Float16>(b, st); break;
            default: batch_step_t<bf16_t>(b, st); break;
        }
    } else {
        // every case retired: keep the step counter moving
        k_set_counters<<<1, 1, 0, st>>>(bws<int64_t>(b, b->o_tdev), b->t + 1, bws<int>(b, b->o_err));
    }
    b->t += 1;
}

template <typename T, int W>
void batch_monitor_tw(lbm_batch* b, hipStream_t st, int k_steps, double tol) {
    const int p = (int)(b->t & 1);
    k_batch_force<T><<<(unsigned)b->chunks.size(), kBlock, 0, st>>>(
        bws<CaseDev>(b, b->o_cases), bws<BatchChunk>(b, b->o_chunks), bws<int>(b, b->o_conv),
        bws<T>(b, b->o_f), bws<uint32_t>(b, b->o_links), bws<int>(b, b->o_segcnt), bws<int>(b, b->o_segoff),
        bws<SolidDev>(b, b->o_sol), bws<double>(b, b->o_vtab), bws<double>(b, b->o_fpart), p, b->t);
    if (b->n_tiles > 0)
        k_batch_monitor<T, W><<<b->n_tiles, W * 64, 0, st>>>(
            bws<CaseDev>(b, b->o_cases), bws<Tile>(b, b->o_tiles), bws<int>(b, b->o_conv), bws<T>(b, b->o_f),
            bws<uint8_t>(b, b->o_own), bws<double>(b, b->o_snap), bws<double>(b, b->o_mpart), p);
    k_batch_finalize<<<(b->n + 255) / 256, 256, 0, st>>>(
        bws<CaseDev>(b, b->o_cases), bws<int>(b, b->o_tfirst), bws<int>(b, b->o_tcount),
        bws<double>(b, b->o_mpart), bws<BatchChunk>(b, b->o_chunks), bws<double>(b, b->o_fpart),
        bws<CaseResult>(b, b->o_res), bws<int>(b, b->o_conv), bws<double>(b, b->o_forces), b->max_nsol, b->n,
        bws<int64_t>(b, b->o_tdev), p, k_steps, tol);
}

template <typename T>
void batch_monitor_t(lbm_batch* b, hipStream_t st, int k_steps, double tol) {
    switch (b->waves) {
        case 1: batch_monitor_tw<T, 1>(b, st, k_steps, tol); break;
        case 2: batch_monitor_tw<T, 2>(b, st, k_steps, tol); break;
        case 8: batch_monitor_tw<T, 8>(b, st, k_steps, tol); break;
        default: batch_monitor_tw<T, 4>(b, st, k_steps, tol); break;
    }
}

void batch_monitor_one(lbm_batch* b, hipStream_t st, int k_steps, double tol) {
    switch (b->dtype) {
        case LBM_F64: batch_monitor_t<double>(b, st, k_steps, tol); break;
        case LBM_F32: batch_monitor_t<float>(b, st, k_steps, tol); break;
        case LBM_F16: batch_monitor_t<_Float16>(b, st, k_steps, tol); break;
        default: batch_monitor_t<bf16_t>(b, st, k_steps, tol); break;
    }
}

template <typename T>
void batch_init_case(lbm_batch* b, int c, hipStream_t st, const void* rho, const void* ux, const void* uy,
                     int in_dtype) {
    using C = typename Sto<T>::C;
    const CaseDev& d = b->cd[c];
    const int64_t nb = ((int64_t)d.sa.ny * d.sa.rowlen + kBlock - 1) / kBlock;
    CollideParams<C> cp{};
    cp.rho0 = (C)d.cp64.rho0;
    cp.omega = (C)d.cp64.omega;
    cp.gx = (C)d.cp64.gx;
    cp.gy = (C)d.cp64.gy;
    cp.pref = (C)d.cp64.pref;
    T* f = bws<T>(b, b->o_f) + d.f_off[b->t & 1];
    const uint8_t* own = bws<uint8_t>(b, b->o_own) + d.own_off;
    const lbm_grid& g = b->grids[c];
    if (rho == nullptr)
        k_init<T, double><<<(unsigned)nb, kBlock, 0, st>>>(f, own, d.sa, cp, g.u0x, g.u0y, nullptr, nullptr,
                                                           nullptr);
    else if (in_dtype == LBM_F64)
        k_init<T, double><<<(unsigned)nb, kBlock, 0, st>>>(f, own, d.sa, cp, g.u0x, g.u0y, (const double*)rho,
                                                           (const double*)ux, (const double*)uy);
    else
        k_init<T, float><<<(unsigned)nb, kBlock, 0, st>>>(f, own, d.sa, cp, g.u0x, g.u0y, (const float*)rho,
                                                          (const float*)ux, (const float*)uy);
}

template <typename T>
void batch_poiseuille_case(lbm_batch* b, int c, hipStream_t st) {
    using C = typename Sto<T>::C;
    const CaseDev& d = b->cd[c];
    const int64_t nb = ((int64_t)d.sa.ny * d.sa.rowlen + kBlock - 1) / kBlock;
    CollideParams<C> cp{};
    cp.rho0 = (C)d.cp64.rho0;
    cp.omega = (C)d.cp64.omega;
    cp.gx = (C)d.cp64.gx;
    cp.gy = (C)d.cp64.gy;
    cp.pref = (C)d.cp64.pref;
    k_init_poiseuille<T><<<(unsigned)nb, kBlock, 0, st>>>(bws<T>(b, b->o_f) + d.f_off[b->t & 1],
                                                         bws<uint8_t>(b, b->o_own) + d.own_off, d.sa, cp,
                                                         b->grids[c].gx, b->taus[c]);
}

void batch_init_dispatch(lbm_batch* b, int c, hipStream_t st, const void* rho, const void* ux,
                         const void* uy, int in_dtype) {
    switch (b->dtype) {
        case LBM_F64: batch_init_case<double>(b, c, st, rho, ux, uy, in_dtype); break;
        case LBM_F32: batch_init_case<float>(b, c, st, rho, ux, uy, in_dtype); break;
        case LBM_F16: batch_init_case<_Float16>(b, c, st, rho, ux, uy, in_dtype); break;
        default: batch_init_case<bf16_t>(b, c, st, rho, ux, uy, in_dtype); break;
    }
}

// Reset counters and results, initialise every case to f_eq(rho0, u0).
lbm_status batch_reset(lbm_batch* b) {
    hipStream_t st = b->run_stream;
    b->t = 0;
    b->last_snap_t = -1;
    std::fill(b->conv_h.begin(), b->conv_h.end(), 0);
    std::vector<CaseResult> res(b->n, CaseResult{0, 0, 0, -1.0});
    BCHK(b, hipMemcpyAsync(b->ws + b->o_conv, b->conv_h.data(), 4 * (size_t)b->n, hipMemcpyHostToDevice, st));
    BCHK(b, hipMemcpyAsync(b->ws + b->o_res, res.data(), sizeof(CaseResult) * b->n, hipMemcpyHostToDevice, st));
    k_set_counters<<<1, 1, 0, st>>>(bws<int64_t>(b, b->o_tdev), 0, bws<int>(b, b->o_err));
    for (int c = 0; c < b->n; ++c) batch_init_dispatch(b, c, st, nullptr, nullptr, nullptr, LBM_F64);
    BCHK(b, hipGetLastError());
    BCHK(b, hipStreamSynchronize(st));
    return upload_tiles(b);
}

lbm_status batch_sync_flags(lbm_batch* b) {
    BCHK(b, hipMemcpyAsync(b->conv_h.data(), b->ws + b->o_conv, 4 * (size_t)b->n, hipMemcpyDeviceToHost,
                           b->run_stream));
    BCHK(b, hipStreamSynchronize(b->run_stream));
    int e = 0;
    BCHK(b, hipMemcpy(&e, b->ws + b->o_err, 4, hipMemcpyDeviceToHost));
    if (e & 1) {
        set_err(b->err, "a link list overflowed its capacity");
        return LBM_EGEOM;
    }
    return LBM_OK;
}

// Order the run stream after the caller's stream (work enqueued there first).
lbm_status batch_join_user(lbm_batch* b) {
    if (b->user_stream == b->run_stream) return LBM_OK;
    hipEvent_t ev;
    BCHK(b, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    BCHK(b, hipEventRecord(ev, b->user_stream));
    BCHK(b, hipStreamWaitEvent(b->run_stream, ev, 0));
    BCHK(b, hipEventDestroy(ev));
    return LBM_OK;
}

// Cache key of a tuning result: device, dtype, case count, total nodes and
// an FNV-1a hash of the case sizes in order.
std::string batch_signature(const lbm_batch* b) {
    int64_t nodes = 0;
    uint64_t h = 1469598103934665603ull;
    for (const auto& g : b->grids) {
        nodes += (int64_t)g.nx * g.ny;
        for (int v : {g.nx, g.ny}) {
            h ^= (uint64_t)(uint32_t)v;
            h *= 1099511628211ull;
        }
    }
    std::ostringstream os;
    os << "gfx950;dtype=" << b->dtype << ";cases=" << b->n << ";nodes=" << nodes << ";sizes=" << std::hex << h;
    return os.str();
}

}  // namespace

extern "C" {

lbm_status lbm_batch_workspace_bytes(const lbm_grid* grids, const double* taus, const lbm_solid* solids,
                                     const int32_t* n_solids, int32_t n_cases, size_t* bytes) {
    char buf[512];
    BatchLayout B;
    if (!bytes) {
        set_err(g_err, "bytes is NULL");
        return LBM_EINVAL;
    }
    const char* why = batch_layout(grids, taus, solids, n_solids, n_cases, B, buf);
    if (why) {
        set_err(g_err, "%s", why);
        return strstr(why, "closer") || strstr(why, "gap") ? LBM_EGEOM : LBM_EINVAL;
    }
    *bytes = B.total;
    return LBM_OK;
}

lbm_status lbm_batch_create(const lbm_grid* grids, const double* taus, const lbm_solid* solids,
                            const int32_t* n_solids, int32_t n_cases, void* d_workspace, size_t bytes,
                            void* hip_stream, lbm_batch** out) {
    char buf[512];
    if (!out) {
        set_err(g_err, "out is NULL");
        return LBM_EINVAL;
    }
    *out = nullptr;
    BatchLayout B;
    const char* why = batch_layout(grids, taus, solids, n_solids, n_cases, B, buf);
    if (why) {
        set_err(g_err, "%s", why);
        return strstr(why, "closer") || strstr(why, "gap") ? LBM_EGEOM : LBM_EINVAL;
    }
    if (!d_workspace || ((uintptr_t)d_workspace & 255) != 0) {
        set_err(g_err, "workspace must be a non-NULL 256-byte aligned device pointer");
        return LBM_EINVAL;
    }
    if (bytes < B.total) {
        set_err(g_err, "workspace too small: %zu < %zu bytes", bytes, B.total);
        return LBM_ESIZE;
    }
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_EINVAL;
    b->n = n_cases;
    b->dtype = grids[0].dtype;
    b->user_stream = (hipStream_t)hip_stream;
    b->ws = (char*)d_workspace;
    b->ws_bytes = bytes;
    b->grids.assign(grids, grids + n_cases);
    b->taus.assign(taus, taus + n_cases);
    const lbm_solid* sp = solids;
    for (int c = 0; c < n_cases; ++c) {
        b->solids.emplace_back(sp, sp + n_solids[c]);
        sp += n_solids[c];
    }
    b->cd = B.cd;
    b->chunks = B.chunks;
    b->max_nsol = B.max_nsol;
    b->n_tiles_max = B.n_tiles_max;
    b->o_cases = B.o_cases; b->o_tiles = B.o_tiles; b->o_conv = B.o_conv; b->o_f = B.o_f; b->o_side = B.o_side;
    b->o_own = B.o_own; b->o_snap = B.o_snap; b->o_links = B.o_links; b->o_segcnt = B.o_segcnt;
    b->o_segoff = B.o_segoff; b->o_segcap = B.o_segcap; b->o_sol = B.o_sol; b->o_vtab = B.o_vtab; b->o_chunks = B.o_chunks;
    b->o_fpart = B.o_fpart; b->o_mpart = B.o_mpart; b->o_res = B.o_res; b->o_forces = B.o_forces;
    b->o_tdev = B.o_tdev; b->o_tfirst = B.o_tfirst; b->o_tcount = B.o_tcount; b->o_list = B.o_list;
    b->o_err = B.o_err;
    b->conv_h.assign(n_cases, 0);
    b->err[0] = 0;
    // the working set decides the streaming mode of the update
    size_t fb = 0;
    for (const auto& d : b->cd) fb += (size_t)(9 * (int64_t)d.sa.ny * d.sa.rowlen) * dtype_size(b->dtype) * 2;
    b->nt = fb > kStreamBytes ? 1 : 0;
    hipError_t e = hipStreamCreateWithFlags(&b->run_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        set_err(g_err, "stream creation failed: %s", hipGetErrorString(e));
        delete b;
        return LBM_EDEVICE;
    }
    hipStream_t st = b->run_stream;
    if (batch_join_user(b) != LBM_OK) {
        set_err(g_err, "%s", b->err);
        (void)hipStreamDestroy(b->run_stream);
        delete b;
        return LBM_EDEVICE;
    }
    // host tables
    std::vector<SolidDev> sol;
    std::vector<double> vtab;
    std::vector<int> segcnt;
    for (int c = 0; c < n_cases; ++c) {
        const lbm_grid& g = grids[c];
        sol.push_back(SolidDev{0, 0, 0, 0, g.wall_vx, g.wall_vy, 0, 0});
        vtab.push_back(g.wall_vx);
        vtab.push_back(g.wall_vy);
        segcnt.push_back(g.walls_y ? 6 * g.nx : 0);
        for (const auto& s : b->solids[c]) {
            sol.push_back(SolidDev{s.cx, s.cy, s.a, s.b, s.vx, s.vy, s.shape, 0});
            vtab.push_back(s.vx);
            vtab.push_back(s.vy);
            segcnt.push_back(0);
        }
    }
    std::vector<int> list(B.max_nsol);
    for (int k = 0; k < B.max_nsol; ++k) list[k] = k + 1;
    auto up = [&](size_t dst, const void* src, size_t nb) {
        return hipMemcpyAsync(b->ws + dst, src, nb, hipMemcpyHostToDevice, st);
    };
    if (e == hipSuccess) e = up(b->o_cases, b->cd.data(), sizeof(CaseDev) * n_cases);
    if (e == hipSuccess) e = up(b->o_chunks, b->chunks.data(), sizeof(BatchChunk) * b->chunks.size());
    if (e == hipSuccess) e = up(b->o_sol, sol.data(), sizeof(SolidDev) * sol.size());
    if (e == hipSuccess) e = up(b->o_vtab, vtab.data(), 8 * vtab.size());
    if (e == hipSuccess) e = up(b->o_segoff, B.seg_off.data(), 4 * B.seg_off.size());
    if (e == hipSuccess) e = up(b->o_segcap, B.seg_cap.data(), 4 * B.seg_cap.size());
    if (e == hipSuccess) e = up(b->o_segcnt, segcnt.data(), 4 * segcnt.size());
    if (e == hipSuccess) e = up(b->o_list, list.data(), 4 * list.size());
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    // geometry and links per case (one raster and one link workgroup per body)
    for (int c = 0; c < n_cases && e == hipSuccess; ++c) {
        const CaseDev& d = b->cd[c];
        const lbm_grid& g = grids[c];
        uint8_t* own = bws<uint8_t>(b, b->o_own) + d.own_off;
        const int64_t ob = (int64_t)g.ny * d.sa.opitch;
        k_fill_u8<<<(unsigned)((ob + 255) / 256), 256, 0, st>>>(own, ob, 0);
        GeomArgs ga{g.nx, g.ny, d.sa.opitch, g.walls_y};
        const int nb = d.nsol - 1;
        const SolidDev* sd = bws<SolidDev>(b, b->o_sol) + d.solid_base;
        if (nb > 0) k_raster<<<nb, kBlock, 0, st>>>(own, sd, bws<int>(b, b->o_list), 0, ga);
        uint32_t* L = bws<uint32_t>(b, b->o_links) + d.links_base;
        if (g.walls_y) k_wall_links<<<(2 * g.nx + 255) / 256, 256, 0, st>>>(L, g.nx, g.ny);
        if (nb > 0) {
            LinkArgs la{g.nx, g.ny, d.sa.opitch, g.walls_y};
            k_links<<<nb, kBlock, 0, st>>>(own, L, bws<int>(b, b->o_segcnt) + d.solid_base,
                                           bws<int>(b, b->o_segoff) + d.solid_base,
                                           bws<int>(b, b->o_segcap) + d.solid_base, sd, bws<int>(b, b->o_list),
                                           0, la, bws<int>(b, b->o_err));
        }
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_err(g_err, "batch initialisation failed: %s", hipGetErrorString(e));
        (void)hipStreamDestroy(b->run_stream);
        delete b;
        return LBM_EDEVICE;
    }
    k_set_counters<<<1, 1, 0, st>>>(bws<int64_t>(b, b->o_tdev), 0, bws<int>(b, b->o_err));
    lbm_status rs = batch_reset(b);
    if (rs == LBM_OK) rs = batch_sync_flags(b);
    if (rs != LBM_OK) {
        set_err(g_err, "%s", b->err);
        (void)hipStreamDestroy(b->run_stream);
        delete b;
        return rs;
    }
    *out = b;
    return LBM_OK;
}

int64_t lbm_batch_time(const lbm_batch* b) { return b ? b->t : -1; }

lbm_status lbm_batch_step(lbm_batch* b, int64_t n) {
    if (!b || n < 0) return LBM_EINVAL;
    lbm_status rs = batch_join_user(b);
    if (rs != LBM_OK) return rs;
    for (int64_t k = 0; k < n; ++k) batch_step_one(b, b->run_stream);
    BCHK(b, hipGetLastError());
    BCHK(b, hipStreamSynchronize(b->run_stream));
    return LBM_OK;
}

// Residual interval of a monitor call at the current step (1 when no
// snapshot exists yet: the call then only records one).
static int monitor_interval(const lbm_batch* b) {
    return b->last_snap_t < 0 ? 1 : (int)std::max<int64_t>(1, b->t - b->last_snap_t);
}

lbm_status lbm_batch_monitor(lbm_batch* b, double tol) {
    if (!b) return LBM_EINVAL;
    lbm_status rs = batch_join_user(b);
    if (rs != LBM_OK) return rs;
    batch_monitor_one(b, b->run_stream, monitor_interval(b), tol);
    b->last_snap_t = b->t;
    BCHK(b, hipGetLastError());
    const std::vector<int> before = b->conv_h;
    rs = batch_sync_flags(b);
    if (rs != LBM_OK) return rs;
    return before == b->conv_h ? LBM_OK : upload_tiles(b);
}

lbm_status lbm_batch_run(lbm_batch* b, int64_t max_steps, double tol, int32_t check_every, int64_t* steps_done) {
    if (!b) return LBM_EINVAL;
    if (check_every < 2 || max_steps < 0) {
        set_err(b->err, "check_every must be >= 2 and max_steps >= 0");
        return LBM_EINVAL;
    }
    const int k = check_every + (check_every & 1);  // even: a captured interval keeps its parity
    lbm_status rs = batch_join_user(b);
    if (rs != LBM_OK) return rs;
    const int64_t t0 = b->t;
    hipStream_t st = b->run_stream;
    if (steps_done) *steps_done = 0;
    if (b->last_snap_t != b->t) {  // snapshot of the starting state (retires nothing)
        batch_monitor_one(b, st, monitor_interval(b), -1.0);
        b->last_snap_t = b->t;
        BCHK(b, hipGetLastError());
    }
    if ((rs = batch_sync_flags(b)) != LBM_OK) return rs;
    int active = 0;
    for (int c = 0; c < b->n; ++c) active += b->conv_h[c] ? 0 : 1;
    while (active > 0 && b->t - t0 + k <= max_steps) {
        const bool even = (b->t & 1) == 0;
        if (b->use_graph && even && (b->gexec == nullptr || b->graph_k != k || b->graph_tol != tol)) {
            if (b->gexec) {
                (void)hipGraphExecDestroy(b->gexec);
                b->gexec = nullptr;
            }
            hipGraph_t g;
            const int64_t tsave = b->t;
            BCHK(b, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            for (int s = 0; s < k; ++s) batch_step_one(b, st);
            batch_monitor_one(b, st, k, tol);
            b->t = tsave;
            BCHK(b, hipStreamEndCapture(st, &g));
            hipError_t e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return bfail(b, e, "hipGraphInstantiate");
            b->graph_k = k;
            b->graph_tol = tol;
        }
        if (b->use_graph && even) {
            BCHK(b, hipGraphLaunch(b->gexec, st));
            b->t += k;
        } else {
            for (int s = 0; s < k; ++s) batch_step_one(b, st);
            batch_monitor_one(b, st, k, tol);
        }
        b->last_snap_t = b->t;
        BCHK(b, hipGetLastError());
        if ((rs = batch_sync_flags(b)) != LBM_OK) return rs;
        int now = 0;
        for (int c = 0; c < b->n; ++c) now += b->conv_h[c] ? 0 : 1;
        if (now != active && (rs = upload_tiles(b)) != LBM_OK) return rs;  // drop retired cases
        active = now;
        if (steps_done) *steps_done = b->t - t0;
    }
    return LBM_OK;
}

lbm_status lbm_batch_status(lbm_batch* b, int32_t* converged, int64_t* steps, double* residual, double* drag) {
    if (!b) return LBM_EINVAL;
    std::vector<CaseResult> res(b->n);
    std::vector<double> forces((size_t)b->n * b->max_nsol * 6);
    BCHK(b, hipStreamSynchronize(b->user_stream));
    BCHK(b, hipMemcpyAsync(res.data(), b->ws + b->o_res, sizeof(CaseResult) * b->n, hipMemcpyDeviceToHost,
                           b->run_stream));
    BCHK(b, hipMemcpyAsync(forces.data(), b->ws + b->o_forces, 8 * forces.size(), hipMemcpyDeviceToHost,
                           b->run_stream));
    BCHK(b, hipStreamSynchronize(b->run_stream));
    for (int c = 0; c < b->n; ++c) {
        if (converged) converged[c] = res[c].converged;
        if (steps) steps[c] = res[c].converged ? res[c].steps : b->t;
        if (residual) residual[c] = res[c].residual;
        if (drag) {
            double cme = 0.0, gme = 0.0;
            for (int s = 1; s < b->cd[c].nsol; ++s) {
                cme += forces[((size_t)c * b->max_nsol + s) * 6 + 0];
                gme += forces[((size_t)c * b->max_nsol + s) * 6 + 3];
            }
            drag[2 * c] = cme;
            drag[2 * c + 1] = gme;
        }
    }
    return LBM_OK;
}

lbm_status lbm_batch_force(lbm_batch* b, int32_t case_id, int32_t solid_id, int32_t scheme, double out[3]) {
    if (!b || !out || case_id < 0 || case_id >= b->n) return LBM_EINVAL;
    if (solid_id < 0 || solid_id >= b->cd[case_id].nsol || (scheme != LBM_CME && scheme != LBM_GME)) {
        set_err(b->err, "solid or scheme out of range");
        return LBM_EINVAL;
    }
    double rec[6];
    BCHK(b, hipStreamSynchronize(b->run_stream));
    BCHK(b, hipMemcpy(rec, b->ws + b->o_forces + 48 * ((size_t)case_id * b->max_nsol + solid_id), 48,
                      hipMemcpyDeviceToHost));
    const int o = scheme == LBM_CME ? 0 : 3;
    out[0] = rec[o];
    out[1] = rec[o + 1];
    out[2] = rec[o + 2];
    return LBM_OK;
}

lbm_status lbm_batch_fields(lbm_batch* b, int32_t case_id, void* d_rho, void* d_ux, void* d_uy,
                            int32_t out_dtype, uint8_t* d_owner) {
    if (!b || case_id < 0 || case_id >= b->n) return LBM_EINVAL;
    if (out_dtype != LBM_F64 && out_dtype != LBM_F32) {
        set_err(b->err, "fields are written as LBM_F64 or LBM_F32");
        return LBM_EINVAL;
    }
    CaseResult rr;
    lbm_status rs = batch_join_user(b);  // outputs may be in use on the caller's stream
    if (rs != LBM_OK) return rs;
    BCHK(b, hipStreamSynchronize(b->run_stream));
    BCHK(b, hipMemcpy(&rr, b->ws + b->o_res + sizeof(CaseResult) * case_id, sizeof(rr), hipMemcpyDeviceToHost));
    const int64_t tc = rr.converged ? rr.steps : b->t;
    const CaseDev& d = b->cd[case_id];
    const int p = (int)(tc & 1);
    const unsigned nb = (unsigned)(((int64_t)d.sa.ny * d.sa.rowlen + kBlock - 1) / kBlock);
    const uint8_t* own = bws<uint8_t>(b, b->o_own) + d.own_off;
    int* errf = bws<int>(b, b->o_err);
    hipStream_t st = b->run_stream;
#define BFIELDS_T(T)                                                                                      \
    if (out_dtype == LBM_F64)                                                                             \
        k_fields<T, double><<<nb, kBlock, 0, st>>>(bws<T>(b, b->o_f) + d.f_off[p], own, d.sa, d.cp64.gx,    \
                                                   d.cp64.gy, (double*)d_rho, (double*)d_ux, (double*)d_uy, \
                                                   d_owner, errf);                                        \
    else                                                                                                  \
        k_fields<T, float><<<nb, kBlock, 0, st>>>(bws<T>(b, b->o_f) + d.f_off[p], own, d.sa, d.cp64.gx,     \
                                                  d.cp64.gy, (float*)d_rho, (float*)d_ux, (float*)d_uy,   \
                                                  d_owner, errf);
    switch (b->dtype) {
        case LBM_F64: BFIELDS_T(double) break;
        case LBM_F32: BFIELDS_T(float) break;
        case LBM_F16: BFIELDS_T(_Float16) break;
        default: BFIELDS_T(bf16_t) break;
    }
#undef BFIELDS_T
    BCHK(b, hipGetLastError());
    BCHK(b, hipStreamSynchronize(st));
    return LBM_OK;
}

lbm_status lbm_batch_init_fields(lbm_batch* b, int32_t case_id, const void* d_rho, const void* d_ux,
                                 const void* d_uy, int32_t in_dtype) {
    if (!b || case_id < 0 || case_id >= b->n) return LBM_EINVAL;
    const bool cold = !d_rho && !d_ux && !d_uy;
    if (!cold && (!d_rho || !d_ux || !d_uy)) {
        set_err(b->err, "give all three fields, or none for the cold start");
        return LBM_EINVAL;
    }
    if (!cold && in_dtype != LBM_F64 && in_dtype != LBM_F32) {
        set_err(b->err, "fields are read as LBM_F64 or LBM_F32");
        return LBM_EINVAL;
    }
    if (b->conv_h[case_id]) {
        set_err(b->err, "case %d has retired", case_id);
        return LBM_ESTATE;
    }
    lbm_status rs = batch_join_user(b);
    if (rs != LBM_OK) return rs;
    batch_init_dispatch(b, case_id, b->run_stream, d_rho, d_ux, d_uy, in_dtype);
    BCHK(b, hipGetLastError());
    // the residual starts over: the next check records a snapshot only
    CaseResult rr;
    char* rp = b->ws + b->o_res + sizeof(CaseResult) * case_id;
    BCHK(b, hipMemcpyAsync(&rr, rp, sizeof(rr), hipMemcpyDeviceToHost, b->run_stream));
    BCHK(b, hipStreamSynchronize(b->run_stream));
    rr.have_snap = 0;
    rr.residual = -1.0;
    BCHK(b, hipMemcpyAsync(rp, &rr, sizeof(rr), hipMemcpyHostToDevice, b->run_stream));
    BCHK(b, hipStreamSynchronize(b->run_stream));
    return LBM_OK;
}

lbm_status lbm_batch_init_poiseuille(lbm_batch* b, int32_t case_id) {
    if (!b || case_id < 0 || case_id >= b->n) return LBM_EINVAL;
    if (!b->grids[case_id].walls_y) {
        set_err(b->err, "the Poiseuille start needs walls at y (walls_y = 1)");
        return LBM_ESTATE;
    }
    if (b->conv_h[case_id]) {
        set_err(b->err, "case %d has retired", case_id);
        return LBM_ESTATE;
    }
    lbm_status rs = batch_join_user(b);
    if (rs != LBM_OK) return rs;
    switch (b->dtype) {
        case LBM_F64: batch_poiseuille_case<double>(b, case_id, b->run_stream); break;
        case LBM_F32: batch_poiseuille_case<float>(b, case_id, b->run_stream); break;
        case LBM_F16: batch_poiseuille_case<_Float16>(b, case_id, b->run_stream); break;
        default: batch_poiseuille_case<bf16_t>(b, case_id, b->run_stream); break;
    }
    BCHK(b, hipGetLastError());
    BCHK(b, hipStreamSynchronize(b->run_stream));
    return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch* b, const char* cache_path) {
    if (!b) return LBM_EINVAL;
    if (b->t != 0) {
        set_err(b->err, "autotune before the first step");
        return LBM_ESTATE;
    }
    const std::string key = batch_signature(b);
    // cache: one "key|waves|nt|us" line per signature
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k2;
            int w = 0, nt = 0;
            if (std::getline(ls, k2, '|') && k2 == key) {
                char bar;
                ls >> w >> bar >> nt;
                if (w == 1 || w == 2 || w == 4 || w == 8) {
                    b->waves = w;
                    b->nt = nt ? 1 : 0;
                    return upload_tiles(b);
                }
            }
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double best = 1e300;
    int bw = 4, bnt = b->nt;
    const int cand_w[4] = {1, 2, 4, 8};
    lbm_status rs = LBM_OK;
    for (int nt = 0; nt < 2 && e == hipSuccess && rs == LBM_OK; ++nt)
        for (int wi = 0; wi < 4 && e == hipSuccess && rs == LBM_OK; ++wi) {
            rs = lbm_batch_set_tiling(b, cand_w[wi], nt);
            if (rs != LBM_OK) break;
            for (int s = 0; s < 3; ++s) batch_step_one(b, b->run_stream);  // warm-up
            const int R = 12;
            e = hipEventRecord(e0, b->run_stream);
            for (int s = 0; s < R; ++s) batch_step_one(b, b->run_stream);
            if (e == hipSuccess) e = hipEventRecord(e1, b->run_stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms / R < best) {
                best = ms / R;
                bw = cand_w[wi];
                bnt = nt;
            }
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return bfail(b, e, "autotune timing");
    if (rs != LBM_OK) return rs;
    b->waves = bw;
    b->nt = bnt;
    if (cache_path) {
        std::ofstream outf(cache_path, std::ios::app);
        outf << key << "|" << bw << "|" << bnt << "|" << best * 1e3 << "\n";
    }
    return batch_reset(b);  // the timing steps advanced the state: start over
}

lbm_status lbm_batch_set_active(lbm_batch* b, int32_t case_id, int32_t active) {
    if (!b || case_id < 0 || case_id >= b->n) return LBM_EINVAL;
    lbm_status rs = batch_sync_flags(b);
    if (rs != LBM_OK) return rs;
    CaseResult rr;
    BCHK(b, hipMemcpy(&rr, b->ws + b->o_res + sizeof(CaseResult) * case_id, sizeof(rr), hipMemcpyDeviceToHost));
    if (active) {
        if (!b->conv_h[case_id]) return LBM_OK;
        const CaseDev& d = b->cd[case_id];
        if ((rr.steps & 1) != (b->t & 1)) {  // the frozen state sits in the other buffer
            const size_t es = dtype_size(b->dtype);
            const size_t bytes = (size_t)(9 * (int64_t)d.sa.ny * d.sa.rowlen) * es;
            char* dst = b->ws + b->o_f + es * d.f_off[b->t & 1];
            const char* src = b->ws + b->o_f + es * d.f_off[rr.steps & 1];
            BCHK(b, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, b->run_stream));
            if (es == 2) {  // and the FP32 side array and the reference table
                BCHK(b, hipMemcpyAsync(dst + d.sa.side_off, src + d.sa.side_off, 2 * bytes, hipMemcpyDeviceToDevice,
                                       b->run_stream));
                const size_t rb = (size_t)d.sa.ny * d.sa.nseg * kSeg * 4;
                BCHK(b, hipMemcpyAsync(dst + d.sa.ref_off, src + d.sa.ref_off, rb, hipMemcpyDeviceToDevice,
                                       b->run_stream));
            }
        }
        rr.converged = 0;
        rr.have_snap = 0;
        rr.residual = -1.0;
        b->conv_h[case_id] = 0;
    } else {
        if (b->conv_h[case_id]) return LBM_OK;
        rr.converged = 1;
        rr.steps = b->t;
        b->conv_h[case_id] = 1;
    }
    BCHK(b, hipMemcpyAsync(b->ws + b->o_res + sizeof(CaseResult) * case_id, &rr, sizeof(rr), hipMemcpyHostToDevice,
                           b->run_stream));
    BCHK(b, hipMemcpyAsync(b->ws + b->o_conv, b->conv_h.data(), 4 * (size_t)b->n, hipMemcpyHostToDevice,
                           b->run_stream));
    BCHK(b, hipStreamSynchronize(b->run_stream));
    return upload_tiles(b);
}

lbm_status lbm_batch_set_tiling(lbm_batch* b, int32_t waves, int32_t nontemporal) {
    if (!b) return LBM_EINVAL;
    if (waves != 1 && waves != 2 && waves != 4 && waves != 8) {
        set_err(b->err, "waves per workgroup must be 1, 2, 4 or 8");
        return LBM_EINVAL;
    }
    b->waves = waves;
    b->nt = nontemporal ? 1 : 0;
    return upload_tiles(b);
}

lbm_status lbm_batch_set_graph(lbm_batch* b, int32_t enable) {
    if (!b) return LBM_EINVAL;
    b->use_graph = enable != 0;
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    return LBM_OK;
}

int32_t lbm_batch_tiling(const lbm_batch* b, int32_t* nontemporal) {
    if (!b) return -1;
    if (nontemporal) *nontemporal = b->nt;
    return b->waves;
}

void lbm_batch_destroy(lbm_batch* b) {
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->run_stream) {
        (void)hipStreamSynchronize(b->run_stream);
        (void)hipStreamDestroy(b->run_stream);
    }
    delete b;
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err : g_err; }

}  // extern "C"
