// nn_capi.hip -- host side of the warm-start network ABI (lbm_nn_* in
// include/lbm.h): workspace layout, layer table, and the launch sequences of
// the forward pass, the backward pass, Adam and inference.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "nn_kernels.h"

using namespace nn;

namespace {

thread_local char g_nn_err[512] = "";

void nn_set_err(char* buf, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
}

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr int kLayers = 15;

// Activation and gradient tensors (NHWC, compute type), by name.
enum Buf {
    X0, A0, CAT0, X1, A1, CAT1, X2, A2, CAT2, X3, B1, B2, D2A, D2B, D1A, D1B, D0A, D0B,
    G_HEAD, G_D0B, G_D0A, G_CAT0, G_D1B, G_D1A, G_CAT1, G_D2B, G_D2A, G_CAT2, G_B2, G_B1, G_X3,
    G_S2, G_A2, G_X2, G_S1, G_A1, G_X1, G_S0, G_A0, GMEAN, NBUF
};

struct BufShape {
    int level;
    int ch;
};

struct Plan {
    int H, W, B;
    int c[4];
    int es;  // bytes per element of the compute type
    BufShape shape[NBUF];
    LayerDev L[kLayers];
    int64_t n_params, wf_total, wt_total, b_total;
    int level[kLayers];  // level of each layer's input
    int64_t wpart_max;  // floats of the largest weight-gradient partial
    int64_t bpart_max;  // floats of the largest bias partial
    size_t off[NBUF];
    size_t o_master, o_grad, o_m, o_v, o_wf, o_wt, o_bias, o_out, o_tgt, o_fluid, o_wpart, o_bpart,
        o_lpart, o_loss, o_idx, o_gmean, total;
};

int64_t pixels(const Plan& p, int level) { return (int64_t)p.B * (p.H >> level) * (p.W >> level); }

// Splits of the weight-gradient GEMM of a layer whose input lives at `level`.
void wgrad_split(const Plan& p, int level, int tiles, int& splits, int& chunk) {
    const int64_t P = pixels(p, level);
    int s = std::max(1, 2048 / std::max(tiles, 1));
    s = (int)std::min<int64_t>(s, std::max<int64_t>(1, P / 256));
    chunk = (int)(((P + s - 1) / s + 63) / 64 * 64);
    splits = (int)((P + chunk - 1) / chunk);
}

int mb_of(int cout_pad) { return cout_pad % 64 == 0 ? 2 : 1; }

// The nine-tap weight-gradient kernel takes BF16 levels whose row length is
// a multiple of its tile.
bool wgrad9_ok(const Plan& p, int level) { return p.es == 2 && ((p.W >> level) % kWgTile) == 0; }

// Splits of the nine-tap kernel: the count that minimises a cost model of
// the products (tiles per split times the per-tile time of one workgroup,
// in rounds of 512 workgroups) plus the split partials written and read.
// Rates are those measured for this kernel on MI355X: ~3 TFLOP/s per
// workgroup of 6 waves (2.25 of 3), partial round trip ~5 TB/s.
void wgrad9_split(int64_t ntiles, int pairs, int mb, int nb, int64_t nwb, int& splits, int& tps) {
    const double tile_flop = 2.0 * kWgTile * (32.0 * mb) * (32.0 * nb) * 9.0;
    const double rate = 3.0e12 * (nb == 2 ? 1.0 : 0.75);
    double best = 1e300;
    splits = 1;
    tps = (int)ntiles;
    const int smax = (int)std::min<int64_t>(ntiles, 1024);
    for (int s = 1; s <= smax; ++s) {
        const int64_t tp = (ntiles + s - 1) / s;
        const int64_t sp = (ntiles + tp - 1) / tp;
        const int64_t wgs = sp * pairs;
        const double rounds = (double)((wgs + 511) / 512);
        const double est = rounds * (double)tp * tile_flop / rate + 8.0 * (double)sp * (double)nwb / 5.0e12;
        if (est < best - 1e-12) {
            best = est;
            splits = (int)sp;
            tps = (int)tp;
        }
    }
}

// Nodes per workgroup of a column sum: 8 per thread lane (kEw / C lanes per
// channel), so a sum over few nodes with many channels still spreads over
// many workgroups.
constexpr int kColPerLane = 8;
int col_rows(int C) { return kColPerLane * (kEw / C); }

const char* make_plan(const lbm_nn_config& cfg, Plan& p) {
    if (cfg.h < 8 || cfg.h % 8 != 0) return "h must be a positive multiple of 8";
    if (cfg.w < 64 || cfg.w % 64 != 0) return "w must be a positive multiple of 64";
    if (cfg.max_batch < 1) return "max_batch must be >= 1";
    if (cfg.dtype != LBM_BF16 && cfg.dtype != LBM_F32) return "dtype must be LBM_BF16 or LBM_F32";
    for (int k = 0; k < 4; ++k)
        if (cfg.ch[k] < 32 || cfg.ch[k] % 32 != 0 || cfg.ch[k] > 1024) return "channels must be multiples of 32 in [32, 1024]";
    if (cfg.ch[3] > kEw) return "the bottleneck width ch[3] must be <= 256 (its channel means)";
    if (!(cfg.rho_scale > 0.0)) return "rho_scale must be > 0";
    if ((int64_t)cfg.max_batch * cfg.h * cfg.w >= (1LL << 31) / 32) return "max_batch * h * w too large";
    p.H = cfg.h;
    p.W = cfg.w;
    p.B = cfg.max_batch;
    for (int k = 0; k < 4; ++k) p.c[k] = cfg.ch[k];
    p.es = cfg.dtype == LBM_BF16 ? 2 : 4;
    const int c0 = p.c[0], c1 = p.c[1], c2 = p.c[2], c3 = p.c[3];
    const BufShape sh[NBUF] = {
        {0, 16}, {0, c0}, {0, c1 + c0}, {1, c0}, {1, c1}, {1, c2 + c1}, {2, c1}, {2, c2}, {2, 2 * c3 + c2}, {3, c2},
        {3, c3}, {3, c3}, {2, c2}, {2, c2}, {1, c1}, {1, c1}, {0, c0}, {0, c0},
        {0, 32}, {0, c0}, {0, c0}, {0, c1 + c0}, {1, c1}, {1, c1}, {1, c2 + c1}, {2, c2}, {2, c2}, {2, 2 * c3 + c2},
        {3, c3}, {3, c3}, {3, c2}, {2, c2}, {2, c2}, {2, c1}, {1, c1}, {1, c1}, {1, c0}, {0, c0}, {0, c0},
        {-1, c3}};
    for (int k = 0; k < NBUF; ++k) p.shape[k] = sh[k];
    const int cin[kLayers] = {2, c0, c0, c1, c1, c2, c2, c3, 2 * c3 + c2, c2, c2 + c1, c1, c1 + c0, c0, c0};
    const int cout[kLayers] = {c0, c0, c1, c1, c2, c2, c3, c3, c2, c2, c1, c1, c0, c0, 3};
    int64_t off = 0, wf = 0, wt = 0, bo = 0;
    p.wpart_max = 1;
    p.bpart_max = 1;
    const int level_in[kLayers] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0};
    for (int k = 0; k < kLayers; ++k) p.level[k] = level_in[k];
    for (int k = 0; k < kLayers; ++k) {
        LayerDev& L = p.L[k];
        L.off = off;
        L.cin = cin[k];
        L.cout = cout[k];
        L.cin_pad = (cin[k] + 15) / 16 * 16;
        L.cout_pad = (cout[k] + 31) / 32 * 32;
        L.cin_dg = (cin[k] + 31) / 32 * 32;
        L.wf_off = wf;
        L.wt_off = wt;
        L.b_off = bo;
        off += (int64_t)cout[k] * 9 * cin[k] + cout[k];
        wf += (int64_t)L.cout_pad * 9 * L.cin_pad;
        wt += (int64_t)L.cin_dg * 9 * L.cout_pad;
        bo += L.cout_pad;
        const int mb = mb_of(L.cout_pad), nbk = L.cin_dg % 64 == 0 ? 2 : 1;
        const int pairs = (L.cout_pad / (32 * mb)) * (L.cin_dg / (32 * nbk));
        const int64_t nwb = (int64_t)cout[k] * 9 * cin[k] + cout[k];
        for (int b = 1; b <= p.B; ++b) {
            Plan q = p;
            q.B = b;
            int splits, chunk;
            if (wgrad9_ok(q, level_in[k]))
                wgrad9_split(pixels(q, level_in[k]) / kWgTile, pairs, mb, nbk, nwb, splits, chunk);
            else
                wgrad_split(q, level_in[k], pairs * 9, splits, chunk);
            p.wpart_max = std::max<int64_t>(p.wpart_max, (int64_t)splits * nwb);
        }
    }
    // channel means of the bottleneck and their adjoint (per sample, c3 wide)
    // column sums over c3 channels of at most the level-2 nodes of a sample
    p.bpart_max = std::max<int64_t>(
        p.bpart_max, (int64_t)p.B * ((pixels(p, 2) / p.B + col_rows(c3) - 1) / col_rows(c3)) * c3);
    p.n_params = off;
    p.wf_total = wf;
    p.wt_total = wt;
    p.b_total = bo;
    size_t o = 0;
    auto take = [&](size_t& dst, size_t bytes) {
        dst = o;
        o = al256(o + std::max<size_t>(bytes, 4));
    };
    take(p.o_master, 4 * (size_t)off);
    take(p.o_grad, 4 * (size_t)off);
    take(p.o_m, 4 * (size_t)off);
    take(p.o_v, 4 * (size_t)off);
    take(p.o_wf, (size_t)p.es * wf);
    take(p.o_wt, (size_t)p.es * wt);
    take(p.o_bias, 4 * (size_t)bo);
    // level -1: one value per sample (the bottleneck's channel means)
    for (int k = 0; k < NBUF; ++k)
        take(p.off[k], (size_t)p.es * (p.shape[k].level < 0 ? (int64_t)p.B : pixels(p, p.shape[k].level)) *
                           p.shape[k].ch);
    take(p.o_gmean, 4 * (size_t)p.B * c3);
    const int64_t P0 = pixels(p, 0);
    take(p.o_out, 12 * (size_t)P0);
    take(p.o_tgt, 12 * (size_t)P0);
    take(p.o_fluid, (size_t)P0);
    take(p.o_wpart, 4 * (size_t)p.wpart_max);
    take(p.o_bpart, 4 * (size_t)p.bpart_max);
    take(p.o_lpart, 16 * (size_t)((P0 + kEw - 1) / kEw));
    take(p.o_loss, 16);
    take(p.o_idx, 4 * (size_t)p.B);
    p.total = o;
    return nullptr;
}

}  // namespace

struct lbm_nn {
    Plan p;
    int dtype;
    double rho_scale;
    hipStream_t st;
    char* ws;
    int batch = 0;       // batch of the last forward
    int64_t adam_t = 0;  // Adam steps taken
    char err[512];
};

namespace {

template <typename T = void>
T* at(lbm_nn* n, size_t off) {
    return reinterpret_cast<T*>(n->ws + off);
}

lbm_status nn_fail(lbm_nn* n, hipError_t e, const char* what) {
    nn_set_err(n ? n->err : g_nn_err, "%s: %s", what, hipGetErrorString(e));
    return LBM_EDEVICE;
}

#define NNCHK(n, call)                                     \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return nn_fail(n, e_, #call); \
    } while (0)

unsigned blocks(int64_t n, int per = kEw) { return (unsigned)((n + per - 1) / per); }

void* buf(lbm_nn* n, Buf b) { return n->ws + n->p.off[b]; }

// One convolution: input tensor (ptr, channel stride, channels read), layer
// weights (forward or input-gradient form), output (ptr, stride, offset,
// channels), optional ReLU and ReLU mask.
template <typename T, typename OT>
void conv(lbm_nn* n, int level, const void* in, int in_cs, int cin, const void* w, const float* bias, void* out,
          int out_cs, int out_co, int cout, int cout_pad, bool relu, const void* mask, int mask_cs, int mask_co) {
    const Plan& p = n->p;
    ConvArgs a;
    a.in = in;
    a.in_cs = in_cs;
    a.cin = cin;
    a.w = w;
    a.bias = bias;
    a.out = out;
    a.out_cs = out_cs;
    a.out_co = out_co;
    a.cout = cout;
    a.mask = mask;
    a.mask_cs = mask_cs;
    a.mask_co = mask_co;
    a.relu = relu ? 1 : 0;
    a.H = p.H >> level;
    a.W = p.W >> level;
    a.P = (int)((int64_t)n->batch * a.H * a.W);
    a.out_f32 = sizeof(OT) == 4 ? 1 : 0;
    if (sizeof(T) == 2 && cin % 32 == 0 && a.H % kC9Rows == 0 && a.W % 32 == 0) {
        // BF16 with the input tile held across the nine taps, when the
        // launch still gives >= 256 workgroups
        // (with <= 640 workgroups and several chunks the next chunk is
        // prefetched into registers: fewer waves, but its loads overlap)
        const int64_t tiles = (int64_t)n->batch * (a.H / kC9Rows) * (a.W / 32);
        const bool deep = cin >= 128;
        if (cout_pad % 64 == 0 && tiles * (cout_pad / 64) >= 512) {
            const dim3 g((unsigned)tiles, cout_pad / 64);
            if (deep && tiles * (cout_pad / 64) <= 640)
                k_conv9<2, true><<<g, 256, 0, n->st>>>(a);
            else
                k_conv9<2, false><<<g, 256, 0, n->st>>>(a);
            return;
        }
        if (tiles * (cout_pad / 32) >= 256) {
            const dim3 g((unsigned)tiles, cout_pad / 32);
            if (deep && tiles * (cout_pad / 32) <= 640)
                k_conv9<1, true><<<g, 256, 0, n->st>>>(a);
            else
                k_conv9<1, false><<<g, 256, 0, n->st>>>(a);
            return;
        }
    }
    if (sizeof(T) == 2) {
        // BF16: LDS-staged tiles (BM x BN).  The widest tile that divides the
        // output channels and still gives >= 512 workgroups (two per CU),
        // otherwise the tile with the most workgroups.
        struct Shape { int bm, bn; };
        const Shape shapes[5] = {{128, 128}, {128, 64}, {256, 32}, {64, 64}, {128, 32}};
        int pick = -1, most = -1;
        int64_t most_wg = -1;
        for (int k = 0; k < 5; ++k) {
            if (cout_pad % shapes[k].bn) continue;
            const int64_t wg = (int64_t)blocks(a.P, shapes[k].bm) * (cout_pad / shapes[k].bn);
            if (pick < 0 && wg >= 512) pick = k;
            if (wg > most_wg) { most_wg = wg; most = k; }
        }
        if (pick < 0) pick = most;
        const bool bk32 = cin % 32 == 0;
        dim3 g(blocks(a.P, shapes[pick].bm), cout_pad / shapes[pick].bn);
#define CONV_LDS_LAUNCH(MW, NW, WM, WN)                                                   \
    if (bk32) k_conv_lds<MW, NW, WM, WN, 32><<<g, 256, 0, n->st>>>(a);                    \
    else k_conv_lds<MW, NW, WM, WN, 16><<<g, 256, 0, n->st>>>(a);
        switch (pick) {
            case 0: CONV_LDS_LAUNCH(2, 2, 2, 2) break;
            case 1: CONV_LDS_LAUNCH(2, 2, 2, 1) break;
            case 2: CONV_LDS_LAUNCH(4, 1, 2, 1) break;
            case 3: CONV_LDS_LAUNCH(2, 2, 1, 1) break;
            default: CONV_LDS_LAUNCH(4, 1, 1, 1) break;
        }
#undef CONV_LDS_LAUNCH
        return;
    }
    if (cout_pad % 64 == 0) {
        dim3 g(blocks(a.P, 32 * 2 * kConvWaves), cout_pad / 64);
        k_conv<T, OT, 2, 2><<<g, kConvWaves * 64, 0, n->st>>>(a);
    } else {
        dim3 g(blocks(a.P, 32 * 4 * kConvWaves), cout_pad / 32);
        k_conv<T, OT, 4, 1><<<g, kConvWaves * 64, 0, n->st>>>(a);
    }
}

// out[b][c] = scale * sum over the N nodes of segment b of a[.][co + c]
// (c < C <= kEw), in a fixed order; float (fout) and/or T (tout) results.
template <typename T>
void colsum(lbm_nn* n, const void* a, int cs, int co, int C, int64_t N, int B, float scale, float* fout, T* tout) {
    const int R = col_rows(C);
    const int nblk = (int)((N + R - 1) / R);
    float* part = at<float>(n, n->p.o_bpart);
    k_colsum_partial<T><<<dim3(nblk, B), kEw, 0, n->st>>>((const T*)a, cs, co, C, N, R, part);
    k_colsum_final<T><<<blocks((int64_t)B * C, kSumCols), kEw, 0, n->st>>>(part, nblk, C, B, scale, fout, tout);
}

template <typename T>
void layer_fwd(lbm_nn* n, int k, int level, Buf in, Buf out, int out_cs, int out_co) {
    const LayerDev& L = n->p.L[k];
    conv<T, T>(n, level, buf(n, in), n->p.shape[in].ch, L.cin_pad, at<T>(n, n->p.o_wf) + L.wf_off,
               at<float>(n, n->p.o_bias) + L.b_off, buf(n, out), out_cs, out_co, L.cout, L.cout_pad, true, nullptr, 0,
               0);
}

// Input gradient of layer k: g_in = conv(g_pre, flipped weights), times the
// ReLU mask of `act` (the layer's forward input) when given.
template <typename T>
void layer_dgrad(lbm_nn* n, int k, int level, Buf g_pre, Buf g_in, Buf act, int act_cs, int act_co, bool use_mask) {
    const LayerDev& L = n->p.L[k];
    conv<T, T>(n, level, buf(n, g_pre), n->p.shape[g_pre].ch, L.cout_pad, at<T>(n, n->p.o_wt) + L.wt_off, nullptr,
               buf(n, g_in), n->p.shape[g_in].ch, 0, L.cin, L.cin_dg, false, use_mask ? buf(n, act) : nullptr, act_cs,
               act_co);
}

// Weight and bias gradient of layer k from its forward input x (at `level`,
// channel stride x_cs) and its pre-activation gradient g (stride g_cs), for
// the batch of the last forward; the sum goes to out[cout * 9 * cin + cout].
template <typename T>
void layer_wgrad_ptr(lbm_nn* n, int k, int level, const void* xp, int x_cs, const void* gp, int g_cs, float* out) {
    const Plan& p = n->p;
    const LayerDev& L = p.L[k];
    const int64_t nwb = (int64_t)L.cout * 9 * L.cin + L.cout;  // weights and bias, contiguous
    Plan q = p;
    q.B = n->batch;
    if (wgrad9_ok(q, level)) {
        Wgrad9Args a;
        a.g = static_cast<const __bf16*>(gp);
        a.g_cs = g_cs;
        a.x = static_cast<const __bf16*>(xp);
        a.x_cs = x_cs;
        a.cout = L.cout;
        a.cin = L.cin;
        a.H = p.H >> level;
        a.W = p.W >> level;
        const int mb = mb_of(L.cout_pad), nbk = L.cin_dg % 64 == 0 ? 2 : 1;
        const int co_blocks = L.cout_pad / (32 * mb);
        a.ci_blocks = L.cin_dg / (32 * nbk);
        a.ntiles = (int)(pixels(q, level) / kWgTile);
        int splits;
        wgrad9_split(a.ntiles, co_blocks * a.ci_blocks, mb, nbk, nwb, splits, a.tps);
        a.part = at<float>(n, p.o_wpart);
        const dim3 gr(co_blocks * a.ci_blocks, splits);
        if (mb == 2 && nbk == 2)
            k_wgrad9<2, 2><<<gr, 192 * 2, 0, n->st>>>(a);
        else if (mb == 2)
            k_wgrad9<2, 1><<<gr, 192, 0, n->st>>>(a);
        else if (nbk == 2)
            k_wgrad9<1, 2><<<gr, 192 * 2, 0, n->st>>>(a);
        else
            k_wgrad9<1, 1><<<gr, 192, 0, n->st>>>(a);
        k_sum_splits<<<blocks(nwb, kSumCols), kEw, 0, n->st>>>(a.part, splits, nwb, out);
        return;
    }
    WgradArgs a;
    a.g = gp;
    a.g_cs = g_cs;
    a.x = xp;
    a.x_cs = x_cs;
    a.cout = L.cout;
    a.cin = L.cin;
    a.H = p.H >> level;
    a.W = p.W >> level;
    a.P = (int)((int64_t)n->batch * a.H * a.W);
    const int mb = mb_of(L.cout_pad), nbk = L.cin_dg % 64 == 0 ? 2 : 1;
    a.co_blocks = L.cout_pad / (32 * mb);
    a.ci_blocks = L.cin_dg / (32 * nbk);
    const int tiles = a.co_blocks * a.ci_blocks * 9;
    int splits, chunk;
    wgrad_split(q, level, tiles, splits, chunk);
    a.chunk_per_split = chunk;
    a.part = at<float>(n, p.o_wpart);
    dim3 gr(tiles, splits);
    if (mb == 2 && nbk == 2)
        k_wgrad<T, 2, 2><<<gr, 256, 0, n->st>>>(a);
    else if (mb == 2)
        k_wgrad<T, 2, 1><<<gr, 256, 0, n->st>>>(a);
    else if (nbk == 2)
        k_wgrad<T, 1, 2><<<gr, 256, 0, n->st>>>(a);
    else
        k_wgrad<T, 1, 1><<<gr, 256, 0, n->st>>>(a);
    k_sum_splits<<<blocks(nwb, kSumCols), kEw, 0, n->st>>>(a.part, splits, nwb, out);
}

template <typename T>
void layer_wgrad(lbm_nn* n, int k, int level, Buf x, Buf g) {
    const Plan& p = n->p;
    layer_wgrad_ptr<T>(n, k, level, buf(n, x), p.shape[x].ch, buf(n, g), p.shape[g].ch,
                       at<float>(n, p.o_grad) + p.L[k].off);
}

template <typename T>
void forward_t(lbm_nn* n) {
    const Plan& p = n->p;
    const int c0 = p.c[0], c1 = p.c[1], c2 = p.c[2], c3 = p.c[3];
    const int B = n->batch;
    auto H = [&](int l) { return p.H >> l; };
    auto W = [&](int l) { return p.W >> l; };
    // encoder
    layer_fwd<T>(n, 0, 0, X0, A0, c0, 0);
    layer_fwd<T>(n, 1, 0, A0, CAT0, c1 + c0, c1);
    k_pool<T><<<blocks(((int64_t)B * H(1) * W(1) * c0) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, CAT0), c1 + c0, c1, c0, (T*)buf(n, X1), H(1), W(1), B);
    layer_fwd<T>(n, 2, 1, X1, A1, c1, 0);
    layer_fwd<T>(n, 3, 1, A1, CAT1, c2 + c1, c2);
    k_pool<T><<<blocks(((int64_t)B * H(2) * W(2) * c1) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, CAT1), c2 + c1, c2, c1, (T*)buf(n, X2), H(2), W(2), B);
    const int cat2 = 2 * c3 + c2;  // [up(b2), skip_2, mean(b2)]
    layer_fwd<T>(n, 4, 2, X2, A2, c2, 0);
    layer_fwd<T>(n, 5, 2, A2, CAT2, cat2, c3);
    k_pool<T><<<blocks(((int64_t)B * H(3) * W(3) * c2) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, CAT2), cat2, c3, c2, (T*)buf(n, X3), H(3), W(3), B);
    // bottleneck and its global context
    layer_fwd<T>(n, 6, 3, X3, B1, c3, 0);
    layer_fwd<T>(n, 7, 3, B1, B2, c3, 0);
    colsum<T>(n, buf(n, B2), c3, 0, c3, (int64_t)H(3) * W(3), B, 1.0f / (float)(H(3) * W(3)), nullptr,
              (T*)buf(n, GMEAN));
    k_broadcast<T><<<blocks(((int64_t)B * H(2) * W(2) * c3) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, GMEAN), c3, (T*)buf(n, CAT2), cat2, c3 + c2, H(2) * W(2), B);
    // decoder
    k_upsample<T><<<blocks(((int64_t)B * H(2) * W(2) * c3) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, B2), c3, (T*)buf(n, CAT2), cat2, 0, H(2), W(2), B);
    layer_fwd<T>(n, 8, 2, CAT2, D2A, c2, 0);
    layer_fwd<T>(n, 9, 2, D2A, D2B, c2, 0);
    k_upsample<T><<<blocks(((int64_t)B * H(1) * W(1) * c2) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, D2B), c2, (T*)buf(n, CAT1), c2 + c1, 0, H(1), W(1), B);
    layer_fwd<T>(n, 10, 1, CAT1, D1A, c1, 0);
    layer_fwd<T>(n, 11, 1, D1A, D1B, c1, 0);
    k_upsample<T><<<blocks(((int64_t)B * H(0) * W(0) * c1) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, D1B), c1, (T*)buf(n, CAT0), c1 + c0, 0, H(0), W(0), B);
    layer_fwd<T>(n, 12, 0, CAT0, D0A, c0, 0);
    layer_fwd<T>(n, 13, 0, D0A, D0B, c0, 0);
    // head: no activation, FP32 output [P][3]
    const LayerDev& L = p.L[14];
    conv<T, float>(n, 0, buf(n, D0B), c0, L.cin_pad, at<T>(n, p.o_wf) + L.wf_off, at<float>(n, p.o_bias) + L.b_off,
                   at<float>(n, p.o_out), 3, 0, 3, L.cout_pad, false, nullptr, 0, 0);
}

// Backward from the padded head gradient G_HEAD: every parameter gradient.
template <typename T>
void backward_t(lbm_nn* n) {
    const Plan& p = n->p;
    const int c0 = p.c[0], c1 = p.c[1], c2 = p.c[2], c3 = p.c[3];
    const int B = n->batch;
    auto H = [&](int l) { return p.H >> l; };
    auto W = [&](int l) { return p.W >> l; };
    // head and decoder level 0
    layer_wgrad<T>(n, 14, 0, D0B, G_HEAD);
    layer_dgrad<T>(n, 14, 0, G_HEAD, G_D0B, D0B, c0, 0, true);
    layer_wgrad<T>(n, 13, 0, D0A, G_D0B);
    layer_dgrad<T>(n, 13, 0, G_D0B, G_D0A, D0A, c0, 0, true);
    layer_wgrad<T>(n, 12, 0, CAT0, G_D0A);
    layer_dgrad<T>(n, 12, 0, G_D0A, G_CAT0, CAT0, 0, 0, false);
    k_upsample_back<T><<<blocks(((int64_t)B * H(1) * W(1) * c1) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, G_CAT0), c1 + c0, 0, c1, (const T*)buf(n, D1B), nullptr, (T*)buf(n, G_D1B), H(1), W(1), B);
    // decoder level 1
    layer_wgrad<T>(n, 11, 1, D1A, G_D1B);
    layer_dgrad<T>(n, 11, 1, G_D1B, G_D1A, D1A, c1, 0, true);
    layer_wgrad<T>(n, 10, 1, CAT1, G_D1A);
    layer_dgrad<T>(n, 10, 1, G_D1A, G_CAT1, CAT1, 0, 0, false);
    k_upsample_back<T><<<blocks(((int64_t)B * H(2) * W(2) * c2) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, G_CAT1), c2 + c1, 0, c2, (const T*)buf(n, D2B), nullptr, (T*)buf(n, G_D2B), H(2), W(2), B);
    // decoder level 2
    layer_wgrad<T>(n, 9, 2, D2A, G_D2B);
    layer_dgrad<T>(n, 9, 2, G_D2B, G_D2A, D2A, c2, 0, true);
    layer_wgrad<T>(n, 8, 2, CAT2, G_D2A);
    layer_dgrad<T>(n, 8, 2, G_D2A, G_CAT2, CAT2, 0, 0, false);
    const int cat2 = 2 * c3 + c2;
    colsum<T>(n, buf(n, G_CAT2), cat2, c3 + c2, c3, (int64_t)H(2) * W(2), B, 1.0f, at<float>(n, p.o_gmean),
              (T*)nullptr);
    k_upsample_back<T><<<blocks(((int64_t)B * H(3) * W(3) * c3) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, G_CAT2), cat2, 0, c3, (const T*)buf(n, B2), at<float>(n, p.o_gmean), (T*)buf(n, G_B2),
        H(3), W(3), B);
    // bottleneck
    layer_wgrad<T>(n, 7, 3, B1, G_B2);
    layer_dgrad<T>(n, 7, 3, G_B2, G_B1, B1, c3, 0, true);
    layer_wgrad<T>(n, 6, 3, X3, G_B1);
    layer_dgrad<T>(n, 6, 3, G_B1, G_X3, X3, 0, 0, false);
    // encoder level 2
    k_pool_back_skip<T><<<blocks(((int64_t)B * H(2) * W(2) * c2) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, G_X3), (const T*)buf(n, G_CAT2), cat2, c3, (const T*)buf(n, CAT2), c2, (T*)buf(n, G_S2),
        H(2), W(2), B);
    layer_wgrad<T>(n, 5, 2, A2, G_S2);
    layer_dgrad<T>(n, 5, 2, G_S2, G_A2, A2, c2, 0, true);
    layer_wgrad<T>(n, 4, 2, X2, G_A2);
    layer_dgrad<T>(n, 4, 2, G_A2, G_X2, X2, 0, 0, false);
    // encoder level 1
    k_pool_back_skip<T><<<blocks(((int64_t)B * H(1) * W(1) * c1) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, G_X2), (const T*)buf(n, G_CAT1), c2 + c1, c2, (const T*)buf(n, CAT1), c1, (T*)buf(n, G_S1),
        H(1), W(1), B);
    layer_wgrad<T>(n, 3, 1, A1, G_S1);
    layer_dgrad<T>(n, 3, 1, G_S1, G_A1, A1, c1, 0, true);
    layer_wgrad<T>(n, 2, 1, X1, G_A1);
    layer_dgrad<T>(n, 2, 1, G_A1, G_X1, X1, 0, 0, false);
    // encoder level 0
    k_pool_back_skip<T><<<blocks(((int64_t)B * H(0) * W(0) * c0) / 8), kEw, 0, n->st>>>(
        (const T*)buf(n, G_X1), (const T*)buf(n, G_CAT0), c1 + c0, c1, (const T*)buf(n, CAT0), c0, (T*)buf(n, G_S0),
        H(0), W(0), B);
    layer_wgrad<T>(n, 1, 0, A0, G_S0);
    layer_dgrad<T>(n, 1, 0, G_S0, G_A0, A0, c0, 0, true);
    layer_wgrad<T>(n, 0, 0, X0, G_A0);
}

template <typename T>
void pack_weights_t(lbm_nn* n) {
    const Plan& p = n->p;
    for (int k = 0; k < kLayers; ++k) {
        const LayerDev& L = p.L[k];
        const int64_t m = std::max<int64_t>(std::max<int64_t>((int64_t)L.cout_pad * 9 * L.cin_pad,
                                                             (int64_t)L.cin_dg * 9 * L.cout_pad),
                                            L.cout_pad);
        k_pack_weights<T><<<blocks(m), kEw, 0, n->st>>>(at<float>(n, p.o_master), L, at<T>(n, p.o_wf),
                                                       at<T>(n, p.o_wt), at<float>(n, p.o_bias));
    }
}

void pack_weights(lbm_nn* n) {
    if (n->dtype == LBM_BF16)
        pack_weights_t<__bf16>(n);
    else
        pack_weights_t<float>(n);
}

void forward(lbm_nn* n) {
    if (n->dtype == LBM_BF16)
        forward_t<__bf16>(n);
    else
        forward_t<float>(n);
}

void backward(lbm_nn* n) {
    if (n->dtype == LBM_BF16)
        backward_t<__bf16>(n);
    else
        backward_t<float>(n);
}

void adam(lbm_nn* n, double lr, double b1, double b2, double eps) {
    n->adam_t += 1;
    const double c1 = 1.0 - std::pow(b1, (double)n->adam_t);
    const double c2 = 1.0 - std::pow(b2, (double)n->adam_t);
    const Plan& p = n->p;
    k_adam<<<blocks(p.n_params), kEw, 0, n->st>>>(at<float>(n, p.o_master), at<float>(n, p.o_grad),
                                                   at<float>(n, p.o_m), at<float>(n, p.o_v), p.n_params, (float)lr,
                                                   (float)b1, (float)b2, (float)eps, (float)c1, (float)c2);
    pack_weights(n);
}

// Loss of the output against the packed target; writes the head gradient.
template <typename T>
void loss_t(lbm_nn* n) {
    const Plan& p = n->p;
    const int64_t P = (int64_t)n->batch * p.H * p.W;
    const int nb = (int)blocks(P);
    k_loss_partial<<<nb, kEw, 0, n->st>>>(at<float>(n, p.o_out), at<float>(n, p.o_tgt), at<uint8_t>(n, p.o_fluid), P,
                                          at<double>(n, p.o_lpart));
    k_loss_final<<<1, kEw, 0, n->st>>>(at<double>(n, p.o_lpart), nb, at<double>(n, p.o_loss));
    k_loss_grad<T><<<nb, kEw, 0, n->st>>>(at<float>(n, p.o_out), at<float>(n, p.o_tgt), at<uint8_t>(n, p.o_fluid), P,
                                         at<double>(n, p.o_loss), (T*)buf(n, G_HEAD));
}

template <typename T>
void pack_sample_t(lbm_nn* n, const uint8_t* solid, const float* rho, const float* ux, const float* uy,
                   const double* re, const double* gx, const double* tau, const int* idx, const int* aug) {
    const Plan& p = n->p;
    const int64_t P = (int64_t)n->batch * p.H * p.W;
    k_pack_input<T><<<blocks(P), kEw, 0, n->st>>>(solid, re, idx, aug, p.H, p.W, n->batch, (T*)buf(n, X0));
    if (rho)
        k_pack_target<<<blocks(P), kEw, 0, n->st>>>(solid, rho, ux, uy, gx, tau, idx, aug, p.H, p.W, n->batch,
                                                    n->rho_scale, at<float>(n, p.o_tgt), at<uint8_t>(n, p.o_fluid));
}

lbm_status sync_check(lbm_nn* n) {
    NNCHK(n, hipGetLastError());
    return LBM_OK;
}

lbm_status check_batch(lbm_nn* n, int batch) {
    if (batch < 1 || batch > n->p.B) {
        nn_set_err(n->err, "batch must be in [1, %d]", n->p.B);
        return LBM_EINVAL;
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_nn_workspace_bytes(const lbm_nn_config* cfg, size_t* bytes) {
    if (!cfg || !bytes) {
        nn_set_err(g_nn_err, "cfg and bytes must not be NULL");
        return LBM_EINVAL;
    }
    Plan p;
    const char* why = make_plan(*cfg, p);
    if (why) {
        nn_set_err(g_nn_err, "%s", why);
        return LBM_EINVAL;
    }
    *bytes = p.total;
    return LBM_OK;
}

lbm_status lbm_nn_create(const lbm_nn_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
                         lbm_nn** out) {
    if (!cfg || !out) {
        nn_set_err(g_nn_err, "cfg and out must not be NULL");
        return LBM_EINVAL;
    }
    *out = nullptr;
    Plan p;
    const char* why = make_plan(*cfg, p);
    if (why) {
        nn_set_err(g_nn_err, "%s", why);
        return LBM_EINVAL;
    }
    if (!d_workspace || ((uintptr_t)d_workspace & 255) != 0) {
        nn_set_err(g_nn_err, "workspace must be a non-NULL 256-byte aligned device pointer");
        return LBM_EINVAL;
    }
    if (bytes < p.total) {
        nn_set_err(g_nn_err, "workspace too small: %zu < %zu bytes", bytes, p.total);
        return LBM_ESIZE;
    }
    lbm_nn* n = new (std::nothrow) lbm_nn();
    if (!n) return LBM_EINVAL;
    n->p = p;
    n->dtype = cfg->dtype;
    n->rho_scale = cfg->rho_scale;
    n->st = (hipStream_t)hip_stream;
    n->ws = (char*)d_workspace;
    n->err[0] = 0;
    // parameters, gradients and Adam moments start at zero
    for (size_t o : {p.o_master, p.o_grad, p.o_m, p.o_v})
        k_zero_f32<<<blocks(p.n_params), kEw, 0, n->st>>>(at<float>(n, o), p.n_params);
    pack_weights(n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        nn_set_err(g_nn_err, "initialisation failed: %s", hipGetErrorString(e));
        delete n;
        return LBM_EDEVICE;
    }
    *out = n;
    return LBM_OK;
}

int64_t lbm_nn_param_count(const lbm_nn* n) { return n ? n->p.n_params : -1; }

lbm_status lbm_nn_set_params(lbm_nn* n, const float* d_params) {
    if (!n || !d_params) return LBM_EINVAL;
    const Plan& p = n->p;
    NNCHK(n, hipMemcpyAsync(at<float>(n, p.o_master), d_params, 4 * (size_t)p.n_params, hipMemcpyDeviceToDevice, n->st));
    for (size_t o : {p.o_m, p.o_v}) k_zero_f32<<<blocks(p.n_params), kEw, 0, n->st>>>(at<float>(n, o), p.n_params);
    n->adam_t = 0;
    pack_weights(n);
    return sync_check(n);
}

lbm_status lbm_nn_get_params(lbm_nn* n, float* d_out) {
    if (!n || !d_out) return LBM_EINVAL;
    NNCHK(n, hipMemcpyAsync(d_out, at<float>(n, n->p.o_master), 4 * (size_t)n->p.n_params, hipMemcpyDeviceToDevice,
                            n->st));
    return LBM_OK;
}

lbm_status lbm_nn_get_grads(lbm_nn* n, float* d_out) {
    if (!n || !d_out) return LBM_EINVAL;
    NNCHK(n, hipMemcpyAsync(d_out, at<float>(n, n->p.o_grad), 4 * (size_t)n->p.n_params, hipMemcpyDeviceToDevice,
                            n->st));
    return LBM_OK;
}

lbm_status lbm_nn_forward(lbm_nn* n, const float* d_x, int32_t batch, float* d_y) {
    if (!n || !d_x || !d_y) return LBM_EINVAL;
    lbm_status rs = check_batch(n, batch);
    if (rs != LBM_OK) return rs;
    n->batch = batch;
    const int64_t P = (int64_t)batch * n->p.H * n->p.W;
    if (n->dtype == LBM_BF16)
        k_pack_raw<__bf16><<<blocks(P), kEw, 0, n->st>>>(d_x, P, (__bf16*)buf(n, X0));
    else
        k_pack_raw<float><<<blocks(P), kEw, 0, n->st>>>(d_x, P, (float*)buf(n, X0));
    forward(n);
    NNCHK(n, hipMemcpyAsync(d_y, at<float>(n, n->p.o_out), 12 * (size_t)P, hipMemcpyDeviceToDevice, n->st));
    return sync_check(n);
}

lbm_status lbm_nn_backward(lbm_nn* n, const float* d_gy) {
    if (!n || !d_gy) return LBM_EINVAL;
    if (n->batch < 1) {
        nn_set_err(n->err, "backward needs a forward first");
        return LBM_ESTATE;
    }
    const int64_t P = (int64_t)n->batch * n->p.H * n->p.W;
    if (n->dtype == LBM_BF16)
        k_pack_head_grad<__bf16><<<blocks(P), kEw, 0, n->st>>>(d_gy, P, (__bf16*)buf(n, G_HEAD));
    else
        k_pack_head_grad<float><<<blocks(P), kEw, 0, n->st>>>(d_gy, P, (float*)buf(n, G_HEAD));
    backward(n);
    return sync_check(n);
}

lbm_status lbm_nn_layer_forward(lbm_nn* n, int32_t layer, int32_t batch, const void* d_x, int32_t x_cs,
                                void* d_y, int32_t y_cs) {
    if (!n || !d_x || !d_y) return LBM_EINVAL;
    if (layer < 1 || layer > kLayers - 2) {
        nn_set_err(n->err, "layer must be in [1, %d]", kLayers - 2);
        return LBM_EINVAL;
    }
    lbm_status rs = check_batch(n, batch);
    if (rs != LBM_OK) return rs;
    const LayerDev& L = n->p.L[layer];
    if (x_cs < L.cin || x_cs % 8 != 0 || y_cs < L.cout || y_cs % 8 != 0 ||
        ((uintptr_t)d_x | (uintptr_t)d_y) % 16 != 0) {
        nn_set_err(n->err, "layer %d needs x_cs >= %d and y_cs >= %d, multiples of 8, 16-byte aligned tensors",
                   layer, L.cin, L.cout);
        return LBM_EINVAL;
    }
    const int last = n->batch;
    n->batch = batch;
    pack_weights(n);
    const int lv = n->p.level[layer];
    if (n->dtype == LBM_BF16)
        conv<__bf16, __bf16>(n, lv, d_x, x_cs, L.cin_pad, at<__bf16>(n, n->p.o_wf) + L.wf_off,
                             at<float>(n, n->p.o_bias) + L.b_off, d_y, y_cs, 0, L.cout, L.cout_pad, true, nullptr,
                             0, 0);
    else
        conv<float, float>(n, lv, d_x, x_cs, L.cin_pad, at<float>(n, n->p.o_wf) + L.wf_off,
                           at<float>(n, n->p.o_bias) + L.b_off, d_y, y_cs, 0, L.cout, L.cout_pad, true, nullptr, 0,
                           0);
    n->batch = last;
    return sync_check(n);
}

lbm_status lbm_nn_layer_wgrad(lbm_nn* n, int32_t layer, int32_t batch, const void* d_x, int32_t x_cs,
                              const void* d_g, int32_t g_cs, float* d_grad) {
    if (!n || !d_x || !d_g || !d_grad) return LBM_EINVAL;
    if (layer < 0 || layer >= kLayers) {
        nn_set_err(n->err, "layer must be in [0, %d)", kLayers);
        return LBM_EINVAL;
    }
    lbm_status rs = check_batch(n, batch);
    if (rs != LBM_OK) return rs;
    const LayerDev& L = n->p.L[layer];
    const int xmin = layer == 0 ? 16 : L.cin;
    if (x_cs < xmin || x_cs % 8 != 0 || g_cs < L.cout_pad || g_cs % 8 != 0 ||
        ((uintptr_t)d_x | (uintptr_t)d_g) % 16 != 0) {
        nn_set_err(n->err, "layer %d needs x_cs >= %d and g_cs >= %d, multiples of 8, 16-byte aligned tensors", layer,
                   xmin, L.cout_pad);
        return LBM_EINVAL;
    }
    const int last = n->batch;  // the batch of the last forward stays that of the network
    n->batch = batch;
    if (n->dtype == LBM_BF16)
        layer_wgrad_ptr<__bf16>(n, layer, n->p.level[layer], d_x, x_cs, d_g, g_cs, d_grad);
    else
        layer_wgrad_ptr<float>(n, layer, n->p.level[layer], d_x, x_cs, d_g, g_cs, d_grad);
    n->batch = last;
    return sync_check(n);
}

lbm_status lbm_nn_adam(lbm_nn* n, double lr, double beta1, double beta2, double eps) {
    if (!n || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0)) {
        if (n) nn_set_err(n->err, "Adam needs lr > 0, 0 <= beta < 1, eps > 0");
        return LBM_EINVAL;
    }
    adam(n, lr, beta1, beta2, eps);
    return sync_check(n);
}

static lbm_status train_or_eval(lbm_nn* n, const uint8_t* solid, const float* rho, const float* ux, const float* uy,
                                const double* re, const double* gx, const double* tau, const int32_t* idx,
                                const int32_t* aug, int32_t batch, double lr, double* loss, bool train) {
    if (!n || !solid || !rho || !ux || !uy || !re || !gx || !tau) return LBM_EINVAL;
    lbm_status rs = check_batch(n, batch);
    if (rs != LBM_OK) return rs;
    if (train && !(lr > 0.0)) {
        nn_set_err(n->err, "lr must be > 0");
        return LBM_EINVAL;
    }
    n->batch = batch;
    if (n->dtype == LBM_BF16) {
        pack_sample_t<__bf16>(n, solid, rho, ux, uy, re, gx, tau, idx, aug);
        forward_t<__bf16>(n);
        loss_t<__bf16>(n);
        if (train) backward_t<__bf16>(n);
    } else {
        pack_sample_t<float>(n, solid, rho, ux, uy, re, gx, tau, idx, aug);
        forward_t<float>(n);
        loss_t<float>(n);
        if (train) backward_t<float>(n);
    }
    if (train) adam(n, lr, 0.9, 0.999, 1e-8);
    rs = sync_check(n);
    if (rs != LBM_OK) return rs;
    if (loss) {
        double v[2];
        NNCHK(n, hipMemcpyAsync(v, at<double>(n, n->p.o_loss), 16, hipMemcpyDeviceToHost, n->st));
        NNCHK(n, hipStreamSynchronize(n->st));
        *loss = v[0];
    }
    return LBM_OK;
}

lbm_status lbm_nn_train_step(lbm_nn* n, const uint8_t* d_solid, const float* d_rho, const float* d_ux,
                             const float* d_uy, const double* d_re, const double* d_gx, const double* d_tau,
                             const int32_t* d_idx, const int32_t* d_aug, int32_t batch, double lr, double* loss) {
    return train_or_eval(n, d_solid, d_rho, d_ux, d_uy, d_re, d_gx, d_tau, d_idx, d_aug, batch, lr, loss, true);
}

lbm_status lbm_nn_eval(lbm_nn* n, const uint8_t* d_solid, const float* d_rho, const float* d_ux, const float* d_uy,
                       const double* d_re, const double* d_gx, const double* d_tau, const int32_t* d_idx,
                       int32_t batch, double* loss) {
    return train_or_eval(n, d_solid, d_rho, d_ux, d_uy, d_re, d_gx, d_tau, d_idx, nullptr, batch, 0.0, loss, false);
}

lbm_status lbm_nn_infer(lbm_nn* n, const uint8_t* d_solid, const double* d_re, const double* d_gx,
                        const double* d_tau, int32_t batch, float* d_rho, float* d_ux, float* d_uy) {
    if (!n || !d_solid || !d_re || !d_gx || !d_tau || !d_rho || !d_ux || !d_uy) return LBM_EINVAL;
    lbm_status rs = check_batch(n, batch);
    if (rs != LBM_OK) return rs;
    n->batch = batch;
    const Plan& p = n->p;
    const int64_t P = (int64_t)batch * p.H * p.W;
    if (n->dtype == LBM_BF16) {
        pack_sample_t<__bf16>(n, d_solid, nullptr, nullptr, nullptr, d_re, d_gx, d_tau, nullptr, nullptr);
        forward_t<__bf16>(n);
    } else {
        pack_sample_t<float>(n, d_solid, nullptr, nullptr, nullptr, d_re, d_gx, d_tau, nullptr, nullptr);
        forward_t<float>(n);
    }
    k_unpack_fields<<<blocks(P), kEw, 0, n->st>>>(at<float>(n, p.o_out), d_solid, d_gx, d_tau, p.H, p.W, batch,
                                                  n->rho_scale, d_rho, d_ux, d_uy);
    return sync_check(n);
}

lbm_status lbm_warm_project(int32_t nx, int32_t ny, int32_t n_fields, const uint8_t* d_owner, float* d_rho,
                            float* d_ux, float* d_uy, const float* d_rho2, const float* d_ux2, const float* d_uy2,
                            double rho0, void* hip_stream) {
    if (nx < 2 || ny < 1 || nx > kProjMax || ny > kProjMax || (nx & 1) || n_fields < 1) {
        nn_set_err(g_nn_err, "nx must be even and in [2, %d], ny in [1, %d], n_fields >= 1", kProjMax, kProjMax);
        return LBM_EINVAL;
    }
    if (!d_owner || !d_rho || !d_ux || !d_uy || !(rho0 > 0.0)) {
        nn_set_err(g_nn_err, "field pointers must not be NULL and rho0 must be > 0");
        return LBM_EINVAL;
    }
    const hipStream_t st = (hipStream_t)hip_stream;
    if (d_rho2 || d_ux2 || d_uy2) {
        if (!d_rho2 || !d_ux2 || !d_uy2) {
            nn_set_err(g_nn_err, "the second field set needs all three of rho, u_x, u_y");
            return LBM_EINVAL;
        }
        const int64_t n = (int64_t)n_fields * nx * ny;
        k_average<<<blocks(n), kEw, 0, st>>>(d_rho, d_rho2, n);
        k_average<<<blocks(n), kEw, 0, st>>>(d_ux, d_ux2, n);
        k_average<<<blocks(n), kEw, 0, st>>>(d_uy, d_uy2, n);
    }
    k_project<<<n_fields, kEw, 0, st>>>(d_owner, d_rho, d_ux, d_uy, nx, ny, rho0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        nn_set_err(g_nn_err, "projection launch failed: %s", hipGetErrorString(e));
        return LBM_EDEVICE;
    }
    return LBM_OK;
}

lbm_status lbm_warm_check(int32_t nx, int32_t ny, int32_t n_fields, const uint8_t* d_owner, const float* d_rho,
                          const float* d_ux, const float* d_uy, double rho0, double u_max, int32_t* d_ok,
                          void* hip_stream) {
    if (nx < 1 || ny < 1 || n_fields < 1 || !d_owner || !d_rho || !d_ux || !d_uy || !d_ok || !(rho0 > 0.0) ||
        !(u_max > 0.0)) {
        nn_set_err(g_nn_err, "sizes must be >= 1, pointers non-NULL, rho0 and u_max > 0");
        return LBM_EINVAL;
    }
    const hipStream_t st = (hipStream_t)hip_stream;
    k_fill_i32<<<blocks(n_fields), kEw, 0, st>>>(d_ok, n_fields, 1);
    k_warm_check<<<n_fields, kEw, 0, st>>>(d_owner, d_rho, d_ux, d_uy, nx, ny, rho0, u_max, d_ok);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        nn_set_err(g_nn_err, "start check launch failed: %s", hipGetErrorString(e));
        return LBM_EDEVICE;
    }
    return LBM_OK;
}

void lbm_nn_destroy(lbm_nn* n) {
    if (!n) return;
    (void)hipStreamSynchronize(n->st);
    delete n;
}

const char* lbm_nn_last_error(const lbm_nn* n) { return n ? n->err : g_nn_err; }

}  // extern "C"
