// nn_kernels.h -- HIP kernels of the learned warm-start network (gfx950).
//
// Network: 4-level U-Net on a channel lattice (mask, Re) -> (rho, u_x, u_y),
// channels (c0, c1, c2, c3), 3x3 convolutions with bias and ReLU, 2x2 mean
// pooling, nearest 2x upsampling, concatenated skips [up, skip], and the
// bottleneck's per-sample channel mean broadcast into the first decoder level
// (global context: the flow rate of a periodic channel depends on every body
// in it); x periodic, y zero-padded (walls).  Activations are NHWC in the compute type T
// (__bf16 with FP32 accumulation on the matrix cores, or float for an
// all-FP32 mode); weights are FP32 masters repacked into T.
//
// Convolution as an implicit GEMM on MFMA: M = pixels (the flattened
// (b, y, x) index in 32-pixel blocks), N = output channels (32-channel
// blocks), K = 9 taps x input channels in chunks of 16.  Each lane of a
// 32x32 block owns one pixel (A) or one output channel (B) and 8 consecutive
// channels of the chunk, so every operand load is one 16-byte (BF16) or
// 32-byte (FP32) vector.  The input gradient is the same kernel on weights
// flipped in (ky, kx) and transposed to [c_in][tap][c_out]; the weight
// gradient is a second GEMM with K = pixels, split over workgroups and
// combined in a fixed order (no atomics: results are reproducible).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kConvWaves = 4;  // waves per convolution workgroup
constexpr int kEw = 256;       // threads per elementwise workgroup

__device__ inline float to_f(float v) { return v; }
__device__ inline float to_f(__bf16 v) { return (float)v; }
template <typename T>
__device__ inline T from_f(float v);
template <>
__device__ inline float from_f<float>(float v) { return v; }
template <>
__device__ inline __bf16 from_f<__bf16>(float v) { return (__bf16)v; }  // round to nearest even

// Eight consecutive elements of T at p (16- or 32-byte aligned), or zeros.
template <typename T>
struct Frag;
template <>
struct Frag<__bf16> {
    bf16x8 v;
    __device__ inline void load(const __bf16* p) { v = *reinterpret_cast<const bf16x8*>(p); }
    __device__ inline void zero() {
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)0.0f;
    }
    __device__ inline void set(int e, __bf16 x) { v[e] = x; }
};
template <>
struct Frag<float> {
    float v[8];
    __device__ inline void load(const float* p) {
        const float4 a = reinterpret_cast<const float4*>(p)[0];
        const float4 b = reinterpret_cast<const float4*>(p)[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    }
    __device__ inline void zero() {
        for (int e = 0; e < 8; ++e) v[e] = 0.0f;
    }
    __device__ inline void set(int e, float x) { v[e] = x; }
};

// acc += A(32 x 16) * B(16 x 32).  Lane l holds A[l % 32][8 (l / 32) + e] and
// B[8 (l / 32) + e][l % 32], e = 0..7.  The FP32 form issues eight K = 2
// steps pairing element e of the two lane halves, which is the same sum.
__device__ inline void mma(f32x16& acc, const Frag<__bf16>& a, const Frag<__bf16>& b) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, b.v, acc, 0, 0, 0);
}
__device__ inline void mma(f32x16& acc, const Frag<float>& a, const Frag<float>& b) {
#pragma unroll
    for (int e = 0; e < 8; ++e) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[e], b.v[e], acc, 0, 0, 0);
}

// Row m of accumulator register j in lane l of a 32x32 block (column l % 32).
__device__ inline int acc_row(int j, int l) { return 8 * (j >> 2) + 4 * (l >> 5) + (j & 3); }

// ------------------------------------------------------------------ convolution
struct ConvArgs {
    const void* in;        // T [P][in_cs], channels [0, cin) read
    int in_cs, cin;        // cin: multiple of 16
    const void* w;         // T [cout_pad][9][cin]
    const float* bias;     // [cout_pad] or null
    void* out;             // T (or float for the network output) [P][out_cs]
    int out_cs, out_co;    // channel stride and offset of the stored channels
    int cout;              // channels stored: [0, cout)
    const void* mask;      // optional T [P][mask_cs]: out *= (mask[.][mask_co + n] > 0)
    int mask_cs, mask_co;
    int relu;
    int P, H, W;           // P = B * H * W pixels of this level
    int out_f32;           // k_conv_lds: store the output as float (network head)
};

// Workgroup: kConvWaves waves; wave w takes pixels
// [(blockIdx.x * kConvWaves + w) * 32 MB, + 32 MB) and output channels
// [blockIdx.y * 32 NB, + 32 NB).
template <typename T, typename OT, int MB, int NB>
__global__ __launch_bounds__(kConvWaves * 64) void k_conv(ConvArgs a) {
    const int l = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int pbase = (blockIdx.x * kConvWaves + wave) * 32 * MB;
    const int nbase = blockIdx.y * 32 * NB;
    const int kg = l >> 5;
    const T* in = static_cast<const T*>(a.in);
    const T* w = static_cast<const T*>(a.w);
    const int HW = a.H * a.W;
    int pb[MB], py[MB], px[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int p = pbase + 32 * i + (l & 31);
        const int b = p / HW;
        const int r = p - b * HW;
        pb[i] = p < a.P ? b : -1;
        py[i] = r / a.W;
        px[i] = r - py[i] * a.W;
    }
    f32x16 acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.0f;
    const int wrow = 9 * a.cin;
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const T* src[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int yy = py[i] + dy;
            int xx = px[i] + dx;
            xx = xx < 0 ? xx + a.W : (xx >= a.W ? xx - a.W : xx);
            const bool ok = pb[i] >= 0 && yy >= 0 && yy < a.H;
            src[i] = ok ? in + ((int64_t)(pb[i] * a.H + yy) * a.W + xx) * a.in_cs + 8 * kg : nullptr;
        }
        const T* wsrc[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) wsrc[j] = w + (int64_t)(nbase + 32 * j + (l & 31)) * wrow + tap * a.cin + 8 * kg;
        for (int c0 = 0; c0 < a.cin; c0 += 16) {
            Frag<T> fa[MB], fb[NB];
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                if (src[i])
                    fa[i].load(src[i] + c0);
                else
                    fa[i].zero();
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) fb[j].load(wsrc[j] + c0);
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) mma(acc[i][j], fa[i], fb[j]);
        }
    }
    OT* out = static_cast<OT*>(a.out);
    const T* mask = static_cast<const T*>(a.mask);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int n = nbase + 32 * j + (l & 31);
        if (n >= a.cout) continue;
        const float bv = a.bias ? a.bias[n] : 0.0f;
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int p = pbase + 32 * i + acc_row(q, l);
                if (p >= a.P) continue;
                float v = acc[i][j][q] + bv;
                if (a.relu) v = v > 0.0f ? v : 0.0f;
                if (mask && !(to_f(mask[(int64_t)p * a.mask_cs + a.mask_co + n]) > 0.0f)) v = 0.0f;
                out[(int64_t)p * a.out_cs + a.out_co + n] = from_f<OT>(v);
            }
    }
}

// One 16-byte A segment of the BF16 convolution: 8 channels from c of node
// (b, yy, xx) with x periodic, zero outside the walls or for b < 0.
__device__ __forceinline__ uint4 conv_load_a(const __bf16* in, int b, int yy, int xx, int H, int W, int cs, int c) {
    xx = xx < 0 ? xx + W : (xx >= W ? xx - W : xx);
    if (b >= 0 && yy >= 0 && yy < H) return *reinterpret_cast<const uint4*>(in + ((int64_t)(b * H + yy) * W + xx) * cs + c);
    return make_uint4(0, 0, 0, 0);
}

// BF16 convolution with LDS-staged operands.  Workgroup tile: BM = 32 WM MW
// pixels x BN = 32 WN NW output channels, four waves in an MW x NW grid, each
// owning WM x WN MFMA blocks.  The K loop runs over stages of one tap x BK
// input channels: the stage's A tile (BM pixels, shifted by the tap, zero
// outside the walls) and B tile (BN weight rows) are read from global memory
// into registers while the MFMAs of the previous stage run from LDS, then
// written to the other of two LDS buffers (rows padded by 8 elements), with
// one barrier per stage.  Same arguments and epilogue as k_conv.
template <int MW, int NW, int WM, int WN, int BK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 3))) void k_conv_lds(ConvArgs a) {
    static_assert(MW * NW == 4, "four waves");
    constexpr int BM = 32 * WM * MW, BN = 32 * WN * NW;
    constexpr int LDK = BK + 8;                 // padded LDS row (elements)
    constexpr int SEG = BK / 8;                 // 16-byte segments per row
    constexpr int A_SEGS = BM * SEG, B_SEGS = BN * SEG;
    constexpr int A_PER = (A_SEGS + 255) / 256, B_PER = (B_SEGS + 255) / 256;
    __shared__ __align__(16) __bf16 As[2][BM * LDK];
    __shared__ __align__(16) __bf16 Bs[2][BN * LDK];
    const int t = threadIdx.x;
    const int l = t & 63, wave = t >> 6;
    const int wm = wave % MW, wn = wave / MW;
    const int kg = l >> 5;
    const int pbase = blockIdx.x * BM;
    const int nbase = blockIdx.y * BN;
    const __bf16* in = static_cast<const __bf16*>(a.in);
    const __bf16* w = static_cast<const __bf16*>(a.w);
    const int HW = a.H * a.W;
    // the A rows this thread loads, and their (b, y, x)
    int ar[A_PER], as_[A_PER], ab[A_PER], ay[A_PER], ax[A_PER];
#pragma unroll
    for (int r = 0; r < A_PER; ++r) {
        const int id = t + 256 * r;
        ar[r] = id / SEG;
        as_[r] = id % SEG;
        const int p = pbase + ar[r];
        const int b = p / HW, rem = p - b * HW;
        ab[r] = (id < A_SEGS && p < a.P) ? b : -1;
        ay[r] = rem / a.W;
        ax[r] = rem - ay[r] * a.W;
    }
    int br[B_PER], bsg[B_PER];
#pragma unroll
    for (int r = 0; r < B_PER; ++r) {
        const int id = t + 256 * r;
        br[r] = id < B_SEGS ? id / SEG : -1;
        bsg[r] = id % SEG;
    }
    const int kchunks = a.cin / BK;
    const int nst = 9 * kchunks;
    const int wrow = 9 * a.cin;
    uint4 ra[A_PER], rb[B_PER];
    f32x16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.0f;
#define CONV_LDS_GLOAD(ST)                                                                                     \
    {                                                                                                          \
        const int tap_ = (ST) / kchunks, c0_ = ((ST) - tap_ * kchunks) * BK;                                    \
        const int dy_ = tap_ / 3 - 1, dx_ = tap_ % 3 - 1;                                                      \
        _Pragma("unroll") for (int r = 0; r < A_PER; ++r) ra[r] =                                                \
            conv_load_a(in, ab[r], ay[r] + dy_, ax[r] + dx_, a.H, a.W, a.in_cs, c0_ + 8 * as_[r]);              \
        _Pragma("unroll") for (int r = 0; r < B_PER; ++r) if (br[r] >= 0) rb[r] =                                \
            *reinterpret_cast<const uint4*>(w + (int64_t)(nbase + br[r]) * wrow + tap_ * a.cin + c0_ + 8 * bsg[r]); \
    }
#define CONV_LDS_LSTORE(BUF)                                                                                   \
    {                                                                                                          \
        _Pragma("unroll") for (int r = 0; r < A_PER; ++r) if (t + 256 * r < A_SEGS)                              \
            *reinterpret_cast<uint4*>(&As[BUF][ar[r] * LDK + 8 * as_[r]]) = ra[r];                              \
        _Pragma("unroll") for (int r = 0; r < B_PER; ++r) if (br[r] >= 0)                                        \
            *reinterpret_cast<uint4*>(&Bs[BUF][br[r] * LDK + 8 * bsg[r]]) = rb[r];                              \
    }
    CONV_LDS_GLOAD(0)
    CONV_LDS_LSTORE(0)
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        if (st + 1 < nst) CONV_LDS_GLOAD(st + 1)
#pragma unroll
        for (int kk = 0; kk < BK / 16; ++kk) {
            Frag<__bf16> fa[WM], fb[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i)
                fa[i].v = *reinterpret_cast<const bf16x8*>(&As[buf][((wm * WM + i) * 32 + (l & 31)) * LDK + kk * 16 + 8 * kg]);
#pragma unroll
            for (int j = 0; j < WN; ++j)
                fb[j].v = *reinterpret_cast<const bf16x8*>(&Bs[buf][((wn * WN + j) * 32 + (l & 31)) * LDK + kk * 16 + 8 * kg]);
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) mma(acc[i][j], fa[i], fb[j]);
        }
        if (st + 1 < nst) CONV_LDS_LSTORE(buf ^ 1)
        __syncthreads();
    }
#undef CONV_LDS_GLOAD
#undef CONV_LDS_LSTORE
    const __bf16* mask = static_cast<const __bf16*>(a.mask);
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        const int n = nbase + (wn * WN + j) * 32 + (l & 31);
        if (n >= a.cout) continue;
        const float bv = a.bias ? a.bias[n] : 0.0f;
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int p = pbase + (wm * WM + i) * 32 + acc_row(q, l);
                if (p >= a.P) continue;
                float v = acc[i][j][q] + bv;
                if (a.relu) v = v > 0.0f ? v : 0.0f;
                if (mask && !(to_f(mask[(int64_t)p * a.mask_cs + a.mask_co + n]) > 0.0f)) v = 0.0f;
                if (a.out_f32)
                    static_cast<float*>(a.out)[(int64_t)p * a.out_cs + a.out_co + n] = v;
                else
                    static_cast<__bf16*>(a.out)[(int64_t)p * a.out_cs + a.out_co + n] = (__bf16)v;
            }
    }
}

// 3x3 convolution with the input tile held across the nine taps (BF16).  A
// workgroup computes an output tile of kC9Rows rows x 32 pixels of one image
// for 32 NB output channels; per 32-channel chunk of the input it stages in
// LDS the tile's input with a one-pixel halo (rows y0 - 1 .. y0 + kC9Rows,
// columns x0 - 1 .. x0 + 32, x periodic, rows outside the image zero) and
// the chunk's weights of all nine taps, so each input value is read from
// memory once per chunk instead of once per tap.  Wave w takes output rows
// 2w and 2w + 1; the operand of tap (dy, dx) for output pixel (r, m) is the
// staged pixel (r + 1 + dy, m + 1 + dx): 8 consecutive channels, one aligned
// 16-byte LDS vector.  Same epilogue as k_conv_lds.  Needs H % kC9Rows == 0,
// W % 32 == 0, cin % 32 == 0 and cout_pad % (32 NB) == 0.
constexpr int kC9Rows = 8;
constexpr int kC9Pitch = 40;  // LDS elements per staged pixel / weight row (32 + 8 pad)

template <int NB, bool PF>
__global__ __launch_bounds__(256) void k_conv9(ConvArgs a) {
    constexpr int IR = kC9Rows + 2, IX = 34;         // staged input rows, pixels
    constexpr int IN_UNITS = IR * IX * 4;            // 16-byte units (8 channels)
    constexpr int W_UNITS = 32 * NB * 9 * 4;
    __shared__ __align__(16) __bf16 Is[IR * IX * kC9Pitch];
    __shared__ __align__(16) __bf16 Ws[32 * NB * 9 * kC9Pitch];
    const int t = threadIdx.x;
    const int l = t & 63, wave = t >> 6;
    const int kg = l >> 5;
    const int nseg = a.W / 32, nrow = a.H / kC9Rows;
    int tile = blockIdx.x;
    const int seg = tile % nseg;
    tile /= nseg;
    const int rb = tile % nrow;
    const int b = tile / nrow;
    const int x0 = seg * 32, y0 = rb * kC9Rows;
    const int nbase = blockIdx.y * 32 * NB;
    const __bf16* in = static_cast<const __bf16*>(a.in);
    const __bf16* w = static_cast<const __bf16*>(a.w);
    const int wrow = 9 * a.cin;
    f32x16 acc[2][NB];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.0f;
// the products of one staged chunk: nine taps x two K = 16 steps
#define C9_PRODUCTS()                                                                                 \
    _Pragma("unroll") for (int tap = 0; tap < 9; ++tap) {                                            \
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;                                                 \
        _Pragma("unroll") for (int ks = 0; ks < 2; ++ks) {                                            \
            Frag<__bf16> fa[2], fb[NB];                                                               \
            _Pragma("unroll") for (int i = 0; i < 2; ++i) {                                           \
                const int r = 2 * wave + i + 1 + dy, px = (l & 31) + 1 + dx;                          \
                fa[i].v = *reinterpret_cast<const bf16x8*>(&Is[(r * IX + px) * kC9Pitch + 16 * ks + 8 * kg]); \
            }                                                                                         \
            _Pragma("unroll") for (int j = 0; j < NB; ++j) fb[j].v = *reinterpret_cast<const bf16x8*>( \
                &Ws[((32 * j + (l & 31)) * 9 + tap) * kC9Pitch + 16 * ks + 8 * kg]);                  \
            _Pragma("unroll") for (int i = 0; i < 2; ++i)                                            \
                _Pragma("unroll") for (int j = 0; j < NB; ++j) mma(acc[i][j], fa[i], fb[j]);          \
        }                                                                                             \
    }
    // PF: the next chunk's input and weights wait in registers while this
    // chunk's products run (more registers; pays where few tiles share the
    // chip); otherwise each chunk is loaded straight into LDS
    if constexpr (!PF) {
        for (int c0 = 0; c0 < a.cin; c0 += 32) {
            for (int u = t; u < IN_UNITS; u += 256) {
                const int cg = u & 3, px = (u >> 2) % IX, r = (u >> 2) / IX;
                const int yy = y0 - 1 + r;
                int xx = x0 - 1 + px;
                xx = xx < 0 ? xx + a.W : (xx >= a.W ? xx - a.W : xx);
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (yy >= 0 && yy < a.H)
                    v = *reinterpret_cast<const uint4*>(in + ((int64_t)(b * a.H + yy) * a.W + xx) * a.in_cs + c0 + 8 * cg);
                *reinterpret_cast<uint4*>(&Is[(r * IX + px) * kC9Pitch + 8 * cg]) = v;
            }
            for (int u = t; u < W_UNITS; u += 256) {
                const int cg = u & 3, tap = (u >> 2) % 9, n = (u >> 2) / 9;
                *reinterpret_cast<uint4*>(&Ws[(n * 9 + tap) * kC9Pitch + 8 * cg]) =
                    *reinterpret_cast<const uint4*>(w + (int64_t)(nbase + n) * wrow + tap * a.cin + c0 + 8 * cg);
            }
            __syncthreads();
            C9_PRODUCTS()
            __syncthreads();
        }
    } else {
    constexpr int IN_PER = (IN_UNITS + 255) / 256, W_PER = (W_UNITS + 255) / 256;
    u32x4 rin[IN_PER], rw[W_PER];
#define C9_GLOAD(C0)                                                                                             \
    {                                                                                                            \
        _Pragma("unroll") for (int k = 0; k < IN_PER; ++k) {                                                       \
            const int u = t + 256 * k;                                                                           \
            rin[k] = u32x4{0u, 0u, 0u, 0u};                                                                 \
            if (u < IN_UNITS) {                                                                                  \
                const int cg = u & 3, px = (u >> 2) % IX, r = (u >> 2) / IX;                                     \
                const int yy = y0 - 1 + r;                                                                       \
                int xx = x0 - 1 + px;                                                                            \
                xx = xx < 0 ? xx + a.W : (xx >= a.W ? xx - a.W : xx);                                            \
                if (yy >= 0 && yy < a.H)                                                                         \
                    rin[k] = *reinterpret_cast<const u32x4*>(in + ((int64_t)(b * a.H + yy) * a.W + xx) * a.in_cs + \
                                                             (C0) + 8 * cg);                                     \
            }                                                                                                    \
        }                                                                                                        \
        _Pragma("unroll") for (int k = 0; k < W_PER; ++k) {                                                        \
            const int u = t + 256 * k;                                                                           \
            if (u < W_UNITS) {                                                                                   \
                const int cg = u & 3, tap = (u >> 2) % 9, n = (u >> 2) / 9;                                      \
                rw[k] = *reinterpret_cast<const u32x4*>(w + (int64_t)(nbase + n) * wrow + tap * a.cin + (C0) + 8 * cg); \
            }                                                                                                    \
        }                                                                                                        \
    }
#define C9_LSTORE()                                                                                              \
    {                                                                                                            \
        _Pragma("unroll") for (int k = 0; k < IN_PER; ++k) {                                                       \
            const int u = t + 256 * k;                                                                           \
            if (u < IN_UNITS) {                                                                                  \
                const int cg = u & 3, px = (u >> 2) % IX, r = (u >> 2) / IX;                                     \
                *reinterpret_cast<u32x4*>(&Is[(r * IX + px) * kC9Pitch + 8 * cg]) = rin[k];                      \
            }                                                                                                    \
        }                                                                                                        \
        _Pragma("unroll") for (int k = 0; k < W_PER; ++k) {                                                        \
            const int u = t + 256 * k;                                                                           \
            if (u < W_UNITS) {                                                                                   \
                const int cg = u & 3, tap = (u >> 2) % 9, n = (u >> 2) / 9;                                      \
                *reinterpret_cast<u32x4*>(&Ws[(n * 9 + tap) * kC9Pitch + 8 * cg]) = rw[k];                       \
            }                                                                                                    \
        }                                                                                                        \
    }
    C9_GLOAD(0)
    C9_LSTORE()
    __syncthreads();
    for (int c0 = 0; c0 < a.cin; c0 += 32) {
        if (c0 + 32 < a.cin) C9_GLOAD(c0 + 32)
        C9_PRODUCTS()
        __syncthreads();
        if (c0 + 32 < a.cin) {
            C9_LSTORE()
            __syncthreads();
        }
    }
#undef C9_GLOAD
#undef C9_LSTORE
    }
#undef C9_PRODUCTS
    const __bf16* mask = static_cast<const __bf16*>(a.mask);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int n = nbase + 32 * j + (l & 31);
        if (n >= a.cout) continue;
        const float bv = a.bias ? a.bias[n] : 0.0f;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int p = (b * a.H + y0 + 2 * wave + i) * a.W + x0 + acc_row(q, l);
                float v = acc[i][j][q] + bv;
                if (a.relu) v = v > 0.0f ? v : 0.0f;
                if (mask && !(to_f(mask[(int64_t)p * a.mask_cs + a.mask_co + n]) > 0.0f)) v = 0.0f;
                if (a.out_f32)
                    static_cast<float*>(a.out)[(int64_t)p * a.out_cs + a.out_co + n] = v;
                else
                    static_cast<__bf16*>(a.out)[(int64_t)p * a.out_cs + a.out_co + n] = (__bf16)v;
            }
    }
}

// ------------------------------------------------------------------ weight gradient
// dW[co][tap][ci] = sum over pixels p of g[p][co] x(p shifted by tap)[ci].
// Workgroup (tile, split): co block of 32 MB, ci block of 32 NB, one tap;
// pixels [k0, k1) of the split in chunks of 16, chunk c to wave c % 4.  The
// four waves are combined in LDS in wave order; the partial of the split goes
// to part[split][co][tap][ci] (real channels only).  The centre-tap tiles of
// the first ci block also sum their g operand: the bias gradient
// db[co] = sum over p of g[p][co], at part[split][cout * 9 * cin + co].
struct WgradArgs {
    const void* g;   // T [P][g_cs]; channels [0, cout_pad) readable
    int g_cs;
    const void* x;   // T [P][x_cs]; channels [0, cin) used
    int x_cs;
    int cout, cin;   // real channel counts
    int co_blocks, ci_blocks;  // in units of 32 MB / 32 NB
    int P, H, W;
    int chunk_per_split;       // pixels per split (multiple of 64)
    float* part;     // [splits][cout * 9 * cin + cout]: weights, then the bias
};

template <typename T, int MB, int NB>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
    __shared__ float red[3][MB * NB * 16][64];
    __shared__ float bred[3][MB][64];
    const int l = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int kg = l >> 5;
    int tile = blockIdx.x;
    const int tap = tile % 9;
    tile /= 9;
    const int cib = tile % a.ci_blocks;
    const int cob = tile / a.ci_blocks;
    const int split = blockIdx.y;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const T* g = static_cast<const T*>(a.g);
    const T* x = static_cast<const T*>(a.x);
    const int k0 = split * a.chunk_per_split;
    const int k1 = min(a.P, k0 + a.chunk_per_split);
    f32x16 acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.0f;
    const bool bias_tile = tap == 4 && cib == 0;
    float bsum[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) bsum[i] = 0.0f;
    int co_l[MB], ci_l[NB];
#pragma unroll
    for (int i = 0; i < MB; ++i) co_l[i] = (cob * MB + i) * 32 + (l & 31);
#pragma unroll
    for (int j = 0; j < NB; ++j) ci_l[j] = (cib * NB + j) * 32 + (l & 31);
    for (int c = k0 + 16 * wave; c < k1; c += 64) {
        // the lane's 8 pixels c + 8 kg + e lie in one row (W is a multiple of 8)
        const int p0 = c + 8 * kg;
        Frag<T> fa[MB], fb[NB];
        if (p0 < k1) {
            const int row = p0 / a.W;  // b * H + y
            const int x0 = p0 - row * a.W;
            const int b = row / a.H;
            const int yy = row - b * a.H + dy;
            const bool yok = yy >= 0 && yy < a.H;
            const int64_t srow = (int64_t)(b * a.H + yy) * a.W;
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const T gv = g[(int64_t)(p0 + e) * a.g_cs + co_l[i]];
                    fa[i].set(e, gv);
                    if (bias_tile) bsum[i] += to_f(gv);
                }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const bool cok = ci_l[j] < a.cin;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    int xx = x0 + e + dx;
                    xx = xx < 0 ? xx + a.W : (xx >= a.W ? xx - a.W : xx);
                    fb[j].set(e, (yok && cok) ? x[(srow + xx) * a.x_cs + ci_l[j]] : from_f<T>(0.0f));
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < MB; ++i) fa[i].zero();
#pragma unroll
            for (int j = 0; j < NB; ++j) fb[j].zero();
        }
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) mma(acc[i][j], fa[i], fb[j]);
    }
    if (wave > 0) {
#pragma unroll
        for (int i = 0; i < MB; ++i) {
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int q = 0; q < 16; ++q) red[wave - 1][(i * NB + j) * 16 + q][l] = acc[i][j][q];
            bred[wave - 1][i][l] = bsum[i];
        }
    }
    __syncthreads();
    if (wave != 0) return;
    const int64_t nw = (int64_t)a.cout * 9 * a.cin;
    const int64_t slab = nw + a.cout;
    float* part = a.part + (int64_t)split * slab;
    if (bias_tile) {
        // lanes l and l ^ 32 hold the two 8-pixel halves of the same channel
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            float v = ((bsum[i] + bred[0][i][l]) + bred[1][i][l]) + bred[2][i][l];
            v += __shfl_xor(v, 32, 64);
            if (l < 32 && co_l[i] < a.cout) part[nw + co_l[i]] = v;
        }
    }
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int r = (i * NB + j) * 16 + q;
                const float v = ((acc[i][j][q] + red[0][r][l]) + red[1][r][l]) + red[2][r][l];
                const int co = (cob * MB + i) * 32 + acc_row(q, l);
                const int ci = ci_l[j];
                if (co < a.cout && ci < a.cin) part[((int64_t)co * 9 + tap) * a.cin + ci] = v;
            }
}

// Weight gradient with all nine taps in one workgroup (BF16).  A tile is
// kWgTile consecutive pixels of one image row (b, y, [x0, x0 + kWgTile)).
// The workgroup stages, transposed to channel-major so that a lane's eight
// consecutive pixels are one 16-byte LDS vector, the tile's g (its 32 MB
// output channels) and x of rows y - 1, y, y + 1 over columns
// [x0 - 4, x0 + kWgTile + 4) (x periodic, rows outside the image zero), its
// 32 NB input channels.  Wave (j, r) takes input block j and row offset
// dy = r - 1 for all three dx and all MB output blocks: the dx = -1 and +1
// operands are the dx = 0 vector shifted by one pixel, with the neighbouring
// pixel taken from the words before and after it, so the g operand and the
// x vector are read once for three products.  Tiles [split * tps, + tps)
// go through a double-buffered LDS stage (next tile's global loads in
// registers during the products).  Partial sums go to part[split] as for
// k_wgrad; the first input block of a split also sums g into the bias slot,
// per channel group in pixel order, then over the groups in order.
constexpr int kWgTile = 32;                // pixels per tile
constexpr int kWgXPitch = kWgTile + 24;    // x row: halo 4 + 4 guard + tile + 4 + 12 (odd multiple of 16 B)
constexpr int kWgGPitch = kWgTile + 8;     // g row (odd multiple of 16 B)
constexpr int kWgGroups = kWgTile / 4 + 2; // 4-pixel column groups of an x row (with halos)

struct Wgrad9Args {
    const __bf16* g;  // [P][g_cs]; channels [0, cout_pad) readable
    int g_cs;
    const __bf16* x;  // [P][x_cs]; channels [0, cin) read, x_cs and the offset multiples of 8
    int x_cs;
    int cout, cin;    // real channel counts
    int ci_blocks;    // input blocks of 32 NB channels
    int H, W;         // level size; W a multiple of kWgTile
    int ntiles;       // B * H * W / kWgTile
    int tps;          // tiles per split
    float* part;      // [splits][cout * 9 * cin + cout]
};

__device__ inline uint32_t lo_pair(uint32_t a, uint32_t b) { return (a & 0xffffu) | (b << 16); }
__device__ inline uint32_t hi_pair(uint32_t a, uint32_t b) { return (a >> 16) | (b & 0xffff0000u); }
// bf16 elements (1..8) of the 9 consecutive ones (w0.lo .. w4.lo): a shift by one element
__device__ inline uint32_t shift1(uint32_t a, uint32_t b) { return (a >> 16) | (b << 16); }

template <int MB, int NB>
__global__ __launch_bounds__(192 * NB) void k_wgrad9(Wgrad9Args a) {
    constexpr int NT = 192 * NB;
    constexpr int NG = (kWgTile / 4) * 4 * MB;   // g units: 4 pixels x 8 channels
    constexpr int NX = 3 * kWgGroups * 4 * NB;   // x units
    static_assert(NG + NX <= NT, "one staging unit per thread");
    __shared__ __align__(16) __bf16 Xs[2][3][32 * NB][kWgXPitch];
    __shared__ __align__(16) __bf16 Gs[2][32 * MB][kWgGPitch];
    __shared__ float bred[kWgTile / 4][32 * MB];
    const int t = threadIdx.x;
    const int l = t & 63;
    const int wave = t >> 6;
    const int wj = wave / 3, wr = wave % 3;
    const int cob = blockIdx.x / a.ci_blocks, cib = blockIdx.x % a.ci_blocks;
    const int split = blockIdx.y;
    const int nseg = a.W / kWgTile;
    const int t0 = split * a.tps;
    const int t1 = min(a.ntiles, t0 + a.tps);
    const bool bias_wg = cib == 0;

    // this thread's staging unit
    const bool is_g = t < NG;
    const bool is_x = !is_g && t < NG + NX;
    int u_ch, u_grp, u_row;  // channel group (8 channels), pixel group, x row (0..2)
    if (is_g) {
        u_ch = t % (4 * MB);
        u_grp = t / (4 * MB);
        u_row = 0;
    } else {
        const int v = t - NG;
        u_ch = v % (4 * NB);
        u_grp = (v / (4 * NB)) % kWgGroups;
        u_row = v / (4 * NB * kWgGroups);
    }
    const int gch = cob * 32 * MB + 8 * u_ch;             // g channel of the unit
    const int xch = cib * 32 * NB + 8 * u_ch;             // x channel of the unit
    const bool x_ok = is_x && xch < a.cin;                 // group holds real channels
    float bsum[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) bsum[c] = 0.0f;
    uint4 reg[4];

    auto gload = [&](int tile) {
        const int seg = tile % nseg;
        const int row = tile / nseg;  // b * H + y
        const int x0 = seg * kWgTile;
#pragma unroll
        for (int e = 0; e < 4; ++e) reg[e] = make_uint4(0u, 0u, 0u, 0u);
        if (is_g) {
            const int64_t p = (int64_t)row * a.W + x0 + 4 * u_grp;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                reg[e] = *reinterpret_cast<const uint4*>(a.g + (p + e) * a.g_cs + gch);
        } else if (x_ok) {
            const int b = row / a.H;
            const int yy = row - b * a.H + u_row - 1;
            if (yy >= 0 && yy < a.H) {
                int xx = x0 - 4 + 4 * u_grp;
                xx = xx < 0 ? xx + a.W : (xx >= a.W ? xx - a.W : xx);
                const int64_t p = ((int64_t)b * a.H + yy) * a.W + xx;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    reg[e] = *reinterpret_cast<const uint4*>(a.x + (p + e) * a.x_cs + xch);
            }
        }
    };
    auto lstore = [&](int buf) {
        if (!is_g && !is_x) return;
        const uint32_t w[4][4] = {{reg[0].x, reg[0].y, reg[0].z, reg[0].w},
                                  {reg[1].x, reg[1].y, reg[1].z, reg[1].w},
                                  {reg[2].x, reg[2].y, reg[2].z, reg[2].w},
                                  {reg[3].x, reg[3].y, reg[3].z, reg[3].w}};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // channels 2k and 2k + 1 of the four pixels
            const uint2 ev = make_uint2(lo_pair(w[0][k], w[1][k]), lo_pair(w[2][k], w[3][k]));
            const uint2 od = make_uint2(hi_pair(w[0][k], w[1][k]), hi_pair(w[2][k], w[3][k]));
            __bf16* d0;
            __bf16* d1;
            if (is_g) {
                d0 = &Gs[buf][8 * u_ch + 2 * k][4 * u_grp];
                d1 = &Gs[buf][8 * u_ch + 2 * k + 1][4 * u_grp];
            } else {
                d0 = &Xs[buf][u_row][8 * u_ch + 2 * k][4 + 4 * u_grp];
                d1 = &Xs[buf][u_row][8 * u_ch + 2 * k + 1][4 + 4 * u_grp];
            }
            *reinterpret_cast<uint2*>(d0) = ev;
            *reinterpret_cast<uint2*>(d1) = od;
        }
    };
    auto bias_add = [&]() {
        if (!(bias_wg && is_g)) return;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t w[4] = {reg[e].x, reg[e].y, reg[e].z, reg[e].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                bsum[2 * k] += __uint_as_float(w[k] << 16);
                bsum[2 * k + 1] += __uint_as_float(w[k] & 0xffff0000u);
            }
        }
    };

    f32x16 acc[MB][3];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[i][d][q] = 0.0f;

    gload(t0);
    bias_add();
    lstore(0);
    __syncthreads();
    for (int tile = t0; tile < t1; ++tile) {
        const int buf = (tile - t0) & 1;
        if (tile + 1 < t1) gload(tile + 1);
#pragma unroll
        for (int ks = 0; ks < kWgTile / 16; ++ks) {
            const int k8 = 16 * ks + 8 * (l >> 5);
            const __bf16* xr = &Xs[buf][wr][32 * wj + (l & 31)][8 + k8];
            const uint4 mid = *reinterpret_cast<const uint4*>(xr);
            const uint32_t prev = *reinterpret_cast<const uint32_t*>(xr - 2);
            const uint32_t next = *reinterpret_cast<const uint32_t*>(xr + 8);
            Frag<__bf16> fb[3];
            // x at pixel p + dx for dx = -1, 0, +1
            const uint4 bm = make_uint4(shift1(prev, mid.x), shift1(mid.x, mid.y), shift1(mid.y, mid.z),
                                        shift1(mid.z, mid.w));
            const uint4 bp = make_uint4(shift1(mid.x, mid.y), shift1(mid.y, mid.z), shift1(mid.z, mid.w),
                                        shift1(mid.w, next));
            fb[0].v = __builtin_bit_cast(bf16x8, bm);
            fb[1].v = __builtin_bit_cast(bf16x8, mid);
            fb[2].v = __builtin_bit_cast(bf16x8, bp);
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                Frag<__bf16> fa;
                fa.v = *reinterpret_cast<const bf16x8*>(&Gs[buf][32 * i + (l & 31)][k8]);
#pragma unroll
                for (int d = 0; d < 3; ++d) mma(acc[i][d], fa, fb[d]);
            }
        }
        if (tile + 1 < t1) {
            bias_add();
            lstore(buf ^ 1);
        }
        __syncthreads();
    }

    const int64_t nw = (int64_t)a.cout * 9 * a.cin;
    float* part = a.part + (int64_t)split * (nw + a.cout);
    if (bias_wg) {
        if (is_g) {
#pragma unroll
            for (int c = 0; c < 8; ++c) bred[u_grp][8 * u_ch + c] = bsum[c];
        }
        __syncthreads();
        if (t < 32 * MB) {
            float v = bred[0][t];
#pragma unroll
            for (int k = 1; k < kWgTile / 4; ++k) v += bred[k][t];
            const int co = cob * 32 * MB + t;
            if (co < a.cout) part[nw + co] = v;
        }
    }
    const int ci = cib * 32 * NB + 32 * wj + (l & 31);
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int co = cob * 32 * MB + 32 * i + acc_row(q, l);
                if (co < a.cout && ci < a.cin) part[((int64_t)co * 9 + 3 * wr + d) * a.cin + ci] = acc[i][d][q];
            }
}

// grad[i] = sum over splits s of part[s][i], i < n.  Workgroup: 32 outputs
// x 8 rows; row r sums the splits s = r, r + 8, ... in order, then the rows
// are added in row order (a fixed order for a given split count).
constexpr int kSumCols = 32, kSumRows = kEw / kSumCols;
__global__ __launch_bounds__(kEw) void k_sum_splits(const float* __restrict__ part, int splits, int64_t n,
                                                    float* __restrict__ grad) {
    __shared__ float red[kSumRows][kSumCols + 1];
    const int c = threadIdx.x % kSumCols, r = threadIdx.x / kSumCols;
    const int64_t i = (int64_t)blockIdx.x * kSumCols + c;
    float v = 0.0f;
    if (i < n) {
#pragma unroll 4
        for (int s = r; s < splits; s += kSumRows) v += part[(int64_t)s * n + i];
    }
    red[r][c] = v;
    __syncthreads();
    if (r == 0 && i < n) {
        float t = red[0][c];
#pragma unroll
        for (int k = 1; k < kSumRows; ++k) t += red[k][c];
        grad[i] = t;
    }
}

// Column sums over nodes, two stages, fixed order (bias gradients, channel
// means and their adjoints).  Segment b (blockIdx.y) is the node range
// [b N, (b + 1) N) of a tensor a[.][cs] (channels [co, co + C)); workgroup x
// takes nodes [x R, (x + 1) R) of the segment.  Thread t handles channel
// t % C and node lane t / C of J = kEw / C lanes (C <= kEw); lanes are then
// combined in lane order into part[b][x][c].
template <typename T>
__global__ __launch_bounds__(kEw) void k_colsum_partial(const T* __restrict__ a, int cs, int co, int C, int64_t N,
                                                        int R, float* __restrict__ part) {
    __shared__ float red[kEw];
    const int J = kEw / C;
    const int t = threadIdx.x;
    const int c = t % C, j = t / C;
    const int64_t seg = blockIdx.y;
    const int64_t p0 = (int64_t)blockIdx.x * R;
    const int64_t p1 = p0 + R < N ? p0 + R : N;
    float v = 0.0f;
    if (j < J)
        for (int64_t p = p0 + j; p < p1; p += J) v += to_f(a[(seg * N + p) * cs + co + c]);
    red[t] = v;
    __syncthreads();
    if (t < C) {
        float s = 0.0f;
        for (int k = 0; k < J; ++k) s += red[k * C + t];
        part[(seg * gridDim.x + blockIdx.x) * C + t] = s;
    }
}

// out[b][c] = scale * sum over the nblk partials of segment b, written as
// float (fout) or as T (tout).  Workgroup: 32 outputs x 8 rows; row r sums
// the partials k = r, r + 8, ... in order, then the rows are added in order.
template <typename T>
__global__ __launch_bounds__(kEw) void k_colsum_final(const float* __restrict__ part, int nblk, int C, int B,
                                                      float scale, float* __restrict__ fout, T* __restrict__ tout) {
    __shared__ float red[kSumRows][kSumCols + 1];
    const int cc = threadIdx.x % kSumCols, r = threadIdx.x / kSumCols;
    const int i = blockIdx.x * kSumCols + cc;
    const bool ok = i < B * C;
    const int b = ok ? i / C : 0, c = ok ? i % C : 0;
    float v = 0.0f;
    if (ok) {
#pragma unroll 4
        for (int k = r; k < nblk; k += kSumRows) v += part[((int64_t)b * nblk + k) * C + c];
    }
    red[r][cc] = v;
    __syncthreads();
    if (r == 0 && ok) {
        float s = red[0][cc];
#pragma unroll
        for (int k = 1; k < kSumRows; ++k) s += red[k][cc];
        s *= scale;
        if (fout) fout[i] = s;
        if (tout) tout[i] = from_f<T>(s);
    }
}

// ------------------------------------------------------------------ pooling, upsampling
// Every kernel here takes 8 consecutive channels per thread (one 16-byte
// BF16 vector, two float4 in FP32 mode): channel counts, strides and offsets
// are multiples of 8.  The arithmetic per element is the plain elementwise
// one.
template <typename T>
__device__ inline void load8(const T* p, float f[8]);
template <>
__device__ inline void load8<__bf16>(const __bf16* p, float f[8]) {
    const uint4 u = *reinterpret_cast<const uint4*>(p);
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f[2 * k] = __uint_as_float(w[k] << 16);
        f[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
    }
}
template <>
__device__ inline void load8<float>(const float* p, float f[8]) {
    const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
    f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
    f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
}
template <typename T>
__device__ inline void store8(T* p, const float f[8]);
template <>
__device__ inline void store8<__bf16>(__bf16* p, const float f[8]) {
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (__bf16)f[e];  // round to nearest even
    *reinterpret_cast<bf16x8*>(p) = v;
}
template <>
__device__ inline void store8<float>(float* p, const float f[8]) {
    reinterpret_cast<float4*>(p)[0] = make_float4(f[0], f[1], f[2], f[3]);
    reinterpret_cast<float4*>(p)[1] = make_float4(f[4], f[5], f[6], f[7]);
}

// out[b][y][x][c] = mean of in[b][2y + i][2x + j][c] (level l -> l + 1).
template <typename T>
__global__ __launch_bounds__(kEw) void k_pool(const T* __restrict__ in, int in_cs, int in_co, int C,
                                              T* __restrict__ out, int Ho, int Wo, int B) {
    const int64_t i = (int64_t)blockIdx.x * kEw + threadIdx.x;
    const int C8 = C / 8;
    if (i >= (int64_t)B * Ho * Wo * C8) return;
    const int c = (int)(i % C8) * 8;
    const int64_t q = i / C8;
    const int xo = (int)(q % Wo);
    const int64_t by = q / Wo;  // b * Ho + yo
    const int Wi = 2 * Wo;
    const int64_t r0 = (2 * by) * Wi + 2 * xo;  // (b * Hi + 2 yo) * Wi + 2 xo
    float a[8], b1[8], c2[8], d[8], o[8];
    load8(in + r0 * in_cs + in_co + c, a);
    load8(in + (r0 + 1) * in_cs + in_co + c, b1);
    load8(in + (r0 + Wi) * in_cs + in_co + c, c2);
    load8(in + (r0 + Wi + 1) * in_cs + in_co + c, d);
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = 0.25f * ((a[e] + b1[e]) + (c2[e] + d[e]));
    store8(out + q * C + c, o);
}

// out[b][y][x][out_co + c] = in[b][y / 2][x / 2][c] (level l + 1 -> l).
template <typename T>
__global__ __launch_bounds__(kEw) void k_upsample(const T* __restrict__ in, int C, T* __restrict__ out,
                                                  int out_cs, int out_co, int Ho, int Wo, int B) {
    const int64_t i = (int64_t)blockIdx.x * kEw + threadIdx.x;
    const int C8 = C / 8;
    if (i >= (int64_t)B * Ho * Wo * C8) return;
    const int c = (int)(i % C8) * 8;
    const int64_t q = i / C8;
    const int xo = (int)(q % Wo);
    const int64_t by = q / Wo;
    const int64_t src = (by >> 1) * (Wo >> 1) + (xo >> 1);
    float v[8];
    load8(in + src * C + c, v);
    store8(out + q * out_cs + out_co + c, v);
}

// Adjoint of the upsampling, then the ReLU mask of the lower-level activation:
// out[q][c] = (sum over the 2x2 children of g[child][g_co + c]
//              + gmean[b][c] / (Hl Wl)) * (act[q][c] > 0),
// gmean (optional) the gradient of the sample's channel mean of act.
template <typename T>
__global__ __launch_bounds__(kEw) void k_upsample_back(const T* __restrict__ g, int g_cs, int g_co, int C,
                                                       const T* __restrict__ act, const float* __restrict__ gmean,
                                                       T* __restrict__ out, int Hl, int Wl, int B) {
    const int64_t i = (int64_t)blockIdx.x * kEw + threadIdx.x;
    const int C8 = C / 8;
    if (i >= (int64_t)B * Hl * Wl * C8) return;
    const int c = (int)(i % C8) * 8;
    const int64_t q = i / C8;
    const int xl = (int)(q % Wl);
    const int64_t by = q / Wl;
    const int Wh = 2 * Wl;
    const int64_t r0 = (2 * by) * Wh + 2 * xl;
    float a[8], b1[8], c2[8], d[8], m[8], o[8];
    load8(g + r0 * g_cs + g_co + c, a);
    load8(g + (r0 + 1) * g_cs + g_co + c, b1);
    load8(g + (r0 + Wh) * g_cs + g_co + c, c2);
    load8(g + (r0 + Wh + 1) * g_cs + g_co + c, d);
    load8(act + q * C + c, m);
    const int b = (int)(by / Hl);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        float v = (a[e] + b1[e]) + (c2[e] + d[e]);
        if (gmean) v += gmean[(int64_t)b * C + c + e] / (float)(Hl * Wl);
        o[e] = m[e] > 0.0f ? v : 0.0f;
    }
    store8(out + q * C + c, o);
}

// out[p][out_co + c] = m[b(p)][c] for every node p of a level with N nodes per sample.
template <typename T>
__global__ __launch_bounds__(kEw) void k_broadcast(const T* __restrict__ m, int C, T* __restrict__ out, int out_cs,
                                                   int out_co, int N, int B) {
    const int64_t i = (int64_t)blockIdx.x * kEw + threadIdx.x;
    const int C8 = C / 8;
    if (i >= (int64_t)B * N * C8) return;
    const int c = (int)(i % C8) * 8;
    const int64_t p = i / C8;
    float v[8];
    load8(m + (p / N) * C + c, v);
    store8(out + p * out_cs + out_co + c, v);
}

// Encoder skip: out[p][c] = (g_low[parent][c] / 4 + g_cat[p][skip_co + c]) *
// (act[p][act_co + c] > 0), act the skip activation (inside the concat buffer).
template <typename T>
__global__ __launch_bounds__(kEw) void k_pool_back_skip(const T* __restrict__ g_low, const T* __restrict__ g_cat,
                                                        int cat_cs, int skip_co, const T* __restrict__ act,
                                                        int C, T* __restrict__ out, int H, int W, int B) {
    const int64_t i = (int64_t)blockIdx.x * kEw + threadIdx.x;
    const int C8 = C / 8;
    if (i >= (int64_t)B * H * W * C8) return;
    const int c = (int)(i % C8) * 8;
    const int64_t p = i / C8;
    const int x = (int)(p % W);
    const int64_t by = p / W;
    const int64_t parent = (by >> 1) * (W >> 1) + (x >> 1);
    float lo[8], sk[8], ac[8], o[8];
    load8(g_low + parent * C + c, lo);
    load8(g_cat + p * cat_cs + skip_co + c, sk);
    load8(act + p * cat_cs + skip_co + c, ac);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float v = 0.25f * lo[e] + sk[e];
        o[e] = ac[e] > 0.0f ? v : 0.0f;
    }
    store8(out + p * C + c, o);
}

// ------------------------------------------------------------------ data
// Source node of output node (y, x) of sample b under the augmentation code
// aug[b] (optional): bits 0..15 shift x periodically by that many nodes, bit
// 16 mirrors y about the channel centre line (y -> H - 1 - y).  Both map a
// steady channel flow onto the steady flow of the transformed geometry (u_y
// changes sign under the mirror).
__device__ inline int64_t aug_source(const int* aug, int b, int s, int y, int x, int H, int W, bool& flip) {
    int shift = 0;
    flip = false;
    if (aug) {
        shift = aug[b] & 0xFFFF;
        flip = ((aug[b] >> 16) & 1) != 0;
    }
    const int ys = flip ? H - 1 - y : y;
    int xs = x - shift;
    xs = xs < 0 ? xs + W : xs;
    return ((int64_t)s * H + ys) * W + xs;
}

// Network input from a solid mask and Re: channel 0 = solid, 1 = Re / 100,
// channels 2..15 zero.  idx (optional) selects samples of a larger set.
template <typename T>
__global__ __launch_bounds__(kEw) void k_pack_input(const uint8_t* __restrict__ solid, const double* __restrict__ re,
                                                    const int* __restrict__ idx, const int* __restrict__ aug, int H,
                                                    int W, int B, T* __restrict__ x0) {
    const int HW = H * W;
    const int64_t p = (int64_t)blockIdx.x * kEw + threadIdx.x;
    if (p >= (int64_t)B * HW) return;
    const int b = (int)(p / HW);
    const int s = idx ? idx[b] : b;
    const int r = (int)(p - (int64_t)b * HW);
    bool flip;
    const int64_t src = aug_source(aug, b, s, r / W, r % W, H, W, flip);
    T* o = x0 + p * 16;
    o[0] = from_f<T>(solid[src] ? 1.0f : 0.0f);
    o[1] = from_f<T>((float)(re[s] / 100.0));
    for (int c = 2; c < 16; ++c) o[c] = from_f<T>(0.0f);
}

// Raw input [P][2] (float) into the padded input tensor.
template <typename T>
__global__ __launch_bounds__(kEw) void k_pack_raw(const float* __restrict__ xin, int64_t P, T* __restrict__ x0) {
    const int64_t p = (int64_t)blockIdx.x * kEw + threadIdx.x;
    if (p >= P) return;
    T* o = x0 + p * 16;
    o[0] = from_f<T>(xin[2 * p]);
    o[1] = from_f<T>(xin[2 * p + 1]);
    for (int c = 2; c < 16; ++c) o[c] = from_f<T>(0.0f);
}

// Centre-line speed of the unobstructed channel of sample s, g H^2 / (8 nu),
// nu = (tau - 1/2) / 3.
__device__ inline double u_centre(double gx, double tau, int ny) {
    const double nu = (tau - 0.5) / 3.0;
    return gx * (double)ny * (double)ny / (8.0 * nu);
}

// Normalised target and fluid flag of the selected samples:
// t = ((rho - 1) / (U_c s_rho), u_x / U_c, u_y / U_c).
__global__ __launch_bounds__(kEw) void k_pack_target(const uint8_t* __restrict__ solid, const float* __restrict__ rho,
                                                     const float* __restrict__ ux, const float* __restrict__ uy,
                                                     const double* __restrict__ gx, const double* __restrict__ tau,
                                                     const int* __restrict__ idx, const int* __restrict__ aug, int H,
                                                     int W, int B, double rho_scale, float* __restrict__ tgt,
                                                     uint8_t* __restrict__ fluid) {
    const int HW = H * W;
    const int64_t p = (int64_t)blockIdx.x * kEw + threadIdx.x;
    if (p >= (int64_t)B * HW) return;
    const int b = (int)(p / HW);
    const int s = idx ? idx[b] : b;
    const int r = (int)(p - (int64_t)b * HW);
    bool flip;
    const int64_t src = aug_source(aug, b, s, r / W, r % W, H, W, flip);
    const double uc = u_centre(gx[s], tau[s], H);
    const bool fl = solid[src] == 0;
    fluid[p] = fl ? 1 : 0;
    tgt[3 * p + 0] = fl ? (float)(((double)rho[src] - 1.0) / (uc * rho_scale)) : 0.0f;
    tgt[3 * p + 1] = fl ? (float)((double)ux[src] / uc) : 0.0f;
    tgt[3 * p + 2] = fl ? (float)((flip ? -1.0 : 1.0) * (double)uy[src] / uc) : 0.0f;
}

// Fields from the network output (inference): fluid nodes get
// rho = 1 + y0 U_c s_rho, u = (y1, y2) U_c; solid nodes 0.
__global__ __launch_bounds__(kEw) void k_unpack_fields(const float* __restrict__ y, const uint8_t* __restrict__ solid,
                                                       const double* __restrict__ gx, const double* __restrict__ tau,
                                                       int H, int W, int B, double rho_scale, float* __restrict__ rho,
                                                       float* __restrict__ ux, float* __restrict__ uy) {
    const int HW = H * W;
    const int64_t p = (int64_t)blockIdx.x * kEw + threadIdx.x;
    if (p >= (int64_t)B * HW) return;
    const int b = (int)(p / HW);
    const double uc = u_centre(gx[b], tau[b], H);
    const bool fl = solid[p] == 0;
    rho[p] = fl ? (float)(1.0 + (double)y[3 * p] * uc * rho_scale) : 0.0f;
    ux[p] = fl ? (float)((double)y[3 * p + 1] * uc) : 0.0f;
    uy[p] = fl ? (float)((double)y[3 * p + 2] * uc) : 0.0f;
}

// ------------------------------------------------------------------ warm-start projection
// Projection of a warm-start field of one channel (one workgroup per sample,
// fluid nodes only): rho shifted so that the mean density is rho0 (the mass
// of the cold start), u_x of column x scaled so that its flux
// J(x) = sum_y rho u_x equals the mean flux over the columns, u_y of row y
// shifted so that its flux K(y) = sum_x rho u_y is zero.  Equal column fluxes
// (continuity) give zero staggered momentum sum_x (-1)^x J(x) for even nx,
// zero row fluxes zero sum_y (-1)^y K(y): the start then excites no
// period-2 staggered mode, which no relaxation would damp.  Sums in double,
// in a fixed order.
constexpr int kProjMax = 2048;  // largest nx and ny of a projected field (LDS: 52 KB)

__global__ __launch_bounds__(kEw) void k_fill_i32(int* __restrict__ p, int64_t n, int v) {
    const int64_t q = (int64_t)blockIdx.x * kEw + threadIdx.x;
    if (q < n) p[q] = v;
}

// Start check of warm fields: workgroup k clears ok[k] when a fluid node of
// field set k has a density that is not finite or outside (0, 2 rho0), or a
// velocity that is not finite or of magnitude above u_max (the flag is set
// to 1 first by the host).
__global__ __launch_bounds__(kEw) void k_warm_check(const uint8_t* __restrict__ own,
                                                    const float* __restrict__ rho, const float* __restrict__ ux,
                                                    const float* __restrict__ uy, int nx, int ny, double rho0,
                                                    double u_max, int* __restrict__ ok) {
    const int k = blockIdx.x;
    const int64_t n = (int64_t)nx * ny, base = (int64_t)k * n;
    bool bad = false;
    for (int64_t q = threadIdx.x; q < n; q += kEw) {
        if (own[base + q] != 0) continue;
        const double r = rho[base + q], u = ux[base + q], v = uy[base + q];
        const double uu = u * u + v * v;
        // comparisons written so that NaN fails them
        if (!(r > 0.0 && r < 2.0 * rho0) || !(uu <= u_max * u_max)) bad = true;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) ok[k] = 0;
}

// a = (a + b) / 2 elementwise (the mean of the fields of two consecutive
// steps: modes that change sign every step cancel, slowly varying ones stay).
__global__ __launch_bounds__(kEw) void k_average(float* __restrict__ a, const float* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kEw + threadIdx.x;
    if (i < n) a[i] = 0.5f * (a[i] + b[i]);
}

__global__ __launch_bounds__(kEw) void k_project(const uint8_t* __restrict__ own, float* __restrict__ rho,
                                                 float* __restrict__ ux, float* __restrict__ uy, int nx, int ny,
                                                 double rho0) {
    __shared__ double colsum[kProjMax];
    __shared__ double rowsum[kProjMax];
    __shared__ double rowrho[kProjMax];
    __shared__ double red[2][kEw];
    const int64_t base = (int64_t)blockIdx.x * nx * ny;
    const uint8_t* o = own + base;
    float* r = rho + base;
    float* u = ux + base;
    float* v = uy + base;
    // mass
    double m = 0.0, nf = 0.0;
    for (int64_t i = threadIdx.x; i < (int64_t)nx * ny; i += kEw)
        if (o[i] == 0) {
            m += (double)r[i];
            nf += 1.0;
        }
    red[0][threadIdx.x] = m;
    red[1][threadIdx.x] = nf;
    __syncthreads();
    for (int off = kEw / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    const double shift = red[1][0] > 0.0 ? rho0 - red[0][0] / red[1][0] : 0.0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < (int64_t)nx * ny; i += kEw)
        if (o[i] == 0) r[i] = (float)((double)r[i] + shift);
    __syncthreads();
    // column fluxes of u_x, row fluxes of u_y
    for (int x = threadIdx.x; x < nx; x += kEw) {
        double j = 0.0;
        for (int y = 0; y < ny; ++y) {
            const int64_t i = (int64_t)y * nx + x;
            if (o[i] == 0) j += (double)r[i] * (double)u[i];
        }
        colsum[x] = j;
    }
    for (int y = threadIdx.x; y < ny; y += kEw) {
        double k = 0.0, rr = 0.0;
        for (int x = 0; x < nx; ++x) {
            const int64_t i = (int64_t)y * nx + x;
            if (o[i] == 0) {
                k += (double)r[i] * (double)v[i];
                rr += (double)r[i];
            }
        }
        rowsum[y] = k;
        rowrho[y] = rr;
    }
    __syncthreads();
    double jm = 0.0;
    for (int x = 0; x < nx; ++x) jm += colsum[x];
    jm /= (double)nx;
    for (int64_t i = threadIdx.x; i < (int64_t)nx * ny; i += kEw) {
        if (o[i] != 0) continue;
        const int y = (int)(i / nx), x = (int)(i - (int64_t)y * nx);
        if (colsum[x] != 0.0) u[i] = (float)((double)u[i] * (jm / colsum[x]));
        if (rowrho[y] > 0.0) v[i] = (float)((double)v[i] - rowsum[y] / rowrho[y]);
    }
}

// ------------------------------------------------------------------ loss
// Masked mean squared error over fluid nodes and 3 channels.  Stage 1: block
// partial sums {sum (y - t)^2, fluid count}; stage 2 (one thread) sums the
// blocks in order, then every node writes its gradient 2 (y - t) / (3 n_f)
// into the padded head-gradient tensor (channels 3..31 zero).
__global__ __launch_bounds__(kEw) void k_loss_partial(const float* __restrict__ y, const float* __restrict__ t,
                                                      const uint8_t* __restrict__ fluid, int64_t P,
                                                      double* __restrict__ part) {
    __shared__ double s1[kEw], s2[kEw];
    const int64_t p = (int64_t)blockIdx.x * kEw + threadIdx.x;
    double a = 0.0, c = 0.0;
    if (p < P && fluid[p]) {
        for (int k = 0; k < 3; ++k) {
            const double d = (double)y[3 * p + k] - (double)t[3 * p + k];
            a += d * d;
        }
        c = 1.0;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = c;
    __syncthreads();
    for (int off = kEw / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s1[threadIdx.x] += s1[threadIdx.x + off];
            s2[threadIdx.x] += s2[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

// One workgroup: thread t sums the partials [t K, (t + 1) K) in order, then a
// fixed tree combines the threads.
__global__ __launch_bounds__(kEw) void k_loss_final(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    __shared__ double s1[kEw], s2[kEw];
    const int K = (nblk + kEw - 1) / kEw;
    double a = 0.0, c = 0.0;
    for (int b = threadIdx.x * K; b < (threadIdx.x + 1) * K && b < nblk; ++b) {
        a += part[2 * b];
        c += part[2 * b + 1];
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = c;
    __syncthreads();
    for (int off = kEw / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s1[threadIdx.x] += s1[threadIdx.x + off];
            s2[threadIdx.x] += s2[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s2[0] > 0.0 ? s1[0] / (3.0 * s2[0]) : 0.0;
        out[1] = s2[0];
    }
}

template <typename T>
__global__ __launch_bounds__(kEw) void k_loss_grad(const float* __restrict__ y, const float* __restrict__ t,
                                                   const uint8_t* __restrict__ fluid, int64_t P,
                                                   const double* __restrict__ lossv, T* __restrict__ g_head) {
    const int64_t p = (int64_t)blockIdx.x * kEw + threadIdx.x;
    if (p >= P) return;
    const double nf = lossv[1];
    const double sc = nf > 0.0 ? 2.0 / (3.0 * nf) : 0.0;
    T* o = g_head + p * 32;
    for (int k = 0; k < 3; ++k)
        o[k] = from_f<T>(fluid[p] ? (float)(sc * ((double)y[3 * p + k] - (double)t[3 * p + k])) : 0.0f);
    for (int k = 3; k < 32; ++k) o[k] = from_f<T>(0.0f);
}

// Raw output gradient [P][3] (float) into the padded head-gradient tensor.
template <typename T>
__global__ __launch_bounds__(kEw) void k_pack_head_grad(const float* __restrict__ gy, int64_t P, T* __restrict__ g_head) {
    const int64_t p = (int64_t)blockIdx.x * kEw + threadIdx.x;
    if (p >= P) return;
    T* o = g_head + p * 32;
    for (int k = 0; k < 3; ++k) o[k] = from_f<T>(gy[3 * p + k]);
    for (int k = 3; k < 32; ++k) o[k] = from_f<T>(0.0f);
}

// ------------------------------------------------------------------ parameters
struct LayerDev {
    int64_t off;        // first weight in the master vector (bias follows the weights)
    int cin, cout;      // real channel counts
    int cin_pad, cout_pad;
    int64_t wf_off;     // forward weights T [cout_pad][9][cin_pad]
    int64_t wt_off;     // input-gradient weights T [cin_dg][9][cout_pad], flipped taps
    int cin_dg;         // rows of the input-gradient weights (cin rounded up to 32)
    int64_t b_off;      // padded bias [cout_pad]
};

// Master FP32 parameters -> forward weights, flipped/transposed weights and
// padded biases of layer L (one thread per padded element of the largest).
template <typename T>
__global__ __launch_bounds__(kEw) void k_pack_weights(const float* __restrict__ master, LayerDev L,
                                                      T* __restrict__ wf, T* __restrict__ wt,
                                                      float* __restrict__ bias) {
    const int64_t i = (int64_t)blockIdx.x * kEw + threadIdx.x;
    const int64_t nf = (int64_t)L.cout_pad * 9 * L.cin_pad;
    if (i < nf) {
        const int ci = (int)(i % L.cin_pad);
        const int64_t r = i / L.cin_pad;
        const int tap = (int)(r % 9);
        const int co = (int)(r / 9);
        const float v = (co < L.cout && ci < L.cin) ? master[L.off + ((int64_t)co * 9 + tap) * L.cin + ci] : 0.0f;
        wf[L.wf_off + i] = from_f<T>(v);
    }
    const int64_t nt = (int64_t)L.cin_dg * 9 * L.cout_pad;
    if (i < nt) {
        const int co = (int)(i % L.cout_pad);
        const int64_t r = i / L.cout_pad;
        const int tapf = (int)(r % 9);
        const int ci = (int)(r / 9);
        const int tap = 8 - tapf;  // (ky, kx) -> (2 - ky, 2 - kx)
        const float v = (co < L.cout && ci < L.cin) ? master[L.off + ((int64_t)co * 9 + tap) * L.cin + ci] : 0.0f;
        wt[L.wt_off + i] = from_f<T>(v);
    }
    if (i < L.cout_pad) bias[L.b_off + i] = i < L.cout ? master[L.off + (int64_t)L.cout * 9 * L.cin + i] : 0.0f;
}

// Adam (Kingma and Ba) on the FP32 master vector; t counts from 1.
__global__ __launch_bounds__(kEw) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * kEw + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(kEw) void k_zero_f32(float* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kEw + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

}  // namespace nn
