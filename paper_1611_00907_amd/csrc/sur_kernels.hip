// HIP kernels of the convolutional surrogate (encoder-decoder of 3x3 convolutions)
// for CDNA4: BF16 activations and weights, FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16), FP32 master weights and Adam.
//
// Activations are NHWC with a channel stride and offset per tensor view, so a
// convolution can read from or write into a slice of a concatenation buffer.
// Weights are [9][Cout_p][Cin_p] (tap-major, input channels contiguous, both
// padded with zeros: Cin_p to a multiple of 32, Cout_p to a multiple of 16).
//
// MFMA 16x16x32 operand layout: lane l supplies A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j = 0..7, and receives D[4 (l / 16) + i][l % 16],
// i = 0..3.  A convolution is the GEMM out[pixel][co] = sum_k in_col[pixel][k] W[k][co]
// with k = (tap, ci): A rows are pixels, B columns output channels.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sur_internal.h"

namespace cplbm {
namespace sur {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// float -> bfloat16 bits, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40);
    return uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// ---------------------------------------------------------------- convolution
// One wave computes WM x 16 pixels by WN x 16 output channels.
template <int WM, int WN>
__global__ __launch_bounds__(256) void conv3x3_kernel(ConvArgs a) {
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    const int co_tiles = a.cout_p / (16 * WN);
    const long long npx = (long long)a.N * a.H * a.W;
    const int co_tile = wave % co_tiles;
    const long long px0 = (long long)(wave / co_tiles) * (16 * WM);
    if (px0 >= npx) return;

    f32x4 acc[WM][WN];
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
        for (int n = 0; n < WN; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    // the pixel each lane feeds into A rows of block m
    int py[WM], pxx[WM];
    long long pn[WM];
    bool pvalid[WM];
#pragma unroll
    for (int m = 0; m < WM; ++m) {
        const long long p = px0 + 16 * m + r;
        pvalid[m] = p < npx;
        const long long q = pvalid[m] ? p : 0;
        pxx[m] = int(q % a.W);
        const long long t = q / a.W;
        py[m] = int(t % a.H);
        pn[m] = t / a.H;
    }
    const int co_base = co_tile * 16 * WN;
    for (int tap = 0; tap < 9; ++tap) {
        const int du = tap / 3 - 1, dv = tap % 3 - 1;
        long long src[WM];
        bool sval[WM];
#pragma unroll
        for (int m = 0; m < WM; ++m) {
            const int yy = py[m] + du, xx = pxx[m] + dv;
            sval[m] = pvalid[m] && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
            src[m] = ((pn[m] * a.H + yy) * a.W + xx) * a.in.cs + a.in.co;
        }
        for (int ci0 = 0; ci0 < a.cin_p; ci0 += 32) {
            const int ci = ci0 + 8 * g;
            const bool cin_ok = ci < a.cin;
            bf16x8 av[WM], bv[WN];
#pragma unroll
            for (int m = 0; m < WM; ++m) {
                uint4 v = make_uint4(0, 0, 0, 0);
                if (sval[m] && cin_ok) v = *reinterpret_cast<const uint4*>(a.in.p + src[m] + ci);
                av[m] = as_bf16x8(v);
            }
#pragma unroll
            for (int n = 0; n < WN; ++n) {
                const int co = co_base + 16 * n + r;
                const uint4 v = *reinterpret_cast<const uint4*>(a.w + ((size_t)(tap * a.cout_p + co) * a.cin_p + ci));
                bv[n] = as_bf16x8(v);
            }
#pragma unroll
            for (int m = 0; m < WM; ++m)
#pragma unroll
                for (int n = 0; n < WN; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv[n], acc[m][n], 0, 0, 0);
        }
    }

    // epilogue: lane holds pixels px0 + 16 m + 4 g + i, channel co_base + 16 n + r
#pragma unroll
    for (int n = 0; n < WN; ++n) {
        const int co = co_base + 16 * n + r;
        if (co >= a.cout) continue;
        const float b = (a.bias != nullptr) ? a.bias[co] : 0.0f;
#pragma unroll
        for (int m = 0; m < WM; ++m) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long p = px0 + 16 * m + 4 * g + i;
                if (p >= npx) continue;
                float v = acc[m][n][i] + b;
                switch (a.epi) {
                case EPI_RELU_BF16:
                    a.out.p[p * a.out.cs + a.out.co + co] = f2bf(v > 0.f ? v : 0.f);
                    break;
                case EPI_MASK_BF16: {
                    const float mk = bf2f(a.mask.p[p * a.mask.cs + a.mask.co + co]);
                    a.out.p[p * a.out.cs + a.out.co + co] = f2bf(mk > 0.f ? v : 0.f);
                    break;
                }
                case EPI_BF16:
                    a.out.p[p * a.out.cs + a.out.co + co] = f2bf(v);
                    break;
                default:  // EPI_F32
                    a.out_f32[p * a.out_f32_cs + co] = v;
                }
            }
        }
    }
}

// LDS-staged convolution: a workgroup of four waves computes a (4 RW) x 16 pixel tile of
// one image for CO_B output channels (32, 64 or 96), each wave RW pixel rows of 16 for all
// CO_B channels.  For each block of 32 input channels it stages the (4 RW + 2) x 18
// input halo and the 9 x CO_B x 32 weights in LDS; per tap a wave then reads CO_B / 16
// weight blocks and RW pixel blocks and issues RW x CO_B / 16 MFMAs (2 x 2 for RW = 2,
// CO_B = 32: one LDS read per MFMA; 4 x 4 for RW = 4, CO_B = 64: one per two).
// Convolution to one output channel with an FP32 output (the output layer), on the
// vector ALUs: a matrix-core block would be 1/16 full.  A workgroup stages a 16 x 16
// pixel tile with its one-pixel ring (32 input channels at a time, pixels padded to
// 40 channels so that the lanes' 16-byte reads of consecutive pixels fall in
// distinct LDS banks) and the block's 9 x 32 weights in FP32; each thread sums the
// 9 x 32 products of its pixel.  Needs input views whose strides and offsets are
// multiples of 8 channels.
constexpr int C1_T = 16, C1_HW = C1_T + 2, C1_PX = 40;
__global__ __launch_bounds__(256) void conv3x3_c1_kernel(ConvArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[C1_HW * C1_HW * C1_PX];
    __shared__ __attribute__((aligned(16))) float ws[9 * 32];
    const int tiles_x = (a.W + C1_T - 1) / C1_T, tiles_y = (a.H + C1_T - 1) / C1_T;
    int b = blockIdx.x;
    const int x0 = (b % tiles_x) * C1_T;
    b /= tiles_x;
    const int y0 = (b % tiles_y) * C1_T, img = b / tiles_y;
    const int lx = threadIdx.x % C1_T, ly = threadIdx.x / C1_T;
    float acc = 0.f;
    for (int ci0 = 0; ci0 < a.cin_p; ci0 += 32) {
        for (int q = threadIdx.x; q < C1_HW * C1_HW * 4; q += 256) {
            const int pix = q >> 2, cg = q & 3;
            const int yy = y0 - 1 + pix / C1_HW, xx = x0 - 1 + pix % C1_HW, ci = ci0 + 8 * cg;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W && ci < a.cin)
                v = *reinterpret_cast<const uint4*>(a.in.p + (((long long)img * a.H + yy) * a.W + xx) * a.in.cs +
                                                    a.in.co + ci);
            *reinterpret_cast<uint4*>(xs + pix * C1_PX + 8 * cg) = v;
        }
        for (int q = threadIdx.x; q < 9 * 32; q += 256) {
            const int tap = q >> 5, ci = ci0 + (q & 31);
            ws[q] = ci < a.cin ? bf2f(a.w[(size_t)tap * a.cout_p * a.cin_p + ci]) : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const uint16_t* px = xs + ((ly + tap / 3) * C1_HW + (lx + tap % 3)) * C1_PX;
            const float* w = ws + 32 * tap;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint4 v = *reinterpret_cast<const uint4*>(px + 8 * k);
                const float4 w0 = *reinterpret_cast<const float4*>(w + 8 * k);
                const float4 w1 = *reinterpret_cast<const float4*>(w + 8 * k + 4);
                acc = fmaf(w0.x, __uint_as_float(v.x << 16), acc);
                acc = fmaf(w0.y, __uint_as_float(v.x & 0xffff0000u), acc);
                acc = fmaf(w0.z, __uint_as_float(v.y << 16), acc);
                acc = fmaf(w0.w, __uint_as_float(v.y & 0xffff0000u), acc);
                acc = fmaf(w1.x, __uint_as_float(v.z << 16), acc);
                acc = fmaf(w1.y, __uint_as_float(v.z & 0xffff0000u), acc);
                acc = fmaf(w1.z, __uint_as_float(v.w << 16), acc);
                acc = fmaf(w1.w, __uint_as_float(v.w & 0xffff0000u), acc);
            }
        }
        __syncthreads();  // the next block overwrites the LDS
    }
    const int x = x0 + lx, y = y0 + ly;
    if (x < a.W && y < a.H)
        a.out_f32[(((long long)img * a.H + y) * a.W + x) * a.out_f32_cs] = acc + (a.bias != nullptr ? a.bias[0] : 0.f);
}

// Convolution from one input channel to at most 32 (the output layer's input
// gradient: dX = the flipped convolution of its one-channel output gradient, masked
// by the ReLU of its input), on the vector ALUs: a 16 x 16 pixel tile of the input
// channel with its ring and the 9 x 32 weights in LDS, each thread the 32 outputs of
// one pixel, staged in LDS and stored as BF16 in 16-byte pieces of 8 channels with
// the mask applied as in the matrix-core kernels (a BF16 output whose mask value is
// not > 0 is zeroed).
__global__ __launch_bounds__(256) void conv3x3_from1_kernel(ConvArgs a) {
    __shared__ float zs[C1_HW * C1_HW];
    __shared__ __attribute__((aligned(16))) float ws[9 * 32];
    const int tiles_x = (a.W + C1_T - 1) / C1_T, tiles_y = (a.H + C1_T - 1) / C1_T;
    int b = blockIdx.x;
    const int x0 = (b % tiles_x) * C1_T;
    b /= tiles_x;
    const int y0 = (b % tiles_y) * C1_T, img = b / tiles_y;
    const int lx = threadIdx.x % C1_T, ly = threadIdx.x / C1_T;
    for (int q = threadIdx.x; q < C1_HW * C1_HW; q += 256) {
        const int yy = y0 - 1 + q / C1_HW, xx = x0 - 1 + q % C1_HW;
        zs[q] = (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
                    ? bf2f(a.in.p[(((long long)img * a.H + yy) * a.W + xx) * a.in.cs + a.in.co])
                    : 0.f;
    }
    for (int q = threadIdx.x; q < 9 * 32; q += 256) {
        const int tap = q >> 5, co = q & 31;
        ws[q] = co < a.cout ? bf2f(a.w[((size_t)tap * a.cout_p + co) * a.cin_p]) : 0.f;
    }
    __syncthreads();
    float acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = 0.f;
    // one tap at a time (unrolled, the compiler would hold all 288 weights in registers)
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
        const float z = zs[(ly + tap / 3) * C1_HW + lx + tap % 3];
#pragma unroll
        for (int c4 = 0; c4 < 8; ++c4) {
            const float4 w = *reinterpret_cast<const float4*>(ws + 32 * tap + 4 * c4);
            acc[4 * c4] = fmaf(w.x, z, acc[4 * c4]);
            acc[4 * c4 + 1] = fmaf(w.y, z, acc[4 * c4 + 1]);
            acc[4 * c4 + 2] = fmaf(w.z, z, acc[4 * c4 + 2]);
            acc[4 * c4 + 3] = fmaf(w.w, z, acc[4 * c4 + 3]);
        }
    }
    // the tile's outputs through LDS (pixels padded to 40 channels against bank
    // conflicts), then stored pixel-major in 16-byte pieces with the mask applied
    __shared__ __attribute__((aligned(16))) uint16_t os[C1_T * C1_T * C1_PX];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        uint32_t d[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            d[k] = uint32_t(f2bf(acc[8 * g + 2 * k])) | (uint32_t(f2bf(acc[8 * g + 2 * k + 1])) << 16);
        *reinterpret_cast<uint4*>(os + threadIdx.x * C1_PX + 8 * g) = make_uint4(d[0], d[1], d[2], d[3]);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < C1_T * C1_T * 4; q += 256) {
        const int pl = q >> 2, g = q & 3;
        const int x = x0 + pl % C1_T, y = y0 + pl / C1_T;
        if (x >= a.W || y >= a.H || 8 * g >= a.cout) continue;
        const long long p = ((long long)img * a.H + y) * a.W + x;
        uint4 v = *reinterpret_cast<const uint4*>(os + pl * C1_PX + 8 * g);
        if (a.epi == EPI_MASK_BF16) {
            const uint4 mk = *reinterpret_cast<const uint4*>(a.mask.p + p * a.mask.cs + a.mask.co + 8 * g);
            auto keep = [](uint32_t w, uint32_t m) {
                const uint32_t lo = bf2f(uint16_t(m)) > 0.f ? 0x0000ffffu : 0u;
                const uint32_t hi = bf2f(uint16_t(m >> 16)) > 0.f ? 0xffff0000u : 0u;
                return w & (lo | hi);
            };
            v.x = keep(v.x, mk.x);
            v.y = keep(v.y, mk.y);
            v.z = keep(v.z, mk.z);
            v.w = keep(v.w, mk.w);
        }
        *reinterpret_cast<uint4*>(a.out.p + p * a.out.cs + a.out.co + 8 * g) = v;
    }
}

constexpr int LT_W = 16;
template <int RW, int CO_B>
struct LdsConv {
    static constexpr int TH = 4 * RW;                      // tile rows
    static constexpr int XIN = (TH + 2) * (LT_W + 2) * 32;  // halo elements
    static constexpr int WSH = 9 * CO_B * 32;               // weight elements
    static constexpr int NB = CO_B / 16;                    // 16-channel blocks per wave
};

// The forward pass's 2 x 2 average of a BF16 output tile staged in LDS as [TH x LT_W
// pixels][CO_B channels] (tile origin and map sides even): its four terms are added in
// the order of the pooling kernel, so that the pooled map is the same bit for bit.
template <int TH, int CO_B>
__device__ __forceinline__ void pool_tile(const ConvArgs& a, const uint16_t* ost, int img, int y0, int x0,
                                          int co_base) {
    static_assert(TH % 2 == 0 && LT_W % 2 == 0, "pooled tiles need even sides");
    for (int q = threadIdx.x; q < (TH / 2) * (LT_W / 2) * (CO_B / 8); q += blockDim.x) {
        const int pp = q / (CO_B / 8), cg = q % (CO_B / 8);
        const int py = pp / (LT_W / 2), px = pp % (LT_W / 2);
        const int y = y0 + 2 * py, x = x0 + 2 * px, co = co_base + 8 * cg;
        if (y >= a.H || x >= a.W || co >= a.cout) continue;
        float sum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const uint4 v =
                    *reinterpret_cast<const uint4*>(ost + ((2 * py + dy) * LT_W + 2 * px + dx) * CO_B + 8 * cg);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    sum[2 * k] += bf2f(uint16_t(w[k]));
                    sum[2 * k + 1] += bf2f(uint16_t(w[k] >> 16));
                }
            }
        uint32_t o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            o[k] = uint32_t(f2bf(0.25f * sum[2 * k])) | (uint32_t(f2bf(0.25f * sum[2 * k + 1])) << 16);
        const long long pq = ((long long)img * (a.H / 2) + y / 2) * (a.W / 2) + x / 2;
        *reinterpret_cast<uint4*>(a.pool.p + pq * a.pool.cs + a.pool.co + co) = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

// The decoder's upsampled copy of a BF16 output tile staged in LDS: each pixel's
// channels repeated over its 2 x 2 block of the map at twice the size.
template <int TH, int CO_B>
__device__ __forceinline__ void upsample_tile(const ConvArgs& a, const uint16_t* ost, int img, int y0, int x0,
                                              int co_base) {
    const int H2 = 2 * a.H, W2 = 2 * a.W;
    for (int q = threadIdx.x; q < TH * LT_W * 4 * (CO_B / 8); q += blockDim.x) {
        const int cg = q % (CO_B / 8), rest = q / (CO_B / 8);
        const int d = rest & 3, pl = rest >> 2;
        const int y = y0 + pl / LT_W, x = x0 + pl % LT_W, co = co_base + 8 * cg;
        if (y >= a.H || x >= a.W || co >= a.cout) continue;
        const uint4 v = *reinterpret_cast<const uint4*>(ost + pl * CO_B + 8 * cg);
        const long long pu = ((long long)img * H2 + 2 * y + (d >> 1)) * W2 + 2 * x + (d & 1);
        *reinterpret_cast<uint4*>(a.up.p + pu * a.up.cs + a.up.co + co) = v;
    }
}

// The upsampling gradient from one 16-channel half of an FP32 output tile staged in
// LDS as [TH x LT_W pixels][16] (no bias; output channels co0 ..): sums over 2 x 2
// pixel blocks, their terms in the order of the separate kernel, zeroed where the
// upsampled activation is not > 0, rounded to BF16 at half size.
template <int TH>
__device__ __forceinline__ void fold_half(const ConvArgs& a, const float* of, int img, int y0, int x0, int co0) {
    static_assert(TH % 2 == 0 && LT_W % 2 == 0, "folded tiles need even sides");
    for (int q = threadIdx.x; q < (TH / 2) * (LT_W / 2) * 4; q += blockDim.x) {
        const int pp = q >> 2, c4 = q & 3;
        const int py = pp / (LT_W / 2), px = pp % (LT_W / 2);
        const int y = y0 + 2 * py, x = x0 + 2 * px, co = co0 + 4 * c4;
        if (y >= a.H || x >= a.W || co >= a.cout) continue;
        float sum[4] = {0.f, 0.f, 0.f, 0.f};
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const float4 v =
                    *reinterpret_cast<const float4*>(of + ((2 * py + dy) * LT_W + 2 * px + dx) * 16 + 4 * c4);
                sum[0] += v.x;
                sum[1] += v.y;
                sum[2] += v.z;
                sum[3] += v.w;
            }
        const long long pq = ((long long)img * (a.H / 2) + y / 2) * (a.W / 2) + x / 2;
        const uint2 mk = *reinterpret_cast<const uint2*>(a.fold_act.p + pq * a.fold_act.cs + a.fold_act.co + co);
        const uint32_t mw[2] = {mk.x, mk.y};
        uint32_t o[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const float lo = bf2f(uint16_t(mw[k])) > 0.f ? sum[2 * k] : 0.f;
            const float hi = bf2f(uint16_t(mw[k] >> 16)) > 0.f ? sum[2 * k + 1] : 0.f;
            o[k] = uint32_t(f2bf(lo)) | (uint32_t(f2bf(hi)) << 16);
        }
        *reinterpret_cast<uint2*>(a.fold.p + pq * a.fold.cs + a.fold.co + co) = make_uint2(o[0], o[1]);
    }
}

template <int RW, int CO_B>
__global__ __launch_bounds__(256) void conv3x3_lds_kernel(ConvArgs a) {
    using K = LdsConv<RW, CO_B>;
    constexpr int TH = K::TH, NB = K::NB;
    __shared__ __attribute__((aligned(16))) uint16_t lds[K::XIN + K::WSH];
    uint16_t* xin = lds;
    uint16_t* wsh = lds + K::XIN;
    const int co_blocks = a.cout_p / CO_B;
    const int tiles_x = (a.W + LT_W - 1) / LT_W, tiles_y = (a.H + TH - 1) / TH;
    int b = blockIdx.x;
    const int co_blk = b % co_blocks;
    b /= co_blocks;
    const int tx = b % tiles_x;
    b /= tiles_x;
    const int ty = b % tiles_y;
    const int img = b / tiles_y;
    const int x0 = tx * LT_W, y0 = ty * TH, co_base = co_blk * CO_B;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;

    f32x4 acc[RW][NB];
#pragma unroll
    for (int m = 0; m < RW; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int ci0 = 0; ci0 < a.cin_p; ci0 += 32) {
        // input halo: (TH + 2) x (LT_W + 2) pixels x 32 channels, zero outside the
        // image and beyond cin; 8 channels (16 bytes) per load
        for (int q = threadIdx.x; q < (TH + 2) * (LT_W + 2) * 4; q += 256) {
            const int pix = q >> 2, cg = q & 3;
            const int yy = y0 - 1 + pix / (LT_W + 2), xx = x0 - 1 + pix % (LT_W + 2);
            const int ci = ci0 + 8 * cg;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W && ci < a.cin)
                v = *reinterpret_cast<const uint4*>(a.in.p + (((long long)img * a.H + yy) * a.W + xx) * a.in.cs +
                                                    a.in.co + ci);
            *reinterpret_cast<uint4*>(xin + pix * 32 + 8 * cg) = v;
        }
        // weights of this block: [tap][CO_B output channels][32 input channels]
        for (int q = threadIdx.x; q < 9 * CO_B * 4; q += 256) {
            const int row = q >> 2, cg = q & 3;
            const int tap = row / CO_B, col = row - tap * CO_B;
            *reinterpret_cast<uint4*>(wsh + row * 32 + 8 * cg) = *reinterpret_cast<const uint4*>(
                a.w + ((size_t)(tap * a.cout_p + co_base + col) * a.cin_p + ci0 + 8 * cg));
        }
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int du = tap / 3 - 1, dv = tap % 3 - 1;
            bf16x8 bv[NB];
#pragma unroll
            for (int n = 0; n < NB; ++n)
                bv[n] = as_bf16x8(*reinterpret_cast<const uint4*>(wsh + (tap * CO_B + 16 * n + r) * 32 + 8 * g));
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int ly = RW * wave + m + 1 + du, lx = r + 1 + dv;
                const bf16x8 av = as_bf16x8(*reinterpret_cast<const uint4*>(xin + (ly * (LT_W + 2) + lx) * 32 + 8 * g));
#pragma unroll
                for (int n = 0; n < NB; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[n], acc[m][n], 0, 0, 0);
            }
        }
        __syncthreads();  // the next block of channels overwrites the LDS
    }

    // BF16 epilogues: bias and ReLU in registers, the TH x 16 x CO_B tile through LDS
    // (free after the last barrier), then 16-byte stores of 8 channels (the mask of
    // EPI_MASK_BF16 read 16 bytes at a time as well)
    if (a.epi != EPI_F32) {
        static_assert(TH * LT_W * CO_B <= K::XIN + K::WSH, "the output tile fits the staging space");
        uint16_t* ost = lds;  // [TH * LT_W pixels][CO_B channels]
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int cl = 16 * n + r, co = co_base + cl;
            const float bias = (a.bias != nullptr && co < a.cout) ? a.bias[co] : 0.0f;
#pragma unroll
            for (int m = 0; m < RW; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float v = acc[m][n][i] + bias;
                    if (a.epi == EPI_RELU_BF16) v = v > 0.f ? v : 0.f;
                    ost[((RW * wave + m) * LT_W + 4 * g + i) * CO_B + cl] = f2bf(v);
                }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < TH * LT_W * (CO_B / 8); q += 256) {
            const int pl = q / (CO_B / 8), cg = q % (CO_B / 8);
            const int y = y0 + pl / LT_W, x = x0 + pl % LT_W, co = co_base + 8 * cg;
            if (y >= a.H || x >= a.W || co >= a.cout) continue;
            const long long p = ((long long)img * a.H + y) * a.W + x;
            uint4 v = *reinterpret_cast<const uint4*>(ost + pl * CO_B + 8 * cg);
            if (a.epi == EPI_MASK_BF16) {
                const uint4 mk = *reinterpret_cast<const uint4*>(a.mask.p + p * a.mask.cs + a.mask.co + co);
                auto keep = [](uint32_t w, uint32_t m) {  // zero each BF16 half whose mask is not > 0
                    const uint32_t lo = bf2f(uint16_t(m)) > 0.f ? 0x0000ffffu : 0u;
                    const uint32_t hi = bf2f(uint16_t(m >> 16)) > 0.f ? 0xffff0000u : 0u;
                    return w & (lo | hi);
                };
                v.x = keep(v.x, mk.x);
                v.y = keep(v.y, mk.y);
                v.z = keep(v.z, mk.z);
                v.w = keep(v.w, mk.w);
            }
            *reinterpret_cast<uint4*>(a.out.p + p * a.out.cs + a.out.co + co) = v;
        }
        if (a.pool.p != nullptr) pool_tile<TH, CO_B>(a, ost, img, y0, x0, co_base);
        if (a.up.p != nullptr) upsample_tile<TH, CO_B>(a, ost, img, y0, x0, co_base);
        return;
    }

    // FP32 epilogue: 16 channels at a time through the LDS (free after the last
    // barrier), then out as 16-byte vectors of 4 channels
    static_assert(TH * LT_W * 16 * 2 <= K::XIN + K::WSH, "16 FP32 channels of the tile fit the staging space");
    float* of = reinterpret_cast<float*>(lds);
    const bool vec = (a.out_f32_cs & 3) == 0;
    // channels folded into the upsampling gradient are not stored themselves
    const bool fold = a.fold.p != nullptr && co_base + CO_B <= a.fold_c;
#pragma unroll
    for (int n = 0; n < NB; ++n) {
        if (n > 0) __syncthreads();  // the previous half is stored
        // lane holds pixels (RW wave + m, 4 g + i) of the tile, channel 16 n + r
#pragma unroll
        for (int m = 0; m < RW; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) of[((RW * wave + m) * LT_W + 4 * g + i) * 16 + r] = acc[m][n][i];
        __syncthreads();
        if (fold) fold_half<TH>(a, of, img, y0, x0, co_base + 16 * n);
        for (int q = threadIdx.x; q < (fold ? 0 : TH * LT_W * 4); q += 256) {
            const int pl = q >> 2, c4 = q & 3;
            const int y = y0 + pl / LT_W, x = x0 + pl % LT_W, co = co_base + 16 * n + 4 * c4;
            if (y >= a.H || x >= a.W || co >= a.cout) continue;
            float4 v = *reinterpret_cast<const float4*>(of + pl * 16 + 4 * c4);
            if (a.bias != nullptr) {
                v.x += a.bias[co];
                if (co + 1 < a.cout) v.y += a.bias[co + 1];
                if (co + 2 < a.cout) v.z += a.bias[co + 2];
                if (co + 3 < a.cout) v.w += a.bias[co + 3];
            }
            float* dst = a.out_f32 + (((long long)img * a.H + y) * a.W + x) * a.out_f32_cs + co;
            if (vec && co + 3 < a.cout) {
                *reinterpret_cast<float4*>(dst) = v;
            } else {
                const float e[4] = {v.x, v.y, v.z, v.w};
                for (int k = 0; k < 4 && co + k < a.cout; ++k) dst[k] = e[k];
            }
        }
    }
}

// The same convolution with a workgroup walking a run of pixel tiles, each tile in
// steps of one 32-channel input block: the next step's input halo (and, with more
// than one block, its weights) is loaded into registers while the current step's
// MFMAs run, the weights of a single block are staged once for the run, and the
// output tile goes out through an LDS area of its own, so that the load, MFMA and
// store phases of consecutive steps overlap.  The 256^2 layers are close to
// memory-bound, and the one-tile workgroups left these phases back to back.
template <int RW, int CO_B>
__global__ __launch_bounds__(256) void conv3x3_lds_run_kernel(ConvArgs a, int tiles_per_run) {
    using K = LdsConv<RW, CO_B>;
    constexpr int TH = K::TH, NB = K::NB;
    constexpr int HALO = (TH + 2) * (LT_W + 2) * 4;  // 16-byte pieces of the input halo
    constexpr int HR = (HALO + 255) / 256;            // per thread
    constexpr int OST = TH * LT_W * CO_B;
    static_assert(CO_B >= 32, "the FP32 output stages 16 channels per pixel in the output area");
    __shared__ __attribute__((aligned(16))) uint16_t lds[K::XIN + K::WSH + OST];
    uint16_t* xin = lds;
    uint16_t* wsh = lds + K::XIN;
    uint16_t* ost = lds + K::XIN + K::WSH;
    const int co_blocks = a.cout_p / CO_B;
    const int tiles_x = (a.W + LT_W - 1) / LT_W, tiles_y = (a.H + TH - 1) / TH;
    const int tiles = a.N * tiles_y * tiles_x;
    const int co_blk = blockIdx.x % co_blocks, co_base = co_blk * CO_B;
    const int t_begin = (blockIdx.x / co_blocks) * tiles_per_run;
    if (t_begin >= tiles) return;  // the whole workgroup
    const int t_end = min(t_begin + tiles_per_run, tiles);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;

    // The run is a sequence of steps (tile, input-channel block of 32); a tile's
    // accumulators carry over its blocks.  Weights of a block: [tap][CO_B output
    // channels][32 input channels]; with one block they are staged once for the run,
    // with several each step stages its block's weights, prefetched like the halo.
    const int ncb = a.cin_p / 32;
    constexpr int WPC = 9 * CO_B * 4;             // 16-byte pieces of one block's weights
    constexpr int WR = (WPC + 255) / 256;         // per thread
    auto load_w = [&](int cb, uint4* wr) {
#pragma unroll
        for (int k = 0; k < WR; ++k) {
            const int q = threadIdx.x + 256 * k;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (q < WPC) {
                const int row = q >> 2, cg = q & 3;
                const int tap = row / CO_B, col = row - tap * CO_B;
                v = *reinterpret_cast<const uint4*>(a.w + ((size_t)(tap * a.cout_p + co_base + col) * a.cin_p +
                                                           32 * cb + 8 * cg));
            }
            wr[k] = v;
        }
    };
    auto store_w = [&](const uint4* wr) {
#pragma unroll
        for (int k = 0; k < WR; ++k) {
            const int q = threadIdx.x + 256 * k;
            if (q < WPC) *reinterpret_cast<uint4*>(wsh + (q >> 2) * 32 + 8 * (q & 3)) = wr[k];
        }
    };
    uint4 wr[WR];
    load_w(0, wr);
    if (ncb == 1) store_w(wr);
    auto tile_origin = [&](int t, int& img, int& y0, int& x0) {
        img = t / (tiles_y * tiles_x);
        const int tt = t - img * tiles_y * tiles_x;
        y0 = (tt / tiles_x) * TH;
        x0 = (tt % tiles_x) * LT_W;
    };
    // halo piece q of a tile: pixel q / 4 of the (TH + 2) x (LT_W + 2) halo, channels
    // 32 cb + 8 (q % 4) ..
    auto load_halo = [&](int t, int cb, uint4* hr) {
        int img, y0, x0;
        tile_origin(t, img, y0, x0);
#pragma unroll
        for (int k = 0; k < HR; ++k) {
            const int q = threadIdx.x + 256 * k;
            const int pix = q >> 2, cg = q & 3;
            const int yy = y0 - 1 + pix / (LT_W + 2), xx = x0 - 1 + pix % (LT_W + 2);
            const int ci = 32 * cb + 8 * cg;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (q < HALO && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W && ci < a.cin)
                v = *reinterpret_cast<const uint4*>(a.in.p + (((long long)img * a.H + yy) * a.W + xx) * a.in.cs +
                                                    a.in.co + ci);
            hr[k] = v;
        }
    };
    uint4 hr[HR];
    load_halo(t_begin, 0, hr);
    f32x4 acc[RW][NB];
    for (int st = 0, st_end = (t_end - t_begin) * ncb; st < st_end; ++st) {
        const int t = t_begin + st / ncb, cb = st % ncb;
#pragma unroll
        for (int k = 0; k < HR; ++k) {
            const int q = threadIdx.x + 256 * k;
            if (q < HALO) *reinterpret_cast<uint4*>(xin + (q >> 2) * 32 + 8 * (q & 3)) = hr[k];
        }
        if (ncb > 1) store_w(wr);
        __syncthreads();  // halo and weights in place; the last tile's output stored
        if (st + 1 < st_end) {  // in flight during the MFMAs
            load_halo(t_begin + (st + 1) / ncb, (st + 1) % ncb, hr);
            if (ncb > 1) load_w((st + 1) % ncb, wr);
        }
        if (cb == 0) {
#pragma unroll
            for (int m = 0; m < RW; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int du = tap / 3 - 1, dv = tap % 3 - 1;
            bf16x8 bv[NB];
#pragma unroll
            for (int n = 0; n < NB; ++n)
                bv[n] = as_bf16x8(*reinterpret_cast<const uint4*>(wsh + (tap * CO_B + 16 * n + r) * 32 + 8 * g));
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int ly = RW * wave + m + 1 + du, lx = r + 1 + dv;
                const bf16x8 av = as_bf16x8(*reinterpret_cast<const uint4*>(xin + (ly * (LT_W + 2) + lx) * 32 + 8 * g));
#pragma unroll
                for (int n = 0; n < NB; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[n], acc[m][n], 0, 0, 0);
            }
        }
        if (cb + 1 < ncb) {  // the tile's next channel block
            __syncthreads();    // every wave is done with this block's halo and weights
            continue;
        }
        int img, y0, x0;
        tile_origin(t, img, y0, x0);
        if (a.epi == EPI_F32) {
            // FP32 output, 16 channels at a time through the output area (which holds
            // TH x LT_W x 16 floats), then out as 16-byte vectors: pixel-major rows of
            // 64 bytes instead of one float per lane and store
            float* of = reinterpret_cast<float*>(ost);
            const bool vec = (a.out_f32_cs & 3) == 0;
            // channels folded into the upsampling gradient are not stored themselves
            const bool fold = a.fold.p != nullptr && co_base + CO_B <= a.fold_c;
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                // lane holds pixels (RW wave + m, 4 g + i) of the tile, channel 16 n + r
#pragma unroll
                for (int m = 0; m < RW; ++m)
#pragma unroll
                    for (int i = 0; i < 4; ++i) of[((RW * wave + m) * LT_W + 4 * g + i) * 16 + r] = acc[m][n][i];
                __syncthreads();  // this half is in place (and every wave is done with the halo)
                for (int q = threadIdx.x; q < (fold ? 0 : TH * LT_W * 4); q += 256) {
                    const int pl = q >> 2, c4 = q & 3;
                    const int y = y0 + pl / LT_W, x = x0 + pl % LT_W, co = co_base + 16 * n + 4 * c4;
                    if (y >= a.H || x >= a.W || co >= a.cout) continue;
                    float4 v = *reinterpret_cast<const float4*>(of + pl * 16 + 4 * c4);
                    if (a.bias != nullptr) {
                        v.x += a.bias[co];
                        if (co + 1 < a.cout) v.y += a.bias[co + 1];
                        if (co + 2 < a.cout) v.z += a.bias[co + 2];
                        if (co + 3 < a.cout) v.w += a.bias[co + 3];
                    }
                    float* dst = a.out_f32 + (((long long)img * a.H + y) * a.W + x) * a.out_f32_cs + co;
                    if (vec && co + 3 < a.cout) {
                        *reinterpret_cast<float4*>(dst) = v;
                    } else {
                        const float e[4] = {v.x, v.y, v.z, v.w};
                        for (int k = 0; k < 4 && co + k < a.cout; ++k) dst[k] = e[k];
                    }
                }
                if (fold) fold_half<TH>(a, of, img, y0, x0, co_base + 16 * n);
                __syncthreads();  // the area is free for the next half (or the next tile's halo)
            }
            continue;
        }
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int cl = 16 * n + r, co = co_base + cl;
            const float bias = (a.bias != nullptr && co < a.cout) ? a.bias[co] : 0.0f;
#pragma unroll
            for (int m = 0; m < RW; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float v = acc[m][n][i] + bias;
                    if (a.epi == EPI_RELU_BF16) v = v > 0.f ? v : 0.f;
                    ost[((RW * wave + m) * LT_W + 4 * g + i) * CO_B + cl] = f2bf(v);
                }
        }
        __syncthreads();  // the output tile is in LDS; every wave is done with the halo
        for (int q = threadIdx.x; q < TH * LT_W * (CO_B / 8); q += 256) {
            const int pl = q / (CO_B / 8), cg = q % (CO_B / 8);
            const int y = y0 + pl / LT_W, x = x0 + pl % LT_W, co = co_base + 8 * cg;
            if (y >= a.H || x >= a.W || co >= a.cout) continue;
            const long long p = ((long long)img * a.H + y) * a.W + x;
            uint4 v = *reinterpret_cast<const uint4*>(ost + pl * CO_B + 8 * cg);
            if (a.epi == EPI_MASK_BF16) {
                const uint4 mk = *reinterpret_cast<const uint4*>(a.mask.p + p * a.mask.cs + a.mask.co + co);
                auto keep = [](uint32_t w, uint32_t mm) {  // zero each BF16 half whose mask is not > 0
                    const uint32_t lo = bf2f(uint16_t(mm)) > 0.f ? 0x0000ffffu : 0u;
                    const uint32_t hi = bf2f(uint16_t(mm >> 16)) > 0.f ? 0xffff0000u : 0u;
                    return w & (lo | hi);
                };
                v.x = keep(v.x, mk.x);
                v.y = keep(v.y, mk.y);
                v.z = keep(v.z, mk.z);
                v.w = keep(v.w, mk.w);
            }
            *reinterpret_cast<uint4*>(a.out.p + p * a.out.cs + a.out.co + co) = v;
        }
        if (a.pool.p != nullptr) pool_tile<TH, CO_B>(a, ost, img, y0, x0, co_base);
        if (a.up.p != nullptr) upsample_tile<TH, CO_B>(a, ost, img, y0, x0, co_base);
    }
}

// ---------------------------------------------------------------- weight gradient
// dW[tap][co][ci] += sum_p dZ[p][co] X[p shifted by tap][ci]: GEMM with the pixels as
// the reduction axis.  A = dZ^T (rows co), B = shifted X (columns ci); the operands
// are gathered 8 pixels at a time.  Each wave owns one tap, a (16 WM) x (16 WN)
// block of (co, ci) and a chunk of pixels, and adds its partial block to dW
// atomically; every gathered operand feeds WN (A) or WM (B) MFMAs.  A lane's pixel
// coordinates come from one division per 32 pixels and then by increments; inside
// the image, the tap's source pixel is p + du W + dv.  The waves of the centre tap
// and the first ci block also sum dZ for the bias gradient db[co] = sum_p dZ[p][co].
template <int WM, int WN, bool PA, bool PB>
__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(WgradArgs a) {
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    const int co_blocks = (a.cout + 16 * WM - 1) / (16 * WM), ci_blocks = (a.cin + 16 * WN - 1) / (16 * WN);
    const int tiles = 9 * co_blocks * ci_blocks;
    const int tile = wave % tiles;
    const int chunk = wave / tiles;
    const int npx = a.N * a.H * a.W;  // the host keeps pixel indices below 2^31
    const int cpx = int(a.chunk_px);
    const int p_begin = chunk * cpx;
    if (p_begin >= npx) return;
    const int p_end = p_begin < npx - cpx ? p_begin + cpx : npx;
    const int tap = tile % 9;
    const int co_t = (tile / 9) % co_blocks, ci_t = tile / 9 / co_blocks;
    const int du = tap / 3 - 1, dv = tap % 3 - 1;
    const int shift = du * a.W + dv;
    int co_a[WM], ci_b[WN];  // A rows / B columns of this lane
    bool co_ok[WM], ci_ok[WN];
    // PA / PB (2 tiles along that side; even channel count, stride and offset): tile
    // m (n) holds the channels of parity m (n), so one 32-bit load brings a lane both
    // of its channels of dZ (of X).
    static_assert((!PA || WM == 2) && (!PB || WN == 2), "channel pairs need 2 tiles along that side");
#pragma unroll
    for (int m = 0; m < WM; ++m) {
        co_a[m] = PA ? co_t * 32 + 2 * r + m : co_t * 16 * WM + 16 * m + r;
        co_ok[m] = co_a[m] < a.cout;
    }
#pragma unroll
    for (int n = 0; n < WN; ++n) {
        ci_b[n] = PB ? ci_t * 32 + 2 * r + n : ci_t * 16 * WN + 16 * n + r;
        ci_ok[n] = ci_b[n] < a.cin;
    }
    const bool bias = tap == 4 && ci_t == 0;  // wave-uniform
    const unsigned W = unsigned(a.W), H = unsigned(a.H);
    f32x4 acc[WM][WN];
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
        for (int n = 0; n < WN; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[WM];
#pragma unroll
    for (int m = 0; m < WM; ++m) bsum[m] = 0.f;
    for (int pk = p_begin; pk < p_end; pk += 32) {
        const int p0 = pk + 8 * g;
        const unsigned q = unsigned(p0) / W;
        int x = int(unsigned(p0) - q * W);
        int y = int(q % H);
        uint16_t ah[WM][8], bh[WN][8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int p = p0 + j;
            const int yy = y + du, xx = x + dv;
            const bool in = p < p_end, src = in && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
            const long long oz = (long long)p * a.dz.cs + a.dz.co, ox = (long long)(p + shift) * a.x.cs + a.x.co;
            if constexpr (PA) {
                const uint32_t va = (in && co_ok[0]) ? *reinterpret_cast<const uint32_t*>(a.dz.p + oz + co_a[0]) : 0u;
                ah[0][j] = uint16_t(va);
                ah[1][j] = uint16_t(va >> 16);
            } else {
#pragma unroll
                for (int m = 0; m < WM; ++m) ah[m][j] = (in && co_ok[m]) ? a.dz.p[oz + co_a[m]] : uint16_t(0);
            }
            if constexpr (PB) {
                const uint32_t vb = (src && ci_ok[0]) ? *reinterpret_cast<const uint32_t*>(a.x.p + ox + ci_b[0]) : 0u;
                bh[0][j] = uint16_t(vb);
                bh[1][j] = uint16_t(vb >> 16);
            } else {
#pragma unroll
                for (int n = 0; n < WN; ++n) bh[n][j] = (src && ci_ok[n]) ? a.x.p[ox + ci_b[n]] : uint16_t(0);
            }
            if (++x == a.W) {
                x = 0;
                if (++y == a.H) y = 0;
            }
        }
        if (bias) {
#pragma unroll
            for (int m = 0; m < WM; ++m)
#pragma unroll
                for (int j = 0; j < 8; ++j) bsum[m] += bf2f(ah[m][j]);
        }
        bf16x8 av[WM], bv[WN];
#pragma unroll
        for (int m = 0; m < WM; ++m) {
            uint4 v;
            v.x = ah[m][0] | (uint32_t(ah[m][1]) << 16);
            v.y = ah[m][2] | (uint32_t(ah[m][3]) << 16);
            v.z = ah[m][4] | (uint32_t(ah[m][5]) << 16);
            v.w = ah[m][6] | (uint32_t(ah[m][7]) << 16);
            av[m] = as_bf16x8(v);
        }
#pragma unroll
        for (int n = 0; n < WN; ++n) {
            uint4 v;
            v.x = bh[n][0] | (uint32_t(bh[n][1]) << 16);
            v.y = bh[n][2] | (uint32_t(bh[n][3]) << 16);
            v.z = bh[n][4] | (uint32_t(bh[n][5]) << 16);
            v.w = bh[n][6] | (uint32_t(bh[n][7]) << 16);
            bv[n] = as_bf16x8(v);
        }
#pragma unroll
        for (int m = 0; m < WM; ++m)
#pragma unroll
            for (int n = 0; n < WN; ++n)
                acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv[n], acc[m][n], 0, 0, 0);
    }
    // lane holds D[4 g + i][r] of each 16 x 16 tile (m, n)
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
        for (int n = 0; n < WN; ++n)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = PA ? co_t * 32 + 2 * (4 * g + i) + m : co_t * 16 * WM + 16 * m + 4 * g + i;
                const int ci = ci_b[n];
                if (co < a.cout && ci < a.cin)
                    atomicAdd(&a.dw[((size_t)tap * a.cout_p + co) * a.cin_p + ci], acc[m][n][i]);
            }
    if (bias) {  // lanes r, r + 16, r + 32, r + 48 hold partial sums of channel co_a[m]
#pragma unroll
        for (int m = 0; m < WM; ++m) {
            float v = bsum[m];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (g == 0 && co_ok[m]) atomicAdd(&a.db[co_a[m]], v);
        }
    }
}

// One output channel (the output layer): dW[tap][0][ci] = sum_p dZ[p] X[p shifted by
// tap][ci] and db[0] = sum_p dZ[p] on the vector ALUs, where a matrix-core block would
// be 1/32 full.  Lane k of a 16-lane group holds channels 2k and 2k + 1 for all nine
// taps; group s of the block takes pixels p_begin + s, p_begin + s + 16, ... of the
// block's run, so a wave reads four consecutive pixels' channel rows per tap.  Taps
// that leave the image load the lane's own pixel and weigh it by zero (no branch
// around the loads); a pass takes eight of the group's pixels at once.  The groups
// meet in LDS and the block adds one partial sum per weight atomically.  Needs an
// even channel count of at most 32 and even X strides.
constexpr int C1_GROUPS = 16, C1_UNROLL = 8;
__global__ __launch_bounds__(256) void conv3x3_wgrad_c1_kernel(WgradArgs a) {
    __shared__ float part[C1_GROUPS][9 * 32 + 1];
    const int k = threadIdx.x & 15, grp = threadIdx.x >> 4;
    const int npx = a.N * a.H * a.W;  // the host keeps pixel indices below 2^31
    const int p_begin = blockIdx.x * int(a.chunk_px);
    const int p_end = p_begin < npx - int(a.chunk_px) ? p_begin + int(a.chunk_px) : npx;
    const int ch = 2 * k < a.cin ? 2 * k : 0;  // lanes past the channels read channel 0, write nothing
    const unsigned W = unsigned(a.W), H = unsigned(a.H);
    float acc[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t][0] = acc[t][1] = 0.f;
    float bsum = 0.f;
    // C1_UNROLL pixels per pass, all their loads issued before the arithmetic; a pixel
    // past the run stands in as the run's first pixel of this group, weighed by zero
    for (int p0 = p_begin + grp; p0 < p_end; p0 += C1_UNROLL * C1_GROUPS) {
        float z[C1_UNROLL];
        uint32_t v[C1_UNROLL][9];
        bool in[C1_UNROLL][9];
#pragma unroll
        for (int u = 0; u < C1_UNROLL; ++u) {
            const bool live = p0 + u * C1_GROUPS < p_end;
            const int p = live ? p0 + u * C1_GROUPS : p0;
            const unsigned q = unsigned(p) / W;
            const int x = int(unsigned(p) - q * W), y = int(q % H);
            const float zz = bf2f(a.dz.p[(long long)p * a.dz.cs + a.dz.co]);
            z[u] = live ? zz : 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int du = t / 3 - 1, dv = t % 3 - 1;
                in[u][t] = y + du >= 0 && y + du < a.H && x + dv >= 0 && x + dv < a.W;
                const int src = in[u][t] ? p + du * a.W + dv : p;
                v[u][t] = *reinterpret_cast<const uint32_t*>(a.x.p + (long long)src * a.x.cs + a.x.co + ch);
            }
        }
#pragma unroll
        for (int u = 0; u < C1_UNROLL; ++u) {
            bsum += z[u];
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const float w = in[u][t] ? z[u] : 0.f;
                acc[t][0] += w * bf2f(uint16_t(v[u][t]));
                acc[t][1] += w * bf2f(uint16_t(v[u][t] >> 16));
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        part[grp][t * 32 + 2 * k] = acc[t][0];
        part[grp][t * 32 + 2 * k + 1] = acc[t][1];
    }
    if (k == 0) part[grp][9 * 32] = bsum;
    __syncthreads();
    for (int i = threadIdx.x; i <= 9 * 32; i += 256) {
        float v = 0.f;
#pragma unroll
        for (int g2 = 0; g2 < C1_GROUPS; ++g2) v += part[g2][i];
        if (i == 9 * 32) {
            atomicAdd(&a.db[0], v);
        } else {
            const int tap = i / 32, ci = i % 32;
            if (ci < a.cin) atomicAdd(&a.dw[(size_t)tap * a.cout_p * a.cin_p + ci], v);
        }
    }
}

// Weight gradient through LDS, for 32, 64, 96 or 128 output channels (WCO = cout / 32)
// and a block of 32 input channels: 2 WCO waves, each owning 32 output by 16 input
// channels (few enough registers for two waves per SIMD, so that one wave's staging
// overlaps another's MFMAs).  The tap offset
// (du, dv) is split between the operands: dW[du, dv] = sum_q dZ[q - (du, 0)] X[q + (0, dv)]
// over the pixels q of the image (dZ and X zero outside it), so that for each pixel
// tile the workgroup stages dZ once, with one halo row above and below, and X in three
// copies shifted by dv = -1, 0, +1, all transposed to channel-major rows of 32 pixels
// (an MFMA operand lane reads 8 consecutive pixels of one channel with one 16-byte LDS
// read).  Per row of the tile a wave reads 3 x 2 A blocks and 3 B blocks and issues
// 18 MFMAs, one per (tap, 16 x 16 block).  A workgroup walks a run of tiles of
// WG_TH x 32 pixels and adds its sums to dW atomically once; the waves of the first
// input-channel block also sum dZ for the bias gradient.  Needs W % 32 == 0,
// H % WG_TH == 0, channel counts, strides and offsets that are multiples of 8.
constexpr int WG_TH = 4;
constexpr int WG_DZ_CH = (WG_TH + 2) * 32 + 8;  // LDS elements per channel: dZ rows y0-1 .. y0+TH, padded
constexpr int WG_X_CH = WG_TH * 32 + 8;         // LDS elements per channel of one shifted X copy

// 8 x 8 transpose of BF16 values: v[j] holds channels 0..7 of pixel j; o[c] gets pixels
// 0..7 of channel c.
__device__ __forceinline__ void transpose8(const uint4* v, uint4* o) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint32_t sel = (c & 1) ? 0x07060302u : 0x05040100u;
        uint32_t d[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint4 lo = v[2 * k], hi = v[2 * k + 1];
            const uint32_t a = (c >> 1) == 0 ? lo.x : (c >> 1) == 1 ? lo.y : (c >> 1) == 2 ? lo.z : lo.w;
            const uint32_t b = (c >> 1) == 0 ? hi.x : (c >> 1) == 1 ? hi.y : (c >> 1) == 2 ? hi.z : hi.w;
            d[k] = __builtin_amdgcn_perm(b, a, sel);  // low half: pixel 2k, high half: pixel 2k + 1
        }
        o[c] = make_uint4(d[0], d[1], d[2], d[3]);
    }
}

template <int WCO>
__global__ __launch_bounds__(128 * WCO) void conv3x3_wgrad_lds_kernel(WgradArgs a, int ci_blocks, int tiles_per_run) {
    constexpr int NT = 128 * WCO, CO_B = 32 * WCO, CG = CO_B / 8;
    __shared__ __attribute__((aligned(16))) uint16_t dzs[CO_B * WG_DZ_CH];
    __shared__ __attribute__((aligned(16))) uint16_t xs[3 * 32 * WG_X_CH];
    const int cib = blockIdx.x % ci_blocks, run = blockIdx.x / ci_blocks;
    const int ci0 = 32 * cib;
    const int tiles_x = a.W / 32, tiles_img = tiles_x * (a.H / WG_TH), tiles = a.N * tiles_img;
    const int t_begin = run * tiles_per_run;
    if (t_begin >= tiles) return;  // the whole workgroup
    const int t_end = min(t_begin + tiles_per_run, tiles);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    const int wco = wave >> 1, wci = wave & 1;  // 32 output channels 32 wco.., 16 input channels 16 wci..
    const bool bias = cib == 0;  // workgroup-uniform
    f32x4 acc[3][3][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int m = 0; m < 2; ++m) acc[i][j][m] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[8];  // channels 8 (threadIdx.x % CG) .. + 7: the same for every dZ unit of this thread
#pragma unroll
    for (int c = 0; c < 8; ++c) bsum[c] = 0.f;

    for (int t = t_begin; t < t_end; ++t) {
        const int img = t / tiles_img, tt = t - img * tiles_img;
        const int y0 = (tt / tiles_x) * WG_TH, x0 = (tt % tiles_x) * 32;
        // dZ rows y0 - 1 .. y0 + TH, channel-major; units of 8 channels x 8 pixels
        for (int u = threadIdx.x; u < CG * (WG_TH + 2) * 4; u += NT) {
            const int cg = u % CG, rb = u / CG, row = rb >> 2, b = rb & 3;
            const int y = y0 - 1 + row;
            const bool rin = y >= 0 && y < a.H;
            uint4 v[8], o[8];
            const long long p0 = ((long long)img * a.H + y) * a.W + x0 + 8 * b;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v[j] = rin ? *reinterpret_cast<const uint4*>(a.dz.p + (p0 + j) * a.dz.cs + a.dz.co + 8 * cg)
                           : make_uint4(0, 0, 0, 0);
            transpose8(v, o);
#pragma unroll
            for (int c = 0; c < 8; ++c)
                *reinterpret_cast<uint4*>(dzs + (8 * cg + c) * WG_DZ_CH + row * 32 + 8 * b) = o[c];
            if (bias && row >= 1 && row <= WG_TH) {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const uint32_t w[4] = {o[c].x, o[c].y, o[c].z, o[c].w};
                    float sum = 0.f;
#pragma unroll
                    for (int k = 0; k < 4; ++k) sum += bf2f(uint16_t(w[k])) + bf2f(uint16_t(w[k] >> 16));
                    bsum[c] += sum;
                }
            }
        }
        // X rows y0 .. y0 + TH - 1 in three copies: copy s holds X[y][x0 + i + s - 1], i = 0..31
        for (int u = threadIdx.x; u < 4 * WG_TH * 4; u += NT) {
            const int cg = u & 3, rb = u >> 2, row = rb >> 2, b = rb & 3;
            const int y = y0 + row, ci = ci0 + 8 * cg;
            const bool cin_ok = ci < a.cin;
            uint4 w[10], o[8];
            const long long prow = ((long long)img * a.H + y) * a.W;
#pragma unroll
            for (int j = 0; j < 10; ++j) {
                const int x = x0 + 8 * b - 1 + j;
                w[j] = (cin_ok && x >= 0 && x < a.W)
                           ? *reinterpret_cast<const uint4*>(a.x.p + (prow + x) * a.x.cs + a.x.co + ci)
                           : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int sft = 0; sft < 3; ++sft) {
                transpose8(w + sft, o);
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    *reinterpret_cast<uint4*>(xs + (sft * 32 + 8 * cg + c) * WG_X_CH + row * 32 + 8 * b) = o[c];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < WG_TH; ++k) {
            bf16x8 A[3][2], B[3];
#pragma unroll
            for (int i = 0; i < 3; ++i)  // du = i - 1: dZ row k - du of the tile, staged row k - du + 1
#pragma unroll
                for (int m = 0; m < 2; ++m)
                    A[i][m] = as_bf16x8(*reinterpret_cast<const uint4*>(
                        dzs + (32 * wco + 16 * m + r) * WG_DZ_CH + (k + 2 - i) * 32 + 8 * g));
#pragma unroll
            for (int j = 0; j < 3; ++j)  // dv = j - 1: copy j
                B[j] = as_bf16x8(
                    *reinterpret_cast<const uint4*>(xs + (j * 32 + 16 * wci + r) * WG_X_CH + k * 32 + 8 * g));
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int m = 0; m < 2; ++m)
                        acc[i][j][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i][m], B[j], acc[i][j][m], 0, 0, 0);
        }
        __syncthreads();  // the next tile overwrites the LDS
    }
    // lane holds D[4 g + q][r] of block m: output channel 32 wco + 16 m + 4 g + q, input
    // channel ci0 + 16 wci + r, tap (i, j)
    const int ci = ci0 + 16 * wci + r;
    if (ci < a.cin) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int co = 32 * wco + 16 * m + 4 * g + q;
                        atomicAdd(&a.dw[((size_t)(3 * i + j) * a.cout_p + co) * a.cin_p + ci], acc[i][j][m][q]);
                    }
    }
    if (bias) {  // the CO_B / 8 groups of 16 threads meet in LDS (free after the last barrier)
        float* red = reinterpret_cast<float*>(dzs);
#pragma unroll
        for (int c = 0; c < 8; ++c) red[threadIdx.x * 8 + c] = bsum[c];
        __syncthreads();
        if (threadIdx.x < CO_B) {
            const int co = threadIdx.x, cg = co >> 3;
            float v = 0.f;
            for (int k = 0; k < NT / CG; ++k) v += red[(cg + k * CG) * 8 + (co & 7)];
            if (co < a.cout) atomicAdd(&a.db[co], v);
        }
    }
}

// ---------------------------------------------------------------- elementwise
__global__ void avgpool2_kernel(TView in, TView out, int N, int H, int W, int C) {
    const int Ho = H / 2, Wo = W / 2;
    const long long total = (long long)N * Ho * Wo * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int c = int(i % C);
        const long long q = i / C;
        const int x = int(q % Wo);
        const long long t = q / Wo;
        const int y = int(t % Ho);
        const long long n = t / Ho;
        float s = 0.f;
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                s += bf2f(in.p[((n * H + 2 * y + dy) * W + 2 * x + dx) * in.cs + in.co + c]);
        out.p[q * out.cs + out.co + c] = f2bf(0.25f * s);
    }
}

// Four channels per thread (channel counts, strides and offsets multiples of 4, so
// the BF16 accesses are 8-byte and the FP32 ones 16-byte aligned).
__device__ __forceinline__ void ld4(const uint16_t* p, float v[4]) {
    const uint2 u = *reinterpret_cast<const uint2*>(p);
    v[0] = bf2f(uint16_t(u.x));
    v[1] = bf2f(uint16_t(u.x >> 16));
    v[2] = bf2f(uint16_t(u.y));
    v[3] = bf2f(uint16_t(u.y >> 16));
}
__device__ __forceinline__ void st4(uint16_t* p, const float v[4]) {
    uint2 u;
    u.x = uint32_t(f2bf(v[0])) | (uint32_t(f2bf(v[1])) << 16);
    u.y = uint32_t(f2bf(v[2])) | (uint32_t(f2bf(v[3])) << 16);
    *reinterpret_cast<uint2*>(p) = u;
}
// V = 4 or 8 channels: one 8- or 16-byte access (channel counts, strides and offsets
// multiples of V).
template <int V>
__device__ __forceinline__ void ldv(const uint16_t* p, float v[V]) {
    ld4(p, v);
    if constexpr (V == 8) ld4(p + 4, v + 4);
}
template <int V>
__device__ __forceinline__ void stv(uint16_t* p, const float v[V]) {
    if constexpr (V == 8) {
        uint4 u;
        u.x = uint32_t(f2bf(v[0])) | (uint32_t(f2bf(v[1])) << 16);
        u.y = uint32_t(f2bf(v[2])) | (uint32_t(f2bf(v[3])) << 16);
        u.z = uint32_t(f2bf(v[4])) | (uint32_t(f2bf(v[5])) << 16);
        u.w = uint32_t(f2bf(v[6])) | (uint32_t(f2bf(v[7])) << 16);
        *reinterpret_cast<uint4*>(p) = u;
    } else {
        st4(p, v);
    }
}
template <int V>
__device__ __forceinline__ void ldf(const float* p, float v[V]) {
#pragma unroll
    for (int k = 0; k < V; k += 4) {
        const float4 g = *reinterpret_cast<const float4*>(p + k);
        v[k] = g.x;
        v[k + 1] = g.y;
        v[k + 2] = g.z;
        v[k + 3] = g.w;
    }
}

// Index type I of the four- and eight-channel kernels: 32-bit where the element count
// stays below 2^31 (a division by a run-time size then costs a fraction of a 64-bit one),
// 64-bit otherwise; element offsets, and the fine-grid pixel indices of the kernels
// that count coarse pixels, are formed in 64 bits either way.
template <typename I, int V>
__global__ void avgpool2_vec_kernel(TView in, TView out, int N, int H, int W, int C) {
    const int Ho = H / 2, Wo = W / 2, CV = C / V;
    const I total = I(N) * I(Ho) * I(Wo) * I(CV);
    for (I i = I(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += I(gridDim.x) * blockDim.x) {
        const int c = int(i % I(CV)) * V;
        const I q = i / I(CV);
        const int x = int(q % I(Wo));
        const I t = q / I(Wo);
        const int y = int(t % I(Ho));
        const I n = t / I(Ho);
        float sum[V];
#pragma unroll
        for (int k = 0; k < V; ++k) sum[k] = 0.f;
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const long long pix = ((long long)n * H + 2 * y + dy) * W + 2 * x + dx;  // the fine grid
                float v[V];
                ldv<V>(in.p + pix * in.cs + in.co + c, v);
#pragma unroll
                for (int k = 0; k < V; ++k) sum[k] += v[k];
            }
        float o[V];
#pragma unroll
        for (int k = 0; k < V; ++k) o[k] = 0.25f * sum[k];
        stv<V>(out.p + (long long)q * out.cs + out.co + c, o);
    }
}

template <typename I, int V>
__global__ void upsample2_vec_kernel(TView in, TView out, int N, int H, int W, int C) {
    const int CV = C / V;
    const I total = I(N) * I(H) * I(W) * I(CV);
    for (I i = I(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += I(gridDim.x) * blockDim.x) {
        const int c = int(i % I(CV)) * V;
        const I q = i / I(CV);
        const int x = int(q % I(W));
        const I t = q / I(W);
        const int y = int(t % I(H));
        const I n = t / I(H);
        const I src = (n * I(H / 2) + I(y / 2)) * I(W / 2) + I(x / 2);
        if constexpr (V == 8)
            *reinterpret_cast<uint4*>(out.p + (long long)q * out.cs + out.co + c) =
                *reinterpret_cast<const uint4*>(in.p + (long long)src * in.cs + in.co + c);
        else
            *reinterpret_cast<uint2*>(out.p + (long long)q * out.cs + out.co + c) =
                *reinterpret_cast<const uint2*>(in.p + (long long)src * in.cs + in.co + c);
    }
}

template <typename I, int V>
__global__ void upsample2_grad_vec_kernel(const float* __restrict__ dcat, int dcs, int dco, TView act, TView dz,
                                         int N, int Ho, int Wo, int C) {
    const int CV = C / V;
    const I total = I(N) * I(Ho) * I(Wo) * I(CV);
    const int H = 2 * Ho, W = 2 * Wo;
    for (I i = I(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += I(gridDim.x) * blockDim.x) {
        const int c = int(i % I(CV)) * V;
        const I q = i / I(CV);
        const int x = int(q % I(Wo));
        const I t = q / I(Wo);
        const int y = int(t % I(Ho));
        const I n = t / I(Ho);
        float s[V];
#pragma unroll
        for (int k = 0; k < V; ++k) s[k] = 0.f;
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const long long pix = ((long long)n * H + 2 * y + dy) * W + 2 * x + dx;  // the fine grid
                float g[V];
                ldf<V>(dcat + pix * dcs + dco + c, g);
#pragma unroll
                for (int k = 0; k < V; ++k) s[k] += g[k];
            }
        float mk[V], o[V];
        ldv<V>(act.p + (long long)q * act.cs + act.co + c, mk);
#pragma unroll
        for (int k = 0; k < V; ++k) o[k] = mk[k] > 0.f ? s[k] : 0.f;
        stv<V>(dz.p + (long long)q * dz.cs + dz.co + c, o);
    }
}

template <typename I, int V>
__global__ void skip_grad_vec_kernel(const float* __restrict__ dcat, int dcs, int dco, const float* __restrict__ dpool,
                                    int pcs, TView act, TView dz, int N, int H, int W, int C) {
    const int CV = C / V;
    const I total = I(N) * I(H) * I(W) * I(CV);
    for (I i = I(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += I(gridDim.x) * blockDim.x) {
        const int c = int(i % I(CV)) * V;
        const I q = i / I(CV);
        const int x = int(q % I(W));
        const I t = q / I(W);
        const int y = int(t % I(H));
        const I n = t / I(H);
        const I parent = (n * I(H / 2) + I(y / 2)) * I(W / 2) + I(x / 2);
        float gp[V], gc[V], mk[V], o[V];
        ldf<V>(dpool + (long long)parent * pcs + c, gp);
        ldf<V>(dcat + (long long)q * dcs + dco + c, gc);
        ldv<V>(act.p + (long long)q * act.cs + act.co + c, mk);
#pragma unroll
        for (int k = 0; k < V; ++k) o[k] = mk[k] > 0.f ? gc[k] + 0.25f * gp[k] : 0.f;
        stv<V>(dz.p + (long long)q * dz.cs + dz.co + c, o);
    }
}

// out (H, W) = in (H/2, W/2) repeated 2 x 2.
__global__ void upsample2_kernel(TView in, TView out, int N, int H, int W, int C) {
    const long long total = (long long)N * H * W * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int c = int(i % C);
        const long long q = i / C;
        const int x = int(q % W);
        const long long t = q / W;
        const int y = int(t % H);
        const long long n = t / H;
        out.p[q * out.cs + out.co + c] = in.p[((n * (H / 2) + y / 2) * (W / 2) + x / 2) * in.cs + in.co + c];
    }
}

// Gradient of an upsampled tensor (sum of its 2 x 2 children in the FP32 concat
// gradient), times the ReLU mask of the activation it came from.
__global__ void upsample2_grad_kernel(const float* __restrict__ dcat, int dcs, int dco, TView act, TView dz, int N,
                                      int Ho, int Wo, int C) {
    const long long total = (long long)N * Ho * Wo * C;
    const int H = 2 * Ho, W = 2 * Wo;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int c = int(i % C);
        const long long q = i / C;
        const int x = int(q % Wo);
        const long long t = q / Wo;
        const int y = int(t % Ho);
        const long long n = t / Ho;
        float s = 0.f;
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) s += dcat[((n * H + 2 * y + dy) * W + 2 * x + dx) * dcs + dco + c];
        const float mk = bf2f(act.p[q * act.cs + act.co + c]);
        dz.p[q * dz.cs + dz.co + c] = f2bf(mk > 0.f ? s : 0.f);
    }
}

// Gradient of a skip tensor: its share of the FP32 concat gradient plus the
// average-pooling gradient dpool / 4 of its parent pixel, times its ReLU mask.
__global__ void skip_grad_kernel(const float* __restrict__ dcat, int dcs, int dco, const float* __restrict__ dpool,
                                 int pcs, TView act, TView dz, int N, int H, int W, int C) {
    const long long total = (long long)N * H * W * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int c = int(i % C);
        const long long q = i / C;
        const int x = int(q % W);
        const long long t = q / W;
        const int y = int(t % H);
        const long long n = t / H;
        const float gp = dpool[((n * (H / 2) + y / 2) * (W / 2) + x / 2) * pcs + c];
        const float s = dcat[q * dcs + dco + c] + 0.25f * gp;
        const float mk = bf2f(act.p[q * act.cs + act.co + c]);
        dz.p[q * dz.cs + dz.co + c] = f2bf(mk > 0.f ? s : 0.f);
    }
}

// NCHW FP32 input with 4 channels -> NHWC BF16 with 16 channels (12 zero).
// vec: the 16 channels of a pixel go out as two 16-byte stores (views in multiples of 8)
__global__ void pack_input_kernel(const float* __restrict__ in, int N, int H, int W, TView out, bool vec) {
    const long long total = (long long)N * H * W;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const long long n = q / ((long long)H * W), hw = q % ((long long)H * W);
        uint16_t b[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = f2bf(in[(n * 4 + c) * H * W + hw]);
        uint16_t* dst = out.p + q * out.cs + out.co;
        if (vec) {
            reinterpret_cast<uint4*>(dst)[0] =
                make_uint4(uint32_t(b[0]) | (uint32_t(b[1]) << 16), uint32_t(b[2]) | (uint32_t(b[3]) << 16), 0u, 0u);
            reinterpret_cast<uint4*>(dst)[1] = make_uint4(0u, 0u, 0u, 0u);
        } else {
            for (int c = 0; c < 16; ++c) dst[c] = c < 4 ? b[c] : 0;
        }
    }
}

// MSE: dY = 2 (y - t) / count as the BF16 gradient of channel 0 (others 0), and the
// per-block partial sums of (y - t)^2.
__global__ __launch_bounds__(256) void mse_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                  long long count, TView dz, double* __restrict__ partial) {
    // The gradient goes to channel 0 of a 16-channel pixel, the other 15 channels zero;
    // with 8-channel aligned views the pixel is written as two 16-byte stores.
    const bool vec = dz.cs % 8 == 0 && dz.co % 8 == 0;
    double s = 0.0;
    for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < count; q += (long long)gridDim.x * 256) {
        const float d = y[q] - t[q];
        s += double(d) * d;
        const uint16_t g = f2bf(2.0f * d / float(count));
        uint16_t* o = dz.p + q * dz.cs + dz.co;
        if (vec) {
            reinterpret_cast<uint4*>(o)[0] = make_uint4(g, 0u, 0u, 0u);
            reinterpret_cast<uint4*>(o)[1] = make_uint4(0u, 0u, 0u, 0u);
        } else {
            for (int c = 0; c < 16; ++c) o[c] = c == 0 ? g : 0;
        }
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (unsigned o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Adam on the FP32 master copy, then the BF16 working copy.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, uint16_t* __restrict__ p_bf16, long long n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        if (p_bf16) p_bf16[i] = f2bf(pi);
    }
}

// FP32 -> BF16 copy.
__global__ void to_bf16_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = f2bf(src[i]);
}

// Weights for the input gradient: Wt[t'][ci][co] = W[8 - t'][co][ci] (flip the 3 x 3
// window, swap the channel roles), padded as [9][cin_p16][cout_p32].
struct FlipBatch {
    FlipJob job[FLIP_MAX_JOBS];
    long long begin[FLIP_MAX_JOBS + 1];  // prefix sums of the jobs' element counts
    int n;
};

__global__ void flip_weights_kernel(FlipBatch b) {
    const long long total = b.begin[b.n];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        int j = 0;
        while (j + 1 < b.n && i >= b.begin[j + 1]) ++j;
        const FlipJob& J = b.job[j];
        const long long li = i - b.begin[j];
        const int k = int(li % J.t_cin_p);                // original output channel
        const int c = int((li / J.t_cin_p) % J.t_cout_p);  // original input channel
        const int tp = int(li / J.t_cin_p / J.t_cout_p);
        uint16_t v = 0;
        if (c < J.cin && k < J.cout) v = J.w[((size_t)(8 - tp) * J.cout_p + k) * J.cin_p + c];
        J.wt[li] = v;
    }
}

// Gathers minibatch rows of a resident dataset: dst[b] = src[idx[b]] (float rows of len).
// Grid rows walk the batch rows, so no element index is divided; with vec (16-byte
// aligned bases, len % 4 == 0) the rows are copied in 16-byte pieces.
__global__ void gather_rows_kernel(const float* __restrict__ src, const int* __restrict__ idx, long long len, int nb,
                                   float* __restrict__ dst, bool vec) {
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x, stride = (long long)gridDim.x * blockDim.x;
    for (int b = blockIdx.y; b < nb; b += gridDim.y) {
        const float* s = src + (long long)idx[b] * len;
        float* d = dst + (long long)b * len;
        if (vec) {
            for (long long i = t0; i < len / 4; i += stride)
                reinterpret_cast<float4*>(d)[i] = reinterpret_cast<const float4*>(s)[i];
        } else {
            for (long long i = t0; i < len; i += stride) d[i] = s[i];
        }
    }
}

int grid_for(long long n) {
    long long g = (n + 255) / 256;
    return int(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

hipError_t conv3x3(const ConvArgs& a, hipStream_t s) {
    const long long npx = (long long)a.N * a.H * a.W;
    (void)hipGetLastError();
    const bool views8 = a.cout % 8 == 0 && a.out.cs % 8 == 0 && a.out.co % 8 == 0 &&
                        (a.epi != EPI_MASK_BF16 || (a.mask.cs % 8 == 0 && a.mask.co % 8 == 0));
    const int ncb = a.cin_p / 32;
    // the run-of-tiles kernel: one input block, and three or more on large maps (or
    // five or more at any size); two blocks keep the blocked kernel with its wider
    // output blocks (measured per layer: 256^2 of 96 channels 128 -> 113 us,
    // 128^2 of 160 channels 94 -> 80 us, but 128^2 of 64 channels 43 -> 47 us and
    // 64^2 of 96 channels 18 -> 27 us with runs)
    const bool big = a.cout_p % 32 == 0 && (a.epi == EPI_F32 || views8);  // the run or a blocked kernel
    const bool run = big && a.cin_p % 32 == 0 && a.H >= 16 && (ncb == 1 || (ncb >= 3 && a.H >= 128) || ncb >= 5);
    auto blocks_of = [&](int th, int co_b) {
        return (long long)a.N * ((a.H + th - 1) / th) * ((a.W + LT_W - 1) / LT_W) * (a.cout_p / co_b);
    };
    // the blocked kernel's channel block: the widest (each staged halo then serves more
    // output channels) that still gives at least 1024 workgroups (64 or 96 channels, 4
    // rows per wave), else 32 channels with 4 rows per wave if that gives 512, else with
    // 2 (measured: a 64^2 layer of 96 channels takes 46 us as one 96-channel block of
    // 256 workgroups, 32 us as three 32-channel blocks of 4 rows per wave, 37 us of 2)
    constexpr long long ENOUGH = 1024;
    const long long b64 = a.cout_p % 64 == 0 ? blocks_of(LdsConv<4, 64>::TH, 64) : 0;
    const long long b96 = a.cout_p % 96 == 0 ? blocks_of(LdsConv<4, 96>::TH, 96) : 0;
    const long long b32 = blocks_of(LdsConv<4, 32>::TH, 32);
    const int co_b = run ? 32 : b64 >= ENOUGH ? 64 : b96 >= ENOUGH ? 96 : 32;
    // the run and blocked kernels write the pooled and upsampled copies in their
    // epilogues; for other layers separate passes follow
    const bool fuse = a.epi == EPI_RELU_BF16 && big;
    const bool pool_ok = a.pool.p == nullptr || (fuse && a.H % 2 == 0 && a.W % 2 == 0 && a.pool.cs % 8 == 0 &&
                                                 a.pool.co % 8 == 0);
    const bool up_ok = a.up.p == nullptr || (fuse && a.up.cs % 8 == 0 && a.up.co % 8 == 0);
    // and fold the upsampling gradient into their FP32 epilogues when whole channel
    // blocks are folded
    const bool fold_ok = a.fold.p == nullptr ||
                         (big && a.epi == EPI_F32 && a.bias == nullptr && a.H % 2 == 0 && a.W % 2 == 0 &&
                          a.fold_c % co_b == 0 && a.fold_c <= a.cout && a.fold.cs % 4 == 0 && a.fold.co % 4 == 0 &&
                          a.fold_act.cs % 4 == 0 && a.fold_act.co % 4 == 0);
    if (!pool_ok || !up_ok || !fold_ok) {
        ConvArgs b = a;
        if (!pool_ok) b.pool = TView{nullptr, 0, 0};
        if (!up_ok) b.up = TView{nullptr, 0, 0};
        if (!fold_ok) b.fold = TView{nullptr, 0, 0};
        hipError_t e = conv3x3(b, s);
        if (e == hipSuccess && !pool_ok) e = avgpool2(a.out, a.pool, a.N, a.H, a.W, a.cout, s);
        if (e == hipSuccess && !up_ok) e = upsample2(a.out, a.up, a.N, 2 * a.H, 2 * a.W, a.cout, s);
        if (e == hipSuccess && !fold_ok)
            e = upsample2_grad(a.out_f32, a.out_f32_cs, 0, a.fold_act, a.fold, a.N, a.H / 2, a.W / 2, a.fold_c, s);
        return e;
    }
    auto lds = [&](auto kernel, int th, int co_b) {
        hipLaunchKernelGGL(kernel, dim3(unsigned(blocks_of(th, co_b))), dim3(256), 0, s, a);
    };
    if (a.cin == 1 && a.cout <= 32 && a.cout % 8 == 0 && a.epi == EPI_MASK_BF16 && views8) {
        const long long tiles = (long long)a.N * ((a.H + C1_T - 1) / C1_T) * ((a.W + C1_T - 1) / C1_T);
        hipLaunchKernelGGL(conv3x3_from1_kernel, dim3(unsigned(tiles)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    if (big) {
        if (run) {
            // two workgroups per CU
            const int co_blocks = a.cout_p / 32;
            const long long tiles = blocks_of(LdsConv<4, 32>::TH, 32) / co_blocks;
            long long runs = std::max<long long>(1, 512 / co_blocks);
            runs = std::min(runs, tiles);
            const int per_run = int((tiles + runs - 1) / runs);
            runs = (tiles + per_run - 1) / per_run;
            hipLaunchKernelGGL((conv3x3_lds_run_kernel<4, 32>), dim3(unsigned(runs * co_blocks)), dim3(256), 0, s, a,
                               per_run);
            return hipGetLastError();
        }
        if (b64 >= ENOUGH)
            lds(conv3x3_lds_kernel<4, 64>, LdsConv<4, 64>::TH, 64);
        else if (b96 >= ENOUGH)
            lds(conv3x3_lds_kernel<4, 96>, LdsConv<4, 96>::TH, 96);
        else if (b32 >= ENOUGH / 2)
            lds(conv3x3_lds_kernel<4, 32>, LdsConv<4, 32>::TH, 32);
        else
            lds(conv3x3_lds_kernel<2, 32>, LdsConv<2, 32>::TH, 32);
    } else if (a.cout == 1 && a.epi == EPI_F32 && a.cin % 8 == 0 && a.in.cs % 8 == 0 && a.in.co % 8 == 0) {
        const long long tiles = (long long)a.N * ((a.H + C1_T - 1) / C1_T) * ((a.W + C1_T - 1) / C1_T);
        hipLaunchKernelGGL(conv3x3_c1_kernel, dim3(unsigned(tiles)), dim3(256), 0, s, a);
    } else {
        const long long waves = ((npx + 63) / 64) * (a.cout_p / 16);
        hipLaunchKernelGGL((conv3x3_kernel<4, 1>), dim3(int((waves + 3) / 4)), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

template <int WM, int WN, bool PA, bool PB>
hipError_t wgrad_launch(const WgradArgs& a, hipStream_t s) {
    const long long npx = (long long)a.N * a.H * a.W;
    const long long chunks = (npx + a.chunk_px - 1) / a.chunk_px;
    const long long tiles = 9LL * ((a.cout + 16 * WM - 1) / (16 * WM)) * ((a.cin + 16 * WN - 1) / (16 * WN));
    const long long waves = chunks * tiles;
    (void)hipGetLastError();
    hipLaunchKernelGGL((conv3x3_wgrad_kernel<WM, WN, PA, PB>), dim3(int((waves + 3) / 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// 2 x 2 blocks of 16 x 16 tiles for every layer (measured: 4-tile blocks along the
// wider layers leave too few waves and lose more than the shared gathers gain);
// channel pairs in one load where every channel count, stride and offset is even.
hipError_t conv3x3_wgrad(const WgradArgs& a, hipStream_t s) {
    const long long npx = (long long)a.N * a.H * a.W;
    if (npx + a.chunk_px >= (1LL << 31) || a.chunk_px % 32 != 0) return hipErrorInvalidValue;
    const bool even_a = a.cout % 2 == 0 && a.dz.cs % 2 == 0 && a.dz.co % 2 == 0;
    const bool even_b = a.cin % 2 == 0 && a.x.cs % 2 == 0 && a.x.co % 2 == 0;
    // pixel runs sized for about 16384 waves (512 to 8192 pixels): long runs for the
    // large layers (fewer atomic block updates), short ones for the small layers
    WgradArgs b = a;
    const long long tiles = 9LL * ((a.cout + 31) / 32) * ((a.cin + 31) / 32);
    long long c = npx * tiles / 16384;
    c = c < 512 ? 512 : (c > 8192 ? 8192 : c);
    b.chunk_px = c / 32 * 32;
    if (a.cout == 1 && even_b && a.cin <= 32) {  // the output layer
        // runs of 256 to 8192 pixels for about 2048 blocks
        long long r = (npx / 2048 + C1_GROUPS - 1) / C1_GROUPS * C1_GROUPS;
        b.chunk_px = r < 256 ? 256 : (r > 8192 ? 8192 : r);
        (void)hipGetLastError();
        hipLaunchKernelGGL(conv3x3_wgrad_c1_kernel, dim3(unsigned((npx + b.chunk_px - 1) / b.chunk_px)), dim3(256),
                           0, s, b);
        return hipGetLastError();
    }
    // the LDS kernel: 32 to 128 output channels in steps of 32, rows of whole 32-pixel
    // segments, 8-channel-aligned views
    const bool lds_ok = a.cout % 32 == 0 && a.cout <= 128 && a.cout_p == a.cout && a.W % 32 == 0 &&
                        a.H % WG_TH == 0 && a.cin % 8 == 0 && a.dz.cs % 8 == 0 && a.dz.co % 8 == 0 &&
                        a.x.cs % 8 == 0 && a.x.co % 8 == 0;
    if (lds_ok) {
        const int ci_blocks = (a.cin + 31) / 32;
        const long long tiles = (long long)a.N * (a.H / WG_TH) * (a.W / 32);
        // about 512 workgroups over all input-channel blocks, but runs of at least 8 tiles:
        // each run ends in 9 x cout x 32 atomic additions, which would outweigh the MFMA
        // work of shorter runs on the small lower levels (measured: 64^2 and 32^2 layers
        // at 66-170 TFLOP/s with runs of 1-7 tiles)
        long long runs = std::min<long long>(512 / ci_blocks, (tiles + 7) / 8);
        runs = runs < 1 ? 1 : runs;
        const int per_run = int((tiles + runs - 1) / runs);
        runs = (tiles + per_run - 1) / per_run;
        const dim3 grid(unsigned(runs * ci_blocks));
        (void)hipGetLastError();
        switch (a.cout / 32) {
        case 1: hipLaunchKernelGGL(conv3x3_wgrad_lds_kernel<1>, grid, dim3(128), 0, s, a, ci_blocks, per_run); break;
        case 2: hipLaunchKernelGGL(conv3x3_wgrad_lds_kernel<2>, grid, dim3(256), 0, s, a, ci_blocks, per_run); break;
        case 3: hipLaunchKernelGGL(conv3x3_wgrad_lds_kernel<3>, grid, dim3(384), 0, s, a, ci_blocks, per_run); break;
        default:
            hipLaunchKernelGGL(conv3x3_wgrad_lds_kernel<4>, grid, dim3(512), 0, s, a, ci_blocks, per_run);
            break;
        }
        return hipGetLastError();
    }
    if (even_a && even_b) return wgrad_launch<2, 2, true, true>(b, s);
    if (even_b) return wgrad_launch<2, 2, false, true>(b, s);
    if (even_a) return wgrad_launch<2, 2, true, false>(b, s);
    return wgrad_launch<2, 2, false, false>(b, s);
}

static bool byv(int V, int C, const TView& a, const TView& b) {
    return C % V == 0 && a.cs % V == 0 && a.co % V == 0 && b.cs % V == 0 && b.co % V == 0;
}
static bool by4(int C, const TView& a, const TView& b) { return byv(4, C, a, b); }

// Launches a V-channel kernel over `groups` channel groups with the narrowest index
// type that holds the count and the grid stride past it.
#define SUR_LAUNCH_VEC(kernel, V, groups, s, ...)                                                                 \
    do {                                                                                                        \
        if ((groups) < (1LL << 31))                                                                             \
            hipLaunchKernelGGL((kernel<uint32_t, V>), dim3(grid_for(groups)), dim3(256), 0, s, __VA_ARGS__);    \
        else                                                                                                    \
            hipLaunchKernelGGL((kernel<unsigned long long, V>), dim3(grid_for(groups)), dim3(256), 0, s,          \
                               __VA_ARGS__);                                                                    \
    } while (0)

hipError_t avgpool2(TView in, TView out, int N, int H, int W, int C, hipStream_t s) {
    if (byv(8, C, in, out)) {
        SUR_LAUNCH_VEC(avgpool2_vec_kernel, 8, (long long)N * (H / 2) * (W / 2) * (C / 8), s, in, out, N, H, W, C);
        return hipGetLastError();
    }
    if (by4(C, in, out)) {
        SUR_LAUNCH_VEC(avgpool2_vec_kernel, 4, (long long)N * (H / 2) * (W / 2) * (C / 4), s, in, out, N, H, W, C);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(avgpool2_kernel, dim3(grid_for((long long)N * (H / 2) * (W / 2) * C)), dim3(256), 0, s, in,
                       out, N, H, W, C);
    return hipGetLastError();
}

hipError_t upsample2(TView in, TView out, int N, int H, int W, int C, hipStream_t s) {
    if (byv(8, C, in, out)) {
        SUR_LAUNCH_VEC(upsample2_vec_kernel, 8, (long long)N * H * W * (C / 8), s, in, out, N, H, W, C);
        return hipGetLastError();
    }
    if (by4(C, in, out)) {
        SUR_LAUNCH_VEC(upsample2_vec_kernel, 4, (long long)N * H * W * (C / 4), s, in, out, N, H, W, C);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(upsample2_kernel, dim3(grid_for((long long)N * H * W * C)), dim3(256), 0, s, in, out, N, H, W,
                       C);
    return hipGetLastError();
}

// The two gradient kernels take four channels per thread: with eight (two 16-byte FP32
// loads per input) they measured slower.
hipError_t upsample2_grad(const float* dcat, int dcs, int dco, TView act, TView dz, int N, int Ho, int Wo, int C,
                          hipStream_t s) {
    if (by4(C, act, dz) && dcs % 4 == 0 && dco % 4 == 0) {
        SUR_LAUNCH_VEC(upsample2_grad_vec_kernel, 4, (long long)N * Ho * Wo * (C / 4), s, dcat, dcs, dco, act, dz, N,
                       Ho, Wo, C);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(upsample2_grad_kernel, dim3(grid_for((long long)N * Ho * Wo * C)), dim3(256), 0, s, dcat, dcs,
                       dco, act, dz, N, Ho, Wo, C);
    return hipGetLastError();
}

hipError_t skip_grad(const float* dcat, int dcs, int dco, const float* dpool, int pcs, TView act, TView dz, int N,
                     int H, int W, int C, hipStream_t s) {
    if (by4(C, act, dz) && dcs % 4 == 0 && dco % 4 == 0 && pcs % 4 == 0) {
        SUR_LAUNCH_VEC(skip_grad_vec_kernel, 4, (long long)N * H * W * (C / 4), s, dcat, dcs, dco, dpool, pcs, act, dz,
                       N, H, W, C);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(skip_grad_kernel, dim3(grid_for((long long)N * H * W * C)), dim3(256), 0, s, dcat, dcs, dco,
                       dpool, pcs, act, dz, N, H, W, C);
    return hipGetLastError();
}

hipError_t pack_input(const float* in, int N, int H, int W, TView out, hipStream_t s) {
    const bool vec = out.cs % 8 == 0 && out.co % 8 == 0 && out.cs >= 16;
    hipLaunchKernelGGL(pack_input_kernel, dim3(grid_for((long long)N * H * W)), dim3(256), 0, s, in, N, H, W, out,
                       vec);
    return hipGetLastError();
}

hipError_t mse(const float* y, const float* t, long long count, TView dz, double* partial, int blocks,
               hipStream_t s) {
    hipLaunchKernelGGL(mse_kernel, dim3(blocks), dim3(256), 0, s, y, t, count, dz, partial);
    return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, uint16_t* p_bf16, long long n, float lr, int step,
                hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, float(step)), c2 = 1.f - powf(b2, float(step));
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, g, m, v, p_bf16, n, lr, b1, b2, 1e-8f, c1,
                       c2);
    return hipGetLastError();
}

hipError_t to_bf16(const float* src, uint16_t* dst, long long n, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t flip_weights(const FlipJob* jobs, int n, hipStream_t s) {
    if (n < 1 || n > FLIP_MAX_JOBS) return hipErrorInvalidValue;
    FlipBatch b{};
    b.n = n;
    b.begin[0] = 0;
    for (int j = 0; j < n; ++j) {
        b.job[j] = jobs[j];
        b.begin[j + 1] = b.begin[j] + 9LL * jobs[j].t_cout_p * jobs[j].t_cin_p;
    }
    hipLaunchKernelGGL(flip_weights_kernel, dim3(grid_for(b.begin[n])), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t gather_rows(const float* src, const int* idx, long long len, int nb, float* dst, hipStream_t s) {
    const bool vec = len % 4 == 0 && reinterpret_cast<uintptr_t>(src) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(dst) % 16 == 0;
    const dim3 grid(grid_for(vec ? len / 4 : len), nb < 65535 ? nb : 65535);
    hipLaunchKernelGGL(gather_rows_kernel, grid, dim3(256), 0, s, src, idx, len, nb, dst, vec);
    return hipGetLastError();
}

}  // namespace sur
}  // namespace cplbm
