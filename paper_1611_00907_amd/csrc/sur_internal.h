// Internal interface of the surrogate's HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cplbm {
namespace sur {

// NHWC BF16 tensor view: element (pixel p, channel c) is p[p * cs + co + c].
struct TView {
    uint16_t* p;
    int cs;  // channels per pixel in the buffer
    int co;  // first channel of the view
};

enum Epi : int {
    EPI_RELU_BF16 = 0,  // + bias, ReLU, BF16 out
    EPI_MASK_BF16 = 1,  // times (mask > 0), BF16 out (gradient through a ReLU)
    EPI_BF16 = 2,       // + bias, BF16 out
    EPI_F32 = 3         // + bias (if any), FP32 out
};

struct ConvArgs {
    TView in;
    const uint16_t* w;   // [9][cout_p][cin_p] BF16
    const float* bias;   // [cout] or null
    TView out;           // BF16 epilogues
    float* out_f32;      // EPI_F32: out_f32[p * out_f32_cs + c]
    int out_f32_cs;
    TView mask;          // EPI_MASK_BF16
    int N, H, W;
    int cin, cin_p;      // input channels read (multiple of 8), padded k extent (multiple of 32)
    int cout, cout_p;    // output channels stored, padded (multiple of 16)
    int epi;
    TView pool;          // EPI_RELU_BF16: the 2 x 2 average of the output at half size (p null: none)
    TView up;            // EPI_RELU_BF16: the output repeated 2 x 2 at twice the size (p null: none)
    // EPI_F32 without bias: channels [0, fold_c) of the output summed over 2 x 2 pixel
    // blocks, zeroed where fold_act is not > 0, into fold (BF16, half size): the
    // upsampling gradient (p null: none).  A kernel that folds does not store those
    // channels of out_f32; one that cannot leaves the fold to a separate pass.
    TView fold, fold_act;
    int fold_c;
};

struct WgradArgs {
    TView x;             // convolution input
    TView dz;            // gradient at the convolution output (before its bias)
    float* dw;           // [9][cout_p][cin_p] FP32, accumulated atomically
    float* db;           // [cout] FP32 bias gradient, accumulated atomically
    int N, H, W;
    int cin, cin_p, cout, cout_p;
    long long chunk_px;  // pixels per wave
};

hipError_t conv3x3(const ConvArgs& a, hipStream_t s);
hipError_t conv3x3_wgrad(const WgradArgs& a, hipStream_t s);
hipError_t avgpool2(TView in, TView out, int N, int H, int W, int C, hipStream_t s);
hipError_t upsample2(TView in, TView out, int N, int H, int W, int C, hipStream_t s);
hipError_t upsample2_grad(const float* dcat, int dcs, int dco, TView act, TView dz, int N, int Ho, int Wo, int C,
                          hipStream_t s);
hipError_t skip_grad(const float* dcat, int dcs, int dco, const float* dpool, int pcs, TView act, TView dz, int N,
                     int H, int W, int C, hipStream_t s);
hipError_t pack_input(const float* in, int N, int H, int W, TView out, hipStream_t s);
hipError_t mse(const float* y, const float* t, long long count, TView dz, double* partial, int blocks,
               hipStream_t s);
hipError_t adam(float* p, const float* g, float* m, float* v, uint16_t* p_bf16, long long n, float lr, int step,
                hipStream_t s);
hipError_t to_bf16(const float* src, uint16_t* dst, long long n, hipStream_t s);
// The weights of one layer for its input gradient: wt[tap][c][k] = w[8 - tap][k][c]
// (taps mirrored, input and output channels swapped), zero beyond cin / cout.
struct FlipJob {
    const uint16_t* w;
    uint16_t* wt;
    int cout_p, cin_p, cin, cout, t_cout_p, t_cin_p;
};
constexpr int FLIP_MAX_JOBS = 16;
// All layers' flips in one launch (at most FLIP_MAX_JOBS).
hipError_t flip_weights(const FlipJob* jobs, int n, hipStream_t s);
hipError_t gather_rows(const float* src, const int* idx, long long len, int nb, float* dst, hipStream_t s);

}  // namespace sur
}  // namespace cplbm
