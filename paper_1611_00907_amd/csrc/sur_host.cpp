// C ABI of the convolutional surrogate (declared in lbm.h): a 4-level
// encoder-decoder of 3x3 convolutions that maps (solid mask, initial density,
// T/Tc, wall chemical potential) to the equilibrium density field, with BF16
// MFMA forward and backward kernels, FP32 master weights and Adam, all on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm_common.h"
#include "sur_internal.h"

using namespace cplbm;
using namespace cplbm::host;
using namespace cplbm::sur;

namespace {

constexpr int IN_CHANNELS = 4;
constexpr int IN_PADDED = 16;
constexpr int L0 = 32, L1 = 64, L2 = 96, L3 = 128;

int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct LayerDef {
    const char* name;
    int cin, cout;
    bool relu;
};

// Evaluation order; the exchange layout of the parameters follows it.
const LayerDef LAYERS[] = {
    {"e0a", IN_PADDED, L0, true}, {"e0b", L0, L0, true},      {"e1a", L0, L1, true},
    {"e1b", L1, L1, true},        {"e2a", L1, L2, true},      {"e2b", L2, L2, true},
    {"e3a", L2, L3, true},        {"e3b", L3, L3, true},      {"d2a", L3 + L2, L2, true},
    {"d2b", L2, L2, true},        {"d1a", L2 + L1, L1, true}, {"d1b", L1, L1, true},
    {"d0a", L1 + L0, L0, true},   {"d0b", L0, L0, true},      {"out", L0, 1, false},
};
constexpr int NL = sizeof(LAYERS) / sizeof(LAYERS[0]);
enum { E0A, E0B, E1A, E1B, E2A, E2B, E3A, E3B, D2A, D2B, D1A, D1B, D0A, D0B, OUT };
static_assert(NL == OUT + 1, "one enumerator per layer of the table");

struct Layer {
    LayerDef d;
    int cin_p, cout_p;          // kernel layout padding
    size_t w_off, b_off;        // in the FP32 master array (elements)
    size_t ex_w, ex_b;          // in the exchange layout (elements)
    int t_cout_p, t_cin_p;      // flipped weights for the input gradient
    size_t t_off;               // in the flipped BF16 array
};

}  // namespace

struct sur_net {
    int size = 0, max_batch = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<Layer> L;
    size_t n_master = 0, n_exchange = 0, n_flip = 0;
    // parameters
    float *master = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *wbf = nullptr, *wflip = nullptr;
    int adam_step = 0;
    // activations (BF16 NHWC) and gradients
    uint16_t *x0 = nullptr, *e0a = nullptr, *c0 = nullptr, *p0 = nullptr, *e1a = nullptr, *c1 = nullptr;
    uint16_t *p1 = nullptr, *e2a = nullptr, *c2 = nullptr, *p2 = nullptr, *e3a = nullptr, *e3 = nullptr;
    uint16_t *d2a = nullptr, *d2 = nullptr, *d1a = nullptr, *d1 = nullptr, *d0a = nullptr, *d0 = nullptr;
    uint16_t *dz_out = nullptr, *dz_a = nullptr, *dz_b = nullptr;  // gradient scratch (largest level)
    float *dc0 = nullptr, *dc1 = nullptr, *dc2 = nullptr, *dp = nullptr;
    float *y = nullptr, *t = nullptr, *in = nullptr;
    double* partial = nullptr;
    double* partial_host = nullptr;
    int* idx = nullptr;
    // resident dataset
    float *ds_in = nullptr, *ds_t = nullptr;
    int ds_count = 0;
    std::vector<void*> allocs;
    // trace of the last backward pass (sur_trace): each layer's output gradient dz as its
    // weight gradient read it, and the pooled-branch gradients of e3a, e2a, e1a
    bool trace = false;
    uint16_t* trace_dz[15] = {};
    float* trace_dp[3] = {};
    int last_N = 0;         // images of the last forward pass
    bool have_backward = false;
};

namespace {

constexpr int MSE_BLOCKS = 1024;  // four workgroups per compute unit

template <typename T>
lbm_status dalloc(sur_net* n, T** p, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, count * sizeof(T) + 256) != hipSuccess) return LBM_ENOMEM;
    if (hipMemsetAsync(q, 0, count * sizeof(T) + 256, n->stream) != hipSuccess) return LBM_EHIP;
    n->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return LBM_OK;
}

void free_trace(sur_net* n) {
    for (auto& p : n->trace_dz) {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    for (auto& p : n->trace_dp) {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    n->trace = false;
}

void release(sur_net* n) {
    if (!n) return;
    free_trace(n);
    for (void* p : n->allocs) (void)hipFree(p);
    if (n->partial_host) (void)hipHostFree(n->partial_host);
    if (n->stream) (void)hipStreamDestroy(n->stream);
    delete n;
}

TView tv(uint16_t* p, int cs, int co = 0) { return TView{p, cs, co}; }

hipError_t conv(sur_net* n, int li, TView in, int N, int H, int W, int epi, TView out, float* out_f32 = nullptr,
                int out_f32_cs = 0, TView pool = TView{nullptr, 0, 0}, TView up = TView{nullptr, 0, 0}) {
    const Layer& l = n->L[li];
    ConvArgs a{};
    a.in = in;
    a.w = n->wbf + l.w_off;
    a.bias = (epi == EPI_MASK_BF16) ? nullptr : n->master + l.b_off;
    a.out = out;
    a.out_f32 = out_f32;
    a.out_f32_cs = out_f32_cs;
    a.N = N;
    a.H = H;
    a.W = W;
    a.cin = l.d.cin;
    a.cin_p = l.cin_p;
    a.cout = l.d.cout;
    a.cout_p = l.cout_p;
    a.epi = epi;
    a.pool = pool;
    a.up = up;
    return conv3x3(a, n->stream);
}

// Input gradient of layer li: the flipped convolution of dz (its output gradient).
hipError_t conv_back(sur_net* n, int li, TView dz, int N, int H, int W, int epi, TView out, TView mask,
                     float* out_f32 = nullptr, int out_f32_cs = 0, TView fold = TView{nullptr, 0, 0},
                     TView fold_act = TView{nullptr, 0, 0}, int fold_c = 0) {
    const Layer& l = n->L[li];
    ConvArgs a{};
    a.in = dz;
    a.w = n->wflip + l.t_off;
    a.bias = nullptr;
    a.out = out;
    a.mask = mask;
    a.out_f32 = out_f32;
    a.out_f32_cs = out_f32_cs;
    a.N = N;
    a.H = H;
    a.W = W;
    // the matrix-core kernels read 8-channel groups; the one-channel output gradient
    // of the output layer goes to a kernel that reads its one channel
    a.cin = l.d.cout == 1 ? 1 : round_up(l.d.cout, 8);
    a.cin_p = l.t_cin_p;
    a.cout = l.d.cin;
    a.cout_p = l.t_cout_p;
    a.epi = epi;
    a.fold = fold;
    a.fold_act = fold_act;
    a.fold_c = fold_c;
    return conv3x3(a, n->stream);
}

hipError_t wgrad(sur_net* n, int li, TView x, TView dz, int N, int H, int W) {
    const Layer& l = n->L[li];
    WgradArgs a{};
    a.x = x;
    a.dz = dz;
    a.dw = n->grad + l.w_off;
    a.N = N;
    a.H = H;
    a.W = W;
    a.cin = l.d.cin;
    a.cin_p = l.cin_p;
    a.cout = l.d.cout;
    a.cout_p = l.cout_p;
    a.db = n->grad + l.b_off;
    a.chunk_px = 2048;
    if (n->trace && n->trace_dz[li]) {  // dz views start at channel 0 of their buffer
        const hipError_t e = hipMemcpyAsync(n->trace_dz[li], dz.p, (size_t)N * H * W * dz.cs * sizeof(uint16_t),
                                            hipMemcpyDeviceToDevice, n->stream);
        if (e != hipSuccess) return e;
    }
    return conv3x3_wgrad(a, n->stream);
}

// Copy of the pooled-branch gradient dp (FP32, C channels) into trace slot k.
hipError_t trace_dp(sur_net* n, int k, int N, int H, int W, int C) {
    if (!n->trace || !n->trace_dp[k]) return hipSuccess;
    return hipMemcpyAsync(n->trace_dp[k], n->dp, (size_t)N * H * W * C * sizeof(float), hipMemcpyDeviceToDevice,
                          n->stream);
}

// One launch for every layer's flipped weights (they change with every Adam step).
hipError_t refresh_flipped(sur_net* n) {
    static_assert(NL <= FLIP_MAX_JOBS, "one flip job per layer");
    FlipJob jobs[FLIP_MAX_JOBS];
    int k = 0;
    for (const Layer& l : n->L)
        jobs[k++] = FlipJob{n->wbf + l.w_off, n->wflip + l.t_off, l.cout_p, l.cin_p, l.d.cin, l.d.cout,
                            l.t_cout_p, l.t_cin_p};
    return flip_weights(jobs, k, n->stream);
}

#define SUR_TRY(expr)                                       \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_status(e_, #expr); \
    } while (0)

// Forward pass of N images already packed in x0; prediction (FP32) into y.
lbm_status forward(sur_net* n, int N) {
    const int S0 = n->size, S1 = S0 / 2, S2 = S0 / 4, S3 = S0 / 8;
    n->last_N = N;
    n->have_backward = false;
    SUR_TRY(conv(n, E0A, tv(n->x0, IN_PADDED), N, S0, S0, EPI_RELU_BF16, tv(n->e0a, L0)));
    // the encoder's second convolutions also write the 2 x 2 average of their output
    SUR_TRY(conv(n, E0B, tv(n->e0a, L0), N, S0, S0, EPI_RELU_BF16, tv(n->c0, L1 + L0, L1), nullptr, 0, tv(n->p0, L0)));
    SUR_TRY(conv(n, E1A, tv(n->p0, L0), N, S1, S1, EPI_RELU_BF16, tv(n->e1a, L1)));
    SUR_TRY(conv(n, E1B, tv(n->e1a, L1), N, S1, S1, EPI_RELU_BF16, tv(n->c1, L2 + L1, L2), nullptr, 0, tv(n->p1, L1)));
    SUR_TRY(conv(n, E2A, tv(n->p1, L1), N, S2, S2, EPI_RELU_BF16, tv(n->e2a, L2)));
    SUR_TRY(conv(n, E2B, tv(n->e2a, L2), N, S2, S2, EPI_RELU_BF16, tv(n->c2, L3 + L2, L3), nullptr, 0, tv(n->p2, L2)));
    SUR_TRY(conv(n, E3A, tv(n->p2, L2), N, S3, S3, EPI_RELU_BF16, tv(n->e3a, L3)));
    // the last encoder and the decoders' second convolutions also write their output
    // repeated 2 x 2 into the next level's concatenation
    SUR_TRY(conv(n, E3B, tv(n->e3a, L3), N, S3, S3, EPI_RELU_BF16, tv(n->e3, L3), nullptr, 0, TView{nullptr, 0, 0},
                 tv(n->c2, L3 + L2, 0)));
    SUR_TRY(conv(n, D2A, tv(n->c2, L3 + L2), N, S2, S2, EPI_RELU_BF16, tv(n->d2a, L2)));
    SUR_TRY(conv(n, D2B, tv(n->d2a, L2), N, S2, S2, EPI_RELU_BF16, tv(n->d2, L2), nullptr, 0, TView{nullptr, 0, 0},
                 tv(n->c1, L2 + L1, 0)));
    SUR_TRY(conv(n, D1A, tv(n->c1, L2 + L1), N, S1, S1, EPI_RELU_BF16, tv(n->d1a, L1)));
    SUR_TRY(conv(n, D1B, tv(n->d1a, L1), N, S1, S1, EPI_RELU_BF16, tv(n->d1, L1), nullptr, 0, TView{nullptr, 0, 0},
                 tv(n->c0, L1 + L0, 0)));
    SUR_TRY(conv(n, D0A, tv(n->c0, L1 + L0), N, S0, S0, EPI_RELU_BF16, tv(n->d0a, L0)));
    SUR_TRY(conv(n, D0B, tv(n->d0a, L0), N, S0, S0, EPI_RELU_BF16, tv(n->d0, L0)));
    SUR_TRY(conv(n, OUT, tv(n->d0, L0), N, S0, S0, EPI_F32, tv(nullptr, 0), n->y, 1));
    return LBM_OK;
}

// Loss against the targets in t and the gradient of every parameter into grad.
lbm_status backward(sur_net* n, int N, double* loss) {
    const int S0 = n->size, S1 = S0 / 2, S2 = S0 / 4, S3 = S0 / 8;
    const long long cnt = (long long)N * S0 * S0;
    SUR_TRY(hipMemsetAsync(n->grad, 0, n->n_master * sizeof(float), n->stream));
    SUR_TRY(mse(n->y, n->t, cnt, tv(n->dz_out, 16), n->partial, MSE_BLOCKS, n->stream));
    SUR_TRY(hipMemcpyAsync(n->partial_host, n->partial, MSE_BLOCKS * sizeof(double), hipMemcpyDeviceToHost,
                           n->stream));
    TView none = tv(nullptr, 0);
    uint16_t *A = n->dz_a, *B = n->dz_b;
    // level 0 decoder
    SUR_TRY(wgrad(n, OUT, tv(n->d0, L0), tv(n->dz_out, 16), N, S0, S0));
    SUR_TRY(conv_back(n, OUT, tv(n->dz_out, 16), N, S0, S0, EPI_MASK_BF16, tv(A, L0), tv(n->d0, L0)));
    SUR_TRY(wgrad(n, D0B, tv(n->d0a, L0), tv(A, L0), N, S0, S0));
    SUR_TRY(conv_back(n, D0B, tv(A, L0), N, S0, S0, EPI_MASK_BF16, tv(B, L0), tv(n->d0a, L0)));
    SUR_TRY(wgrad(n, D0A, tv(n->c0, L1 + L0), tv(B, L0), N, S0, S0));
    // the input gradients of the decoders' first convolutions also give the upsampling
    // gradient of the level below (its share of the concatenation summed over 2 x 2
    // blocks, masked by the ReLU of the upsampled activation)
    SUR_TRY(conv_back(n, D0A, tv(B, L0), N, S0, S0, EPI_F32, none, none, n->dc0, L1 + L0, tv(A, L1), tv(n->d1, L1),
                      L1));
    // level 1 decoder
    SUR_TRY(wgrad(n, D1B, tv(n->d1a, L1), tv(A, L1), N, S1, S1));
    SUR_TRY(conv_back(n, D1B, tv(A, L1), N, S1, S1, EPI_MASK_BF16, tv(B, L1), tv(n->d1a, L1)));
    SUR_TRY(wgrad(n, D1A, tv(n->c1, L2 + L1), tv(B, L1), N, S1, S1));
    SUR_TRY(conv_back(n, D1A, tv(B, L1), N, S1, S1, EPI_F32, none, none, n->dc1, L2 + L1, tv(A, L2), tv(n->d2, L2),
                      L2));
    // level 2 decoder
    SUR_TRY(wgrad(n, D2B, tv(n->d2a, L2), tv(A, L2), N, S2, S2));
    SUR_TRY(conv_back(n, D2B, tv(A, L2), N, S2, S2, EPI_MASK_BF16, tv(B, L2), tv(n->d2a, L2)));
    SUR_TRY(wgrad(n, D2A, tv(n->c2, L3 + L2), tv(B, L2), N, S2, S2));
    SUR_TRY(conv_back(n, D2A, tv(B, L2), N, S2, S2, EPI_F32, none, none, n->dc2, L3 + L2, tv(A, L3), tv(n->e3, L3),
                      L3));
    // bottleneck
    SUR_TRY(wgrad(n, E3B, tv(n->e3a, L3), tv(A, L3), N, S3, S3));
    SUR_TRY(conv_back(n, E3B, tv(A, L3), N, S3, S3, EPI_MASK_BF16, tv(B, L3), tv(n->e3a, L3)));
    SUR_TRY(wgrad(n, E3A, tv(n->p2, L2), tv(B, L3), N, S3, S3));
    SUR_TRY(conv_back(n, E3A, tv(B, L3), N, S3, S3, EPI_F32, none, none, n->dp, L2));
    SUR_TRY(trace_dp(n, 0, N, S3, S3, L2));
    // level 2 encoder: skip share of dc2 plus the pooling gradient
    SUR_TRY(skip_grad(n->dc2, L3 + L2, L3, n->dp, L2, tv(n->c2, L3 + L2, L3), tv(A, L2), N, S2, S2, L2, n->stream));
    SUR_TRY(wgrad(n, E2B, tv(n->e2a, L2), tv(A, L2), N, S2, S2));
    SUR_TRY(conv_back(n, E2B, tv(A, L2), N, S2, S2, EPI_MASK_BF16, tv(B, L2), tv(n->e2a, L2)));
    SUR_TRY(wgrad(n, E2A, tv(n->p1, L1), tv(B, L2), N, S2, S2));
    SUR_TRY(conv_back(n, E2A, tv(B, L2), N, S2, S2, EPI_F32, none, none, n->dp, L1));
    SUR_TRY(trace_dp(n, 1, N, S2, S2, L1));
    // level 1 encoder
    SUR_TRY(skip_grad(n->dc1, L2 + L1, L2, n->dp, L1, tv(n->c1, L2 + L1, L2), tv(A, L1), N, S1, S1, L1, n->stream));
    SUR_TRY(wgrad(n, E1B, tv(n->e1a, L1), tv(A, L1), N, S1, S1));
    SUR_TRY(conv_back(n, E1B, tv(A, L1), N, S1, S1, EPI_MASK_BF16, tv(B, L1), tv(n->e1a, L1)));
    SUR_TRY(wgrad(n, E1A, tv(n->p0, L0), tv(B, L1), N, S1, S1));
    SUR_TRY(conv_back(n, E1A, tv(B, L1), N, S1, S1, EPI_F32, none, none, n->dp, L0));
    SUR_TRY(trace_dp(n, 2, N, S1, S1, L0));
    // level 0 encoder
    SUR_TRY(skip_grad(n->dc0, L1 + L0, L1, n->dp, L0, tv(n->c0, L1 + L0, L1), tv(A, L0), N, S0, S0, L0, n->stream));
    SUR_TRY(wgrad(n, E0B, tv(n->e0a, L0), tv(A, L0), N, S0, S0));
    SUR_TRY(conv_back(n, E0B, tv(A, L0), N, S0, S0, EPI_MASK_BF16, tv(B, L0), tv(n->e0a, L0)));
    SUR_TRY(wgrad(n, E0A, tv(n->x0, IN_PADDED), tv(B, L0), N, S0, S0));
    SUR_TRY(hipStreamSynchronize(n->stream));
    n->have_backward = true;
    if (loss) {
        double s = 0.0;
        for (int i = 0; i < MSE_BLOCKS; ++i) s += n->partial_host[i];
        *loss = s / double(cnt);
    }
    return LBM_OK;
}

lbm_status upload_batch(sur_net* n, const float* in, const float* target, int N) {
    const size_t px = (size_t)n->size * n->size;
    SUR_TRY(hipMemcpyAsync(n->in, in, (size_t)N * IN_CHANNELS * px * sizeof(float), hipMemcpyHostToDevice,
                           n->stream));
    if (target)
        SUR_TRY(hipMemcpyAsync(n->t, target, (size_t)N * px * sizeof(float), hipMemcpyHostToDevice, n->stream));
    SUR_TRY(pack_input(n->in, N, n->size, n->size, tv(n->x0, IN_PADDED), n->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status sur_create(int32_t size, int32_t max_batch, sur_net** out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (size < 8 || size % 8 || max_batch < 1 || (long long)size * size * max_batch > (1LL << 28)) return LBM_EINVAL;
    sur_net* n = new (std::nothrow) sur_net();
    if (!n) return LBM_ENOMEM;
    n->size = size;
    n->max_batch = max_batch;
    if (hipGetDevice(&n->device) != hipSuccess ||
        hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking) != hipSuccess) {
        release(n);
        return LBM_EHIP;
    }
    size_t off = 0, ex = 0, toff = 0;
    for (const LayerDef& d : LAYERS) {
        Layer l;
        l.d = d;
        l.cin_p = round_up(d.cin, 32);
        l.cout_p = round_up(d.cout, 16);
        l.w_off = off;
        off += 9 * (size_t)l.cout_p * l.cin_p;
        l.b_off = off;
        off += (size_t)l.cout_p;
        l.ex_w = ex;
        ex += (size_t)d.cout * d.cin * 9;
        l.ex_b = ex;
        ex += (size_t)d.cout;
        l.t_cout_p = round_up(d.cin, 16);
        l.t_cin_p = round_up(d.cout, 32);
        l.t_off = toff;
        toff += 9 * (size_t)l.t_cout_p * l.t_cin_p;
        n->L.push_back(l);
    }
    n->n_master = off;
    n->n_exchange = ex;
    n->n_flip = toff;
    const size_t B = max_batch, P0 = (size_t)size * size, P1 = P0 / 4, P2 = P0 / 16, P3 = P0 / 64;
    lbm_status st = LBM_OK;
    auto A16 = [&](uint16_t** p, size_t c) { if (st == LBM_OK) st = dalloc(n, p, c); };
    auto A32 = [&](float** p, size_t c) { if (st == LBM_OK) st = dalloc(n, p, c); };
    A32(&n->master, n->n_master);
    A32(&n->grad, n->n_master);
    A32(&n->m, n->n_master);
    A32(&n->v, n->n_master);
    A16(&n->wbf, n->n_master);
    A16(&n->wflip, n->n_flip);
    A16(&n->x0, B * P0 * IN_PADDED);
    A16(&n->e0a, B * P0 * L0);
    A16(&n->c0, B * P0 * (L1 + L0));
    A16(&n->p0, B * P1 * L0);
    A16(&n->e1a, B * P1 * L1);
    A16(&n->c1, B * P1 * (L2 + L1));
    A16(&n->p1, B * P2 * L1);
    A16(&n->e2a, B * P2 * L2);
    A16(&n->c2, B * P2 * (L3 + L2));
    A16(&n->p2, B * P3 * L2);
    A16(&n->e3a, B * P3 * L3);
    A16(&n->e3, B * P3 * L3);
    A16(&n->d2a, B * P2 * L2);
    A16(&n->d2, B * P2 * L2);
    A16(&n->d1a, B * P1 * L1);
    A16(&n->d1, B * P1 * L1);
    A16(&n->d0a, B * P0 * L0);
    A16(&n->d0, B * P0 * L0);
    A16(&n->dz_out, B * P0 * 16);
    A16(&n->dz_a, B * P0 * L0);  // the largest per-level gradient: level 0, 32 channels
    A16(&n->dz_b, B * P0 * L0);
    A32(&n->dc0, B * P0 * (L1 + L0));
    A32(&n->dc1, B * P1 * (L2 + L1));
    A32(&n->dc2, B * P2 * (L3 + L2));
    A32(&n->dp, B * P1 * L0);  // largest pooled gradient (level 1, 32 channels)
    A32(&n->y, B * P0);
    A32(&n->t, B * P0);
    A32(&n->in, B * P0 * IN_CHANNELS);
    if (st == LBM_OK) st = dalloc(n, &n->partial, MSE_BLOCKS);
    if (st == LBM_OK) st = dalloc(n, &n->idx, (size_t)max_batch);
    if (st == LBM_OK && hipHostMalloc(&n->partial_host, MSE_BLOCKS * sizeof(double), hipHostMallocDefault) != hipSuccess)
        st = LBM_EHIP;
    if (st == LBM_OK && hipStreamSynchronize(n->stream) != hipSuccess) st = LBM_EHIP;
    if (st != LBM_OK) {
        release(n);
        return st;
    }
    *out = n;
    return LBM_OK;
}

int64_t sur_param_count(const sur_net* n) { return n ? (int64_t)n->n_exchange : -1; }

lbm_status sur_set_params(sur_net* n, const float* params) {
    if (!n || !params) return LBM_EINVAL;
    for (int64_t i = 0; i < (int64_t)n->n_exchange; ++i)
        if (!std::isfinite(params[i])) return LBM_EINVAL;
    std::vector<float> h(n->n_master, 0.0f);
    for (const Layer& l : n->L) {
        for (int co = 0; co < l.d.cout; ++co) {
            for (int ci = 0; ci < l.d.cin; ++ci)
                for (int t = 0; t < 9; ++t)
                    h[l.w_off + ((size_t)t * l.cout_p + co) * l.cin_p + ci] = params[l.ex_w + ((size_t)co * l.d.cin + ci) * 9 + t];
            h[l.b_off + co] = params[l.ex_b + co];
        }
    }
    SUR_TRY(hipMemcpyAsync(n->master, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, n->stream));
    SUR_TRY(hipMemsetAsync(n->m, 0, n->n_master * sizeof(float), n->stream));
    SUR_TRY(hipMemsetAsync(n->v, 0, n->n_master * sizeof(float), n->stream));
    SUR_TRY(to_bf16(n->master, n->wbf, (long long)n->n_master, n->stream));
    SUR_TRY(refresh_flipped(n));
    SUR_TRY(hipStreamSynchronize(n->stream));
    n->adam_step = 0;
    return LBM_OK;
}

static lbm_status to_exchange(sur_net* n, const float* dev, float* out) {
    std::vector<float> h(n->n_master);
    SUR_TRY(hipMemcpyAsync(h.data(), dev, h.size() * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    SUR_TRY(hipStreamSynchronize(n->stream));
    for (const Layer& l : n->L)
        for (int co = 0; co < l.d.cout; ++co) {
            for (int ci = 0; ci < l.d.cin; ++ci)
                for (int t = 0; t < 9; ++t)
                    out[l.ex_w + ((size_t)co * l.d.cin + ci) * 9 + t] = h[l.w_off + ((size_t)t * l.cout_p + co) * l.cin_p + ci];
            out[l.ex_b + co] = h[l.b_off + co];
        }
    return LBM_OK;
}

lbm_status sur_get_params(sur_net* n, float* params) {
    if (!n || !params) return LBM_EINVAL;
    return to_exchange(n, n->master, params);
}

lbm_status sur_forward(sur_net* n, const float* in, int32_t count, float* out) {
    if (!n || !in || !out || count < 1) return LBM_EINVAL;
    if (hipSetDevice(n->device) != hipSuccess) return LBM_EHIP;
    const size_t px = (size_t)n->size * n->size;
    for (int32_t b0 = 0; b0 < count; b0 += n->max_batch) {
        const int N = std::min(n->max_batch, count - b0);
        lbm_status st = upload_batch(n, in + (size_t)b0 * IN_CHANNELS * px, nullptr, N);
        if (st != LBM_OK) return st;
        st = forward(n, N);
        if (st != LBM_OK) return st;
        SUR_TRY(hipMemcpyAsync(out + (size_t)b0 * px, n->y, (size_t)N * px * sizeof(float), hipMemcpyDeviceToHost,
                               n->stream));
        SUR_TRY(hipStreamSynchronize(n->stream));
    }
    return LBM_OK;
}

lbm_status sur_gradients(sur_net* n, const float* in, const float* target, int32_t count, float* grads,
                         double* loss) {
    if (!n || !in || !target || count < 1 || count > n->max_batch) return LBM_EINVAL;
    if (hipSetDevice(n->device) != hipSuccess) return LBM_EHIP;
    lbm_status st = upload_batch(n, in, target, count);
    if (st == LBM_OK) st = forward(n, count);
    if (st == LBM_OK) st = backward(n, count, loss);
    if (st == LBM_OK && grads) st = to_exchange(n, n->grad, grads);
    return st;
}

lbm_status sur_set_dataset(sur_net* n, const float* inputs, const float* targets, int32_t count) {
    if (!n || !inputs || !targets || count < 1) return LBM_EINVAL;
    if (hipSetDevice(n->device) != hipSuccess) return LBM_EHIP;
    const size_t px = (size_t)n->size * n->size;
    if (n->ds_in) {
        (void)hipFree(n->ds_in);
        (void)hipFree(n->ds_t);
        n->ds_in = n->ds_t = nullptr;
    }
    if (hipMalloc(&n->ds_in, (size_t)count * IN_CHANNELS * px * sizeof(float)) != hipSuccess) return LBM_ENOMEM;
    if (hipMalloc(&n->ds_t, (size_t)count * px * sizeof(float)) != hipSuccess) return LBM_ENOMEM;
    SUR_TRY(hipMemcpyAsync(n->ds_in, inputs, (size_t)count * IN_CHANNELS * px * sizeof(float), hipMemcpyHostToDevice,
                           n->stream));
    SUR_TRY(hipMemcpyAsync(n->ds_t, targets, (size_t)count * px * sizeof(float), hipMemcpyHostToDevice, n->stream));
    SUR_TRY(hipStreamSynchronize(n->stream));
    n->ds_count = count;
    return LBM_OK;
}

lbm_status sur_train(sur_net* n, int32_t steps, int32_t batch, float lr, uint64_t seed, float* losses) {
    if (!n || steps < 0 || batch < 1 || batch > n->max_batch || !(lr > 0) || n->ds_count < 1) return LBM_EINVAL;
    if (hipSetDevice(n->device) != hipSuccess) return LBM_EHIP;
    const size_t px = (size_t)n->size * n->size;
    std::vector<int> idx(batch);
    uint64_t state = seed;
    for (int32_t s = 0; s < steps; ++s) {
        for (int b = 0; b < batch; ++b) {  // SplitMix64 draws of the minibatch
            state += 0x9E3779B97F4A7C15ull;
            uint64_t z = state;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            idx[b] = int(z % (uint64_t)n->ds_count);
        }
        SUR_TRY(hipMemcpyAsync(n->idx, idx.data(), batch * sizeof(int), hipMemcpyHostToDevice, n->stream));
        SUR_TRY(gather_rows(n->ds_in, n->idx, (long long)IN_CHANNELS * px, batch, n->in, n->stream));
        SUR_TRY(gather_rows(n->ds_t, n->idx, (long long)px, batch, n->t, n->stream));
        SUR_TRY(pack_input(n->in, batch, n->size, n->size, tv(n->x0, IN_PADDED), n->stream));
        lbm_status st = forward(n, batch);
        if (st != LBM_OK) return st;
        double loss = 0.0;
        st = backward(n, batch, &loss);
        if (st != LBM_OK) return st;
        ++n->adam_step;
        SUR_TRY(adam(n->master, n->grad, n->m, n->v, n->wbf, (long long)n->n_master, lr, n->adam_step, n->stream));
        SUR_TRY(refresh_flipped(n));
        if (losses) losses[s] = float(loss);
    }
    SUR_TRY(hipStreamSynchronize(n->stream));
    return LBM_OK;
}

lbm_status sur_trace(sur_net* n, int32_t on) {
    if (!n) return LBM_EINVAL;
    if (hipSetDevice(n->device) != hipSuccess) return LBM_EHIP;
    SUR_TRY(hipStreamSynchronize(n->stream));
    if (!on) {
        free_trace(n);
        return LBM_OK;
    }
    if (n->trace) return LBM_OK;
    const size_t B = n->max_batch, P0 = (size_t)n->size * n->size;
    const int level[NL] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0};
    for (int li = 0; li < NL; ++li) {
        const size_t px = B * (P0 >> (2 * level[li]));
        const size_t ch = li == OUT ? 16 : (size_t)LAYERS[li].cout;  // the output gradient's buffer width
        if (hipMalloc(&n->trace_dz[li], px * ch * sizeof(uint16_t)) != hipSuccess) {
            free_trace(n);
            return LBM_ENOMEM;
        }
    }
    const size_t dp_px[3] = {B * (P0 >> 6), B * (P0 >> 4), B * (P0 >> 2)};
    const int dp_ch[3] = {L2, L1, L0};
    for (int k = 0; k < 3; ++k)
        if (hipMalloc(&n->trace_dp[k], dp_px[k] * dp_ch[k] * sizeof(float)) != hipSuccess) {
            free_trace(n);
            return LBM_ENOMEM;
        }
    n->trace = true;
    return LBM_OK;
}

lbm_status sur_read(sur_net* n, const char* name, float* out, int64_t capacity, int64_t* shape) {
    if (!n || !name || !shape) return LBM_EINVAL;
    const int N = n->last_N;
    if (N < 1) return LBM_ESTATE;
    const int S0 = n->size, S1 = S0 / 2, S2 = S0 / 4, S3 = S0 / 8;
    struct Entry {
        const char* name;
        const void* p;
        int side, ch;
        bool f32, needs_backward;
    };
    const Entry fwd[] = {
        {"x0", n->x0, S0, IN_PADDED, false, false}, {"e0a", n->e0a, S0, L0, false, false},
        {"c0", n->c0, S0, L1 + L0, false, false},   {"p0", n->p0, S1, L0, false, false},
        {"e1a", n->e1a, S1, L1, false, false},      {"c1", n->c1, S1, L2 + L1, false, false},
        {"p1", n->p1, S2, L1, false, false},        {"e2a", n->e2a, S2, L2, false, false},
        {"c2", n->c2, S2, L3 + L2, false, false},   {"p2", n->p2, S3, L2, false, false},
        {"e3a", n->e3a, S3, L3, false, false},      {"e3", n->e3, S3, L3, false, false},
        {"d2a", n->d2a, S2, L2, false, false},      {"d2", n->d2, S2, L2, false, false},
        {"d1a", n->d1a, S1, L1, false, false},      {"d1", n->d1, S1, L1, false, false},
        {"d0a", n->d0a, S0, L0, false, false},      {"d0", n->d0, S0, L0, false, false},
        {"y", n->y, S0, 1, true, false},            {"dc0", n->dc0, S0, L1 + L0, true, true},
        {"dc1", n->dc1, S1, L2 + L1, true, true},   {"dc2", n->dc2, S2, L3 + L2, true, true},
    };
    const int side_of[NL] = {S0, S0, S1, S1, S2, S2, S3, S3, S2, S2, S1, S1, S0, S0, S0};
    Entry e{nullptr, nullptr, 0, 0, false, false};
    for (const Entry& f : fwd)
        if (std::strcmp(f.name, name) == 0) e = f;
    if (!e.name && std::strncmp(name, "dz_", 3) == 0) {
        for (int li = 0; li < NL; ++li)
            if (std::strcmp(name + 3, LAYERS[li].name) == 0)
                e = Entry{name, n->trace_dz[li], side_of[li], li == OUT ? 16 : LAYERS[li].cout, false, true};
    }
    const char* dp_names[3] = {"dp_e3a", "dp_e2a", "dp_e1a"};
    const int dp_side[3] = {S3, S2, S1}, dp_ch[3] = {L2, L1, L0};
    for (int k = 0; k < 3 && !e.name; ++k)
        if (std::strcmp(name, dp_names[k]) == 0) e = Entry{name, n->trace_dp[k], dp_side[k], dp_ch[k], true, true};
    if (!e.name) return LBM_EINVAL;
    if (e.needs_backward && !n->have_backward) return LBM_ESTATE;
    if (!e.p) return LBM_ESTATE;  // a traced tensor while tracing is off
    shape[0] = N;
    shape[1] = e.side;
    shape[2] = e.side;
    shape[3] = e.ch;
    const size_t count = (size_t)N * e.side * e.side * e.ch;
    if (!out) return LBM_OK;
    if (capacity < (int64_t)count) return LBM_EINVAL;
    if (hipSetDevice(n->device) != hipSuccess) return LBM_EHIP;
    if (e.f32) {
        SUR_TRY(hipMemcpyAsync(out, e.p, count * sizeof(float), hipMemcpyDeviceToHost, n->stream));
        SUR_TRY(hipStreamSynchronize(n->stream));
    } else {
        std::vector<uint16_t> h(count);
        SUR_TRY(hipMemcpyAsync(h.data(), e.p, count * sizeof(uint16_t), hipMemcpyDeviceToHost, n->stream));
        SUR_TRY(hipStreamSynchronize(n->stream));
        for (size_t i = 0; i < count; ++i) {  // a BF16 value is the top half of an FP32
            const uint32_t bits = uint32_t(h[i]) << 16;
            std::memcpy(out + i, &bits, sizeof bits);
        }
    }
    return LBM_OK;
}

void sur_destroy(sur_net* n) {
    if (!n) return;
    (void)hipSetDevice(n->device);
    (void)hipStreamSynchronize(n->stream);
    if (n->ds_in) (void)hipFree(n->ds_in);
    if (n->ds_t) (void)hipFree(n->ds_t);
    release(n);
}

}  // extern "C"
