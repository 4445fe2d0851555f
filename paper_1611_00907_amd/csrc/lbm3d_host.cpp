// C ABI of the D3Q19 step (declared in lbm.h): a periodic box advanced by the
// density and step passes of lbm3d_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <new>

#include "lbm3d_internal.h"
#include "lbm_common.h"

using namespace cplbm;
using namespace cplbm::host;

struct lbm3d {
    lbm_params p;
    int nz = 0;
    d3::Args3 A{};
    int device = 0;
    hipStream_t stream = nullptr;
    void* ws = nullptr;
    void* f[2] = {nullptr, nullptr};
    void* rho = nullptr;
    int cur = 0;
    int64_t step = 0;
};

namespace {

lbm_status validate3(const lbm_params* p, int32_t nz) {
    if (!p || nz < 1) return LBM_EINVAL;
    lbm_params q = *p;
    q.ny = 3;  // a 2-D check of everything but the box size
    if (validate(&q) != LBM_OK) return LBM_EINVAL;
    if (p->ny < 1 || p->bc_bottom != LBM_BC_PERIODIC || p->bc_top != LBM_BC_PERIODIC) return LBM_EINVAL;
    if (p->prec != LBM_F64 && p->prec != LBM_F32) return LBM_EINVAL;
    if (p->scheme != 0) return LBM_EINVAL;
    const long long pitch = ((long long)p->nx + 63) / 64 * 64;
    // node indices and plane offsets are 32-bit, and so are the byte offsets in one
    // z slice of one direction
    if ((long long)p->nx * p->ny * nz >= (1LL << 31) || pitch * p->ny * nz >= (1LL << 31)) return LBM_EINVAL;
    if (pitch * p->ny * (p->prec == LBM_F64 ? 8 : 4) >= (1LL << 32)) return LBM_EINVAL;
    return LBM_OK;
}

void release3(lbm3d* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamDestroy(c->stream);
    if (c->ws) (void)hipFree(c->ws);
    delete c;
}

}  // namespace

extern "C" {

lbm_status lbm3d_init(const lbm_params* p, int32_t nz, const double* rho0, lbm3d** out) {
    if (!out || !rho0) return LBM_EINVAL;
    *out = nullptr;
    lbm_status st = validate3(p, nz);
    if (st != LBM_OK) return st;
    const thermo::Fluid fl = thermo::make_fluid(p->eos, p->a, p->b, p->R, p->Tr, p->omega);
    if (!(std::isfinite(fl.T) && fl.T > 0 && std::isfinite(fl.alpha))) return LBM_EINVAL;
    const size_t n = (size_t)p->nx * p->ny * nz;
    const double pole = thermo::rho_pole(p->eos, p->b);
    for (size_t i = 0; i < n; ++i)
        if (!(std::isfinite(rho0[i]) && rho0[i] > 0 && rho0[i] < pole)) return LBM_EDOMAIN;
    lbm3d* c = new (std::nothrow) lbm3d();
    if (!c) return LBM_ENOMEM;
    c->p = *p;
    c->nz = nz;
    const int pitch = (p->nx + 63) / 64 * 64;
    // the 2-D lattice arguments give the EOS constants at T = Tr Tc
    lbm_params q = *p;
    q.ny = 3;
    const LatticeArgs A2 = lattice_args(q, fl, layout_of(q));
    d3::Args3& A = c->A;
    A.nx = p->nx;
    A.ny = p->ny;
    A.nz = nz;
    A.pitch = pitch;
    A.plane = (long long)pitch * p->ny * nz;
    A.tau = p->tau;
    A.inv_tau = 1.0 / p->tau;
    A.kappa = p->kappa;
    A.eos = A2.eos;
    const size_t sb = storage_bytes(p->prec);
    const size_t fbytes = align256(19 * size_t(A.plane) * sb), rbytes = align256(size_t(A.plane) * sb);
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        release3(c);
        return hip_status(e, "lbm3d_init stream");
    }
    if (hipMalloc(&c->ws, 2 * fbytes + rbytes) != hipSuccess) {
        c->ws = nullptr;
        release3(c);
        return LBM_ENOMEM;
    }
    c->f[0] = c->ws;
    c->f[1] = static_cast<char*>(c->ws) + fbytes;
    c->rho = static_cast<char*>(c->ws) + 2 * fbytes;
    double* staging = nullptr;
    e = hipMemsetAsync(c->ws, 0, 2 * fbytes + rbytes, c->stream);
    if (e == hipSuccess) e = hipMalloc(&staging, n * sizeof(double));
    if (e == hipSuccess) e = hipMemcpyAsync(staging, rho0, n * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = d3::launch_init3(p->prec, A, staging, nullptr, c->f[0], c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (staging) (void)hipFree(staging);
    if (e != hipSuccess) {
        release3(c);
        return hip_status(e, "lbm3d_init");
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm3d_step(lbm3d* c, int64_t n) {
    if (!c || n < 0) return LBM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    for (int64_t s = 0; s < n; ++s) {
        HIP_TRY(d3::launch_step3(c->p.prec, c->p.eos, 0, c->A, c->f[c->cur], c->rho, c->f[c->cur ^ 1], nullptr,
                                 c->stream));
        c->cur ^= 1;
        ++c->step;
    }
    return LBM_OK;
}

lbm_status lbm3d_step_timed(lbm3d* c, int64_t n, double* ms) {
    if (!c || n < 0 || !ms) return LBM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    hipEvent_t a = nullptr, b = nullptr;
    lbm_status st = LBM_OK;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipEventRecord(a, c->stream);
    if (e == hipSuccess) st = lbm3d_step(c, n);
    if (e == hipSuccess) e = hipEventRecord(b, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_status(e, "lbm3d_step_timed");
    *ms = t;
    return st;
}

lbm_status lbm3d_get_fields(lbm3d* c, double* rho, double* vx, double* vy, double* vz, double* mu) {
    if (!c) return LBM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    const size_t n = (size_t)c->A.nx * c->A.ny * c->A.nz;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, 5 * n * sizeof(double)));
    hipError_t e = d3::launch_step3(c->p.prec, c->p.eos, 1, c->A, c->f[c->cur], c->rho, nullptr, d, c->stream);
    double* outs[5] = {rho, vx, vy, vz, mu};
    for (int k = 0; k < 5 && e == hipSuccess; ++k)
        if (outs[k]) e = hipMemcpyAsync(outs[k], d + k * n, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    return hip_status(e, "lbm3d_get_fields");
}

lbm_status lbm3d_get_state(lbm3d* c, double* f, int64_t* step) {
    if (!c || !f) return LBM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    const size_t n = 19 * (size_t)c->A.nx * c->A.ny * c->A.nz;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, n * sizeof(double)));
    hipError_t e = d3::launch_state3(c->p.prec, c->A, c->f[c->cur], d, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e == hipSuccess && step) *step = c->step;
    return hip_status(e, "lbm3d_get_state");
}

void lbm3d_destroy(lbm3d* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    release3(c);
}

}  // extern "C"
