// Dispatch of the kernel entry points over the storage type: lbm_kernels.hip is
// compiled once per type (f64, f32, f16dev, bf16dev) into separate objects.
#include "lbm_internal.h"

namespace cplbm {

#define CPLBM_DECLARE(sfx)                                                                                      \
    hipError_t launch_step_##sfx(int, int, const LatticeArgs&, const void*, void*, const void*, double*,       \
                                 hipStream_t);                                                                 \
    hipError_t launch_monitor_##sfx(int, const LatticeArgs&, const void*, void*, double*, double*, hipStream_t); \
    hipError_t launch_batch_step_##sfx(int, int, const CaseDesc*, const int2*, int, int, int, hipStream_t);     \
    hipError_t launch_batch_monitor_##sfx(int, int, const CaseDesc*, const int2*, int, int, double*, const int*, \
                                          int, double*, hipStream_t);                                          \
    int batch_blocks_per_cu_##sfx(int);                                                                        \
    hipError_t launch_init_##sfx(const LatticeArgs&, const double*, const double*, const double*, const double*, \
                                 void*, hipStream_t);                                                          \
    hipError_t launch_get_state_##sfx(const LatticeArgs&, const void*, double*, hipStream_t);

CPLBM_DECLARE(f64)
CPLBM_DECLARE(f32)
CPLBM_DECLARE(f16dev)
CPLBM_DECLARE(bf16dev)

size_t storage_bytes(int prec) { return prec == PREC_F64 ? 8 : (prec == PREC_F32 ? 4 : 2); }
size_t compute_bytes(int prec) { return prec == PREC_F64 ? 8 : 4; }

hipError_t launch_step(int prec, int eos, int mode, const LatticeArgs& A, const void* fin, void* fout,
                       const void* mu_w, double* out, hipStream_t s) {
    switch (prec) {
    case PREC_F64: return launch_step_f64(eos, mode, A, fin, fout, mu_w, out, s);
    case PREC_F32: return launch_step_f32(eos, mode, A, fin, fout, mu_w, out, s);
    case PREC_F16DEV: return launch_step_f16dev(eos, mode, A, fin, fout, mu_w, out, s);
    case PREC_BF16DEV: return launch_step_bf16dev(eos, mode, A, fin, fout, mu_w, out, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_monitor(int prec, int eos, int compare, const LatticeArgs& A, const void* fin, void* rho_mon,
                          double* partials, double* mon, hipStream_t s) {
    (void)eos;
    switch (prec) {
    case PREC_F64: return launch_monitor_f64(compare, A, fin, rho_mon, partials, mon, s);
    case PREC_F32: return launch_monitor_f32(compare, A, fin, rho_mon, partials, mon, s);
    case PREC_F16DEV: return launch_monitor_f16dev(compare, A, fin, rho_mon, partials, mon, s);
    case PREC_BF16DEV: return launch_monitor_bf16dev(compare, A, fin, rho_mon, partials, mon, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_step(int prec, int tile_y, int nt, const CaseDesc* cases, const int2* tiles, int ntiles,
                             int parity, int grid, hipStream_t s) {
    switch (prec) {
    case PREC_F64: return launch_batch_step_f64(tile_y, nt, cases, tiles, ntiles, parity, grid, s);
    case PREC_F32: return launch_batch_step_f32(tile_y, nt, cases, tiles, ntiles, parity, grid, s);
    case PREC_F16DEV: return launch_batch_step_f16dev(tile_y, nt, cases, tiles, ntiles, parity, grid, s);
    case PREC_BF16DEV: return launch_batch_step_bf16dev(tile_y, nt, cases, tiles, ntiles, parity, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_monitor(int prec, int compare, int tile_y, const CaseDesc* cases, const int2* tiles,
                                int ntiles, int parity, double* partials, const int* case_tile_begin, int ncases,
                                double* case_mon, hipStream_t s) {
    switch (prec) {
    case PREC_F64:
        return launch_batch_monitor_f64(compare, tile_y, cases, tiles, ntiles, parity, partials, case_tile_begin,
                                        ncases, case_mon, s);
    case PREC_F32:
        return launch_batch_monitor_f32(compare, tile_y, cases, tiles, ntiles, parity, partials, case_tile_begin,
                                        ncases, case_mon, s);
    case PREC_F16DEV:
        return launch_batch_monitor_f16dev(compare, tile_y, cases, tiles, ntiles, parity, partials,
                                           case_tile_begin, ncases, case_mon, s);
    case PREC_BF16DEV:
        return launch_batch_monitor_bf16dev(compare, tile_y, cases, tiles, ntiles, parity, partials,
                                            case_tile_begin, ncases, case_mon, s);
    default: return hipErrorInvalidValue;
    }
}

int batch_blocks_per_cu(int prec, int tile_y) {
    switch (prec) {
    case PREC_F64: return batch_blocks_per_cu_f64(tile_y);
    case PREC_F32: return batch_blocks_per_cu_f32(tile_y);
    case PREC_F16DEV: return batch_blocks_per_cu_f16dev(tile_y);
    default: return batch_blocks_per_cu_bf16dev(tile_y);
    }
}

hipError_t launch_init(int prec, const LatticeArgs& A, const double* rho0, const double* ux0, const double* uy0,
                       const double* f_in, void* fstore, hipStream_t s) {
    switch (prec) {
    case PREC_F64: return launch_init_f64(A, rho0, ux0, uy0, f_in, fstore, s);
    case PREC_F32: return launch_init_f32(A, rho0, ux0, uy0, f_in, fstore, s);
    case PREC_F16DEV: return launch_init_f16dev(A, rho0, ux0, uy0, f_in, fstore, s);
    case PREC_BF16DEV: return launch_init_bf16dev(A, rho0, ux0, uy0, f_in, fstore, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_get_state(int prec, const LatticeArgs& A, const void* fstore, double* f_out, hipStream_t s) {
    switch (prec) {
    case PREC_F64: return launch_get_state_f64(A, fstore, f_out, s);
    case PREC_F32: return launch_get_state_f32(A, fstore, f_out, s);
    case PREC_F16DEV: return launch_get_state_f16dev(A, fstore, f_out, s);
    case PREC_BF16DEV: return launch_get_state_bf16dev(A, fstore, f_out, s);
    default: return hipErrorInvalidValue;
    }
}

// Plain streaming copy (16-byte vector loads and stores, four in flight per
// thread, grid-stride): the reference for measured bandwidth and for calibrating
// memory counters.
// One 16-byte vector per thread, no loop: the simplest form of a streaming copy and
// the fastest one measured on this part (a grid-stride loop issues fewer requests
// per wave and reaches about 70 % of its bandwidth).
__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                   long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const long long n = (long long)(bytes / sizeof(float4));
    const long long blocks = (n + 255) / 256;
    if (blocks < 1 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    (void)hipGetLastError();
    hipLaunchKernelGGL(copy_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, (const float4*)src, (float4*)dst, n);
    return hipGetLastError();
}

}  // namespace cplbm
