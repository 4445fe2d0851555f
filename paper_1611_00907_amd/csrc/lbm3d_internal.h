// Internal interface between the host library and the D3Q19 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace cplbm {
namespace d3 {

// One periodic D3Q19 box, as the kernels see it; passed by value.
struct Args3 {
    int nx, ny, nz;
    int pitch;        // elements per x row (a multiple of 64)
    long long plane;  // elements per direction plane = nz * ny * pitch
    double tau, inv_tau, kappa;
    EosConst eos;
};

// One step (mode 0: fin -> fout, rho is the density buffer the step writes and
// reads) or the field output (mode 1: out = [5][nz][ny][nx] rho, vx, vy, vz, mu).
hipError_t launch_step3(int prec, int eos, int mode, const Args3& A, const void* fin, void* rho, void* fout,
                        double* out, hipStream_t s);
// Storage form of f = f_eq(rho0, 0) (f_in null) or of the given post-streaming f.
hipError_t launch_init3(int prec, const Args3& A, const double* rho0, const double* f_in, void* fs, hipStream_t s);
// Post-streaming f(t) [19][nz][ny][nx] from the storage.
hipError_t launch_state3(int prec, const Args3& A, const void* fs, double* f_out, hipStream_t s);

}  // namespace d3
}  // namespace cplbm
