// Host-side helpers shared by the single-lattice and the batched C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm.h"
#include "lbm_internal.h"
#include "thermo_host.h"

namespace cplbm {
namespace host {

constexpr int PITCH_ALIGN = 64;

struct Layout {
    int pitch;
    long long plane;
    size_t f0, f1, rho_mon, mu_w, partials, mon, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
// Non-temporal stores of f*(t) for distribution buffers (both together, `bytes`)
// larger than the 256 MB Infinity Cache; measured at 4096^2 FP32 (1.2 GB): 7 %
// faster; at 1024^2 (75 MB, cache-resident) up to 40 % slower, so plain stores there.
constexpr long long NT_STORE_MIN_BYTES = 256LL << 20;
inline int nt_store_for(long long bytes) { return bytes > NT_STORE_MIN_BYTES ? 1 : 0; }
inline bool walled(const lbm_params& p) { return p.bc_bottom != LBM_BC_PERIODIC; }
inline bool is_solid_row(const lbm_params& p, int y) { return walled(p) && (y == 0 || y == p.ny - 1); }

lbm_status validate(const lbm_params* p);
Layout layout_of(const lbm_params& p);
LatticeArgs lattice_args(const lbm_params& p, const thermo::Fluid& fl, const Layout& L);
// Checks the fluid nodes of rho0 (and u0 when given) against the EOS domain.
lbm_status check_initial(const lbm_params& p, const double* rho0, const double* ux0, const double* uy0);
// Uploads rho0/u0 and writes f = f_eq(rho0, u0) in storage form into fstore.
lbm_status init_state(const lbm_params& p, const LatticeArgs& A, const double* rho0, const double* ux0,
                      const double* uy0, void* fstore, hipStream_t s);
// Converts [2][nx] host wall values into the device [2][pitch] array in the compute type.
lbm_status upload_mu_w(const lbm_params& p, int pitch, const double* mu_w_host, void* mu_w_dev, hipStream_t s);

void note_error(hipError_t e, const char* where);
lbm_status hip_status(hipError_t e, const char* where);

}  // namespace host
}  // namespace cplbm

#define HIP_TRY(expr)                                     \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) {                           \
            ::cplbm::host::note_error(e_, #expr);         \
            return LBM_EHIP;                              \
        }                                                 \
    } while (0)
