// Device-side equations of state (Sec. III): the bulk chemical potential psi'(rho)
// of Eqs 18, 21, 24, 27 and the bulk pressure p0(rho) of Eqs 16, 19, 22, 25, in the
// compute type (FP32 with the hardware log2 and reciprocal, about 1 ulp; FP64 with
// the library logarithm and correctly rounded division).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace cplbm {
namespace eosd {

__device__ __forceinline__ float lg(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ __forceinline__ double lg(double x) { return log(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

// psi'(rho): Eq 18 (VdW), Eq 27 (CS), Eq 24 (PR), Eq 21 (RK, RKS).
template <int EOS, typename CT>
__device__ __forceinline__ CT mu_bulk(const EosConst& E, CT rho) {
    const CT RT = CT(E.RT), a = CT(E.a), b = CT(E.b), c1 = CT(E.c1);
    if constexpr (EOS == EOS_CS) {
        const CT q = c1 * rho, om = CT(1) - q;
        return RT * ((CT(3) - q) * rcp(om * om * om) + lg(rho) + CT(1)) - CT(2) * a * rho;
    } else {
        const CT br = b * rho, ib = rcp(CT(1) - br);
        const CT rep = RT * (lg(rho * ib) + ib);
        if constexpr (EOS == EOS_VDW) {
            return rep - CT(2) * a * rho;
        } else if constexpr (EOS == EOS_PR) {
            const CT s2 = CT(1.4142135623730950488);
            return rep - c1 * lg((s2 - CT(1) + br) * rcp(s2 + CT(1) - br)) - a * rho * rcp(CT(1) + CT(2) * br - br * br);
        } else {  // RK, RKS
            return rep - c1 * lg(CT(1) + br) - a * rho * rcp(CT(1) + br);
        }
    }
}

}  // namespace eosd
}  // namespace cplbm
