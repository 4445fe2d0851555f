// HIP kernels of the chemical-potential lattice Boltzmann step for CDNA4 (gfx950).
//
// Storage: the post-collision distributions f*(t-1) as nine rows of one direction
// each per lattice row, f[y][i][x] (row pitch a multiple of 64 elements), or as
// nine direction planes f[i][y][x] where a buffer is too large for 32-bit byte
// offsets; the kernels see either through two strides (direction and row).  A step pulls
// f_i(x, t) = f*_i(x - e_i, t-1), or the reflected f*_opp(i)(x, t-1) when x - e_i
// lies in a solid row (halfway bounce-back, Sec. IV), so reads are the shifted
// ones and every write is aligned and coalesced.  Two such buffers alternate.
//
// One workgroup owns a TILE_X x TILE_Y tile.  It pulls the nodes of the tile and of
// a two-node ring around it, sums their densities into LDS (the ring is redundant
// work that neighbouring tiles also do: it replaces a separate density pass and a
// second trip through HBM), evaluates the chemical potential of Eq 8 on the tile
// plus a one-node ring in LDS, then forms the force of Eq 12, collides (Eqs 13,
// 14 with u + tau F / rho) and writes the tile.  Wall rows get their density from
// Eq 28 and their chemical potential from the surface value (Sec. IV) or from the
// neighbouring fluid node (Sec. V).
#include <algorithm>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lbm_internal.h"

#ifndef CPLBM_ST
#error "compile this file once per storage type: -DCPLBM_ST=float -DCPLBM_SUFFIX=f32, ..."
#endif

namespace cplbm {
namespace {

// ---------------------------------------------------------------- storage codecs
// Offsets are element indices within one direction plane.  They are turned into
// 32-bit byte offsets from the plane's (uniform) base, so loads and stores take a
// scalar base plus one 32-bit vector offset; the host keeps every plane below
// 4 GiB.
template <typename T>
__device__ __forceinline__ const T* at(const T* p, unsigned o) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + (o * unsigned(sizeof(T))));
}
template <typename T>
__device__ __forceinline__ T* at(T* p, unsigned o) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(p) + (o * unsigned(sizeof(T))));
}

// A pointer read from memory (a batch's case descriptors) is generic to the
// compiler, which then emits flat accesses (counted against both the vector-memory
// and the LDS counters, so every LDS wait also waits for memory).  Rebuilding it
// from its bits as a global-address-space pointer lets the compiler use global
// accesses again (a plain cast pair folds away).
template <typename T>
__device__ __forceinline__ T* in_global(T* p) {
    typedef __attribute__((address_space(1))) T* GP;
    return (T*)(GP)__builtin_bit_cast(unsigned long long, p);
}

template <typename ST>
struct Codec;

// stn: the step's stores of f*(t), marked non-temporal, for lattices larger than the
// caches (read back only in the next step, after the whole lattice has streamed
// through, they need not displace the lines that neighbouring tiles are about to
// re-read); a lattice that stays in the Infinity Cache keeps plain stores.
template <>
struct Codec<double> {
    using CT = double;
    static __device__ __forceinline__ double ld(const double* p, unsigned o, double) { return *at(p, o); }
    static __device__ __forceinline__ void st(double* p, unsigned o, double v, double) { *at(p, o) = v; }
    static __device__ __forceinline__ void stn(double* p, unsigned o, double v, double) {
        __builtin_nontemporal_store(v, at(p, o));
    }
};
template <>
struct Codec<float> {
    using CT = float;
    static __device__ __forceinline__ float ld(const float* p, unsigned o, float) { return *at(p, o); }
    static __device__ __forceinline__ void st(float* p, unsigned o, float v, float) { *at(p, o) = v; }
    static __device__ __forceinline__ void stn(float* p, unsigned o, float v, float) {
        __builtin_nontemporal_store(v, at(p, o));
    }
};
// Deviation storage: h = f - w_i rho_ref, rounded to nearest even on store.
template <>
struct Codec<__half> {
    using CT = float;
    static __device__ __forceinline__ float ld(const __half* p, unsigned o, float base) {
        return __half2float(*at(p, o)) + base;
    }
    static __device__ __forceinline__ void st(__half* p, unsigned o, float v, float base) {
        *at(p, o) = __float2half_rn(v - base);
    }
    static __device__ __forceinline__ void stn(__half* p, unsigned o, float v, float base) {
        __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v - base)),
                                    reinterpret_cast<unsigned short*>(at(p, o)));
    }
};
template <>
struct Codec<__hip_bfloat16> {
    using CT = float;
    static __device__ __forceinline__ float ld(const __hip_bfloat16* p, unsigned o, float base) {
        return __bfloat162float(*at(p, o)) + base;
    }
    static __device__ __forceinline__ void st(__hip_bfloat16* p, unsigned o, float v, float base) {
        *at(p, o) = __float2bfloat16(v - base);
    }
    static __device__ __forceinline__ void stn(__hip_bfloat16* p, unsigned o, float v, float base) {
        __builtin_nontemporal_store(__bfloat16_as_ushort(__float2bfloat16(v - base)),
                                    reinterpret_cast<unsigned short*>(at(p, o)));
    }
};

// FP32 arithmetic uses the hardware log2 and reciprocal (about 1 ulp); FP64 keeps
// the correctly rounded division and the library logarithm.
__device__ __forceinline__ float lg(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ __forceinline__ double lg(double x) { return log(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

// D2Q9 weights (Eq 14 coefficients imply c_s^2 = 1/3): rest, axis, diagonal.
template <typename CT>
struct Wt {
    static constexpr CT w0 = CT(4) / CT(9), w1 = CT(1) / CT(9), w2 = CT(1) / CT(36);
};

// ---------------------------------------------------------------- lattice helpers
__device__ __forceinline__ int wrap_fast(int v, int n, bool small) {
    if (small) {
        v %= n;
        return v < 0 ? v + n : v;
    }
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// Row 0 / row ny-1 are solid when the lattice has walls.
__device__ __forceinline__ bool solid_row(const LatticeArgs& A, int y) {
    return A.bottom != BC_PERIODIC && (y == 0 || y == A.ny - 1);
}

template <typename ST>
struct Planes {
    const ST* p[9];
};

// f_i(x, t), i = 0..8, of a fluid node (gx, gy) by pulling from the storage.
// With UNIFORM_ROW the caller guarantees that gy is the same in all lanes of the
// wave: the row, and with it the choice of source planes, is then scalar, so each
// load takes a scalar base and one 32-bit lane offset.
template <typename ST, typename CT, bool UNIFORM_ROW = false>
__device__ __forceinline__ void pull9(const LatticeArgs& A, const Planes<ST>& F, int gx, int gy,
                                      CT f[9]) {
    if (UNIFORM_ROW) gy = __builtin_amdgcn_readfirstlane(gy);
    using C = Codec<ST>;
    const CT b0 = CT(A.rho_ref) * Wt<CT>::w0, b1 = CT(A.rho_ref) * Wt<CT>::w1,
             b2 = CT(A.rho_ref) * Wt<CT>::w2;
    const int xm = gx == 0 ? A.nx - 1 : gx - 1;
    const int xp = gx == A.nx - 1 ? 0 : gx + 1;
    int ym = gy - 1, yp = gy + 1;
    bool sm = false, sp = false;  // is the source row below / above solid?
    if (A.bottom == BC_PERIODIC) {
        ym = ym < 0 ? ym + A.ny : ym;
        yp = yp >= A.ny ? yp - A.ny : yp;
    } else {
        sm = ym == 0;
        sp = yp == A.ny - 1;
    }
    const unsigned pitch = unsigned(A.fpitch), ux = unsigned(gx), uxm = unsigned(xm), uxp = unsigned(xp);
    const unsigned rc = unsigned(gy) * pitch, rm = unsigned(ym) * pitch, rp = unsigned(yp) * pitch;
    // Links that would come from a solid row return reversed from the node itself
    // (halfway bounce-back).  The source plane and offset are selected, not
    // branched on, so that the nine loads issue back to back.
    const unsigned oc = rc + ux;
    f[0] = C::ld(F.p[0], oc, b0);
    f[1] = C::ld(F.p[1], rc + uxm, b1);
    f[3] = C::ld(F.p[3], rc + uxp, b1);
    f[2] = C::ld(sm ? F.p[4] : F.p[2], sm ? oc : rm + ux, b1);
    f[5] = C::ld(sm ? F.p[7] : F.p[5], sm ? oc : rm + uxm, b2);
    f[6] = C::ld(sm ? F.p[8] : F.p[6], sm ? oc : rm + uxp, b2);
    f[4] = C::ld(sp ? F.p[2] : F.p[4], sp ? oc : rp + ux, b1);
    f[7] = C::ld(sp ? F.p[5] : F.p[7], sp ? oc : rp + uxp, b2);
    f[8] = C::ld(sp ? F.p[6] : F.p[8], sp ? oc : rp + uxm, b2);
}

template <typename CT>
__device__ __forceinline__ CT sum9(const CT f[9]) {
    return ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
}

template <typename ST, typename CT>
__device__ __forceinline__ CT fluid_rho(const LatticeArgs& A, const Planes<ST>& F, int gx, int gy) {
    CT f[9];
    pull9<ST, CT>(A, F, gx, gy, f);
    return sum9(f);
}

// Eq 28: density of a solid node from the adjacent fluid row yf.
template <typename ST, typename CT>
__device__ __forceinline__ CT ghost_rho(const LatticeArgs& A, const Planes<ST>& F, int gx, int yf) {
    const int xm = gx == 0 ? A.nx - 1 : gx - 1;
    const int xp = gx == A.nx - 1 ? 0 : gx + 1;
    const CT r0 = fluid_rho<ST, CT>(A, F, gx, yf);
    const CT rl = fluid_rho<ST, CT>(A, F, xm, yf);
    const CT rr = fluid_rho<ST, CT>(A, F, xp, yf);
    return CT(2) / CT(3) * r0 + CT(1) / CT(6) * rl + CT(1) / CT(6) * rr;
}

// Density at wrapped column gx and raw row y (y may lie outside a walled lattice,
// where nothing reads it).
template <typename ST, typename CT>
__device__ __forceinline__ CT node_rho(const LatticeArgs& A, const Planes<ST>& F, int gx, int y,
                                       bool small_y) {
    if (A.bottom == BC_PERIODIC) return fluid_rho<ST, CT>(A, F, gx, wrap_fast(y, A.ny, small_y));
    if (y < 0 || y >= A.ny) return CT(0);
    if (y == 0) return ghost_rho<ST, CT>(A, F, gx, 1);
    if (y == A.ny - 1) return ghost_rho<ST, CT>(A, F, gx, A.ny - 2);
    return fluid_rho<ST, CT>(A, F, gx, y);
}

// ---------------------------------------------------------------- thermodynamics
// FP64 reciprocal and logarithm for psi' inside the spinodal band of the 16-bit
// storage types, whose result is rounded to FP32: far cheaper than the correctly
// rounded division and the library logarithm, and accurate to about 1e-13.
//   rcp_band: the hardware reciprocal estimate and two Newton steps y += y (1 - x y).
//   log_band: x = m 2^e with m in [sqrt(1/2), sqrt 2), then
//             ln x = e ln 2 + 2 artanh s = e ln 2 + 2 s (1 + s^2/3 + ... + s^12/13),
//             s = (m - 1) / (m + 1) (the Taylor series of artanh; |s| <= 0.1716, so the
//             terms left out are below 2e-12 of the sum).
__device__ __forceinline__ double rcp_band(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

__device__ __forceinline__ double log_band(double x) {
    double m = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(x);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) * rcp_band(m + 1.0), t = s * s;
    double p = 1.0 / 13.0;
    p = fma(p, t, 1.0 / 11.0);
    p = fma(p, t, 1.0 / 9.0);
    p = fma(p, t, 1.0 / 7.0);
    p = fma(p, t, 1.0 / 5.0);
    p = fma(p, t, 1.0 / 3.0);
    p = fma(p, t, 1.0);
    return fma(double(e), 0.69314718055994530942, 2.0 * s * p);
}

// Bulk chemical potential psi'(rho): Eq 18 (VdW), Eq 27 (CS), Eq 24 (PR), Eq 21 (RK, RKS).
// BAND: FP64 with rcp_band and log_band (the spinodal band of 16-bit storage).
template <int EOS, typename CT, bool BAND = false>
__device__ __forceinline__ CT mu_bulk(const EosConst& E, CT rho) {
    const CT RT = CT(E.RT), a = CT(E.a), b = CT(E.b), c1 = CT(E.c1);
    const auto L = [](CT v) {
        if constexpr (BAND) return log_band(v);
        else return lg(v);
    };
    const auto Q = [](CT v) {
        if constexpr (BAND) return rcp_band(v);
        else return rcp(v);
    };
    if constexpr (EOS == EOS_CS) {
        const CT q = c1 * rho, om = CT(1) - q;
        return RT * ((CT(3) - q) * Q(om * om * om) + L(rho) + CT(1)) - CT(2) * a * rho;
    } else {
        const CT br = b * rho, ib = Q(CT(1) - br);
        const CT rep = RT * (L(rho * ib) + ib);
        if constexpr (EOS == EOS_VDW) {
            return rep - CT(2) * a * rho;
        } else if constexpr (EOS == EOS_PR) {
            const CT s2 = CT(1.4142135623730950488);
            return rep - c1 * L((s2 - CT(1) + br) * Q(s2 + CT(1) - br)) - a * rho * Q(CT(1) + CT(2) * br - br * br);
        } else {  // RK, RKS
            return rep - c1 * L(CT(1) + br) - a * rho * Q(CT(1) + br);
        }
    }
}

// psi'(rho) of a node: FP64 inside the spinodal band for the 16-bit storage types
// (where psi' is least well conditioned), the compute type elsewhere.
template <int EOS, typename ST>
__device__ __forceinline__ typename Codec<ST>::CT mu_node(const LatticeArgs& A, typename Codec<ST>::CT rho) {
    using CT = typename Codec<ST>::CT;
    if constexpr (sizeof(ST) == 2) {
        if (rho > CT(A.sp_lo) && rho < CT(A.sp_hi)) return CT(mu_bulk<EOS, double, true>(A.eos, double(rho)));
    }
    return mu_bulk<EOS, CT>(A.eos, rho);
}

// Bulk pressure p0(rho) of the EOS: Eq 16 (VdW), Eq 25 (CS), Eq 22 (PR), Eq 19 (RK,
// RKS); it enters the pressure tensor of Eq 9.
template <int EOS, typename CT>
__device__ __forceinline__ CT p_bulk(const EosConst& E, CT rho) {
    const CT RT = CT(E.RT), a = CT(E.a), b = CT(E.b), c1 = CT(E.c1);
    if constexpr (EOS == EOS_CS) {
        const CT q = c1 * rho, om = CT(1) - q;
        return rho * RT * (((CT(1) + q) + q * q) - q * q * q) * rcp(om * om * om) - a * rho * rho;
    } else {
        const CT rep = rho * RT * rcp(CT(1) - b * rho);
        if constexpr (EOS == EOS_VDW) {
            return rep - a * rho * rho;
        } else if constexpr (EOS == EOS_PR) {
            const CT br = b * rho;
            return rep - a * rho * rho * rcp(CT(1) + CT(2) * br - br * br);
        } else {  // RK, RKS
            return rep - a * rho * rho * rcp(CT(1) + b * rho);
        }
    }
}

// Isotropic Laplacian 6 sum_i w_i (phi_i - phi_0) on an LDS tile.
template <typename CT, int W>
__device__ __forceinline__ CT lap9(const CT (*s)[W], int r, int c) {
    const CT axis = (s[r][c - 1] + s[r][c + 1]) + (s[r - 1][c] + s[r + 1][c]);
    const CT diag = (s[r - 1][c - 1] + s[r - 1][c + 1]) + (s[r + 1][c - 1] + s[r + 1][c + 1]);
    return CT(2) / CT(3) * axis + CT(1) / CT(6) * diag - CT(10) / CT(3) * s[r][c];
}

// Isotropic gradient 3 sum_i w_i e_i phi_i on an LDS tile (row r+1 is +y).
template <typename CT, int W>
__device__ __forceinline__ void grad9(const CT (*s)[W], int r, int c, CT& gx, CT& gy) {
    const CT ne = s[r + 1][c + 1], nw = s[r + 1][c - 1], se = s[r - 1][c + 1], sw = s[r - 1][c - 1];
    constexpr CT third = CT(1) / CT(3), twelfth = CT(1) / CT(12);
    gx = (s[r][c + 1] - s[r][c - 1]) * third + ((ne - nw) + (se - sw)) * twelfth;
    gy = (s[r + 1][c] - s[r - 1][c]) * third + ((ne + nw) - (se + sw)) * twelfth;
}

// Momentum sum_i f_i e_i of one node.
template <typename CT>
__device__ __forceinline__ void momentum(const CT f[9], CT& jx, CT& jy) {
    jx = ((f[1] - f[3]) + (f[5] - f[6])) + (f[8] - f[7]);
    jy = ((f[2] - f[4]) + (f[5] + f[6])) - (f[7] + f[8]);
}

// Force of Eq 12 from the chemical-potential and density gradients, then the BGK
// collision of Eqs 13 and 14 with the equilibrium velocity u + tau F / rho:
// fs[i] = f_i - (f_i - f_i^eq) / tau.
template <typename CT>
__device__ __forceinline__ void collide(const CT f[9], CT rho, CT jx, CT jy, CT gmx, CT gmy, CT grx, CT gry,
                                        CT tau, CT inv_tau, CT fs[9]) {
    constexpr CT third = CT(1) / CT(3);
    const CT Fx = -rho * gmx + grx * third;
    const CT Fy = -rho * gmy + gry * third;
    const CT inv_rho = rcp(rho);
    const CT ux = jx * inv_rho, uy = jy * inv_rho;
    const CT uex = ux + tau * Fx * inv_rho, uey = uy + tau * Fy * inv_rho;
    const CT usq = CT(1.5) * (uex * uex + uey * uey);
    const CT r0 = Wt<CT>::w0 * rho, r1 = Wt<CT>::w1 * rho, r2 = Wt<CT>::w2 * rho;
    CT feq[9];
    feq[0] = r0 * (CT(1) - usq);
    {
        const CT e1 = uex, e2 = uey;
        feq[1] = r1 * (CT(1) + CT(3) * e1 + CT(4.5) * e1 * e1 - usq);
        feq[3] = r1 * (CT(1) - CT(3) * e1 + CT(4.5) * e1 * e1 - usq);
        feq[2] = r1 * (CT(1) + CT(3) * e2 + CT(4.5) * e2 * e2 - usq);
        feq[4] = r1 * (CT(1) - CT(3) * e2 + CT(4.5) * e2 * e2 - usq);
        const CT d5 = uex + uey, d6 = uey - uex;
        feq[5] = r2 * (CT(1) + CT(3) * d5 + CT(4.5) * d5 * d5 - usq);
        feq[7] = r2 * (CT(1) - CT(3) * d5 + CT(4.5) * d5 * d5 - usq);
        feq[6] = r2 * (CT(1) + CT(3) * d6 + CT(4.5) * d6 * d6 - usq);
        feq[8] = r2 * (CT(1) - CT(3) * d6 + CT(4.5) * d6 * d6 - usq);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) fs[i] = f[i] - (f[i] - feq[i]) * inv_tau;
}

// Eq 14 at density rho and velocity (ux, uy).
template <typename CT>
__device__ __forceinline__ void feq9(CT rho, CT ux, CT uy, CT fe[9]) {
    const CT usq = CT(1.5) * (ux * ux + uy * uy);
    const CT r0 = Wt<CT>::w0 * rho, r1 = Wt<CT>::w1 * rho, r2 = Wt<CT>::w2 * rho;
    const CT d5 = ux + uy, d6 = uy - ux;
    fe[0] = r0 * (CT(1) - usq);
    fe[1] = r1 * (CT(1) + CT(3) * ux + CT(4.5) * ux * ux - usq);
    fe[3] = r1 * (CT(1) - CT(3) * ux + CT(4.5) * ux * ux - usq);
    fe[2] = r1 * (CT(1) + CT(3) * uy + CT(4.5) * uy * uy - usq);
    fe[4] = r1 * (CT(1) - CT(3) * uy + CT(4.5) * uy * uy - usq);
    fe[5] = r2 * (CT(1) + CT(3) * d5 + CT(4.5) * d5 * d5 - usq);
    fe[7] = r2 * (CT(1) - CT(3) * d5 + CT(4.5) * d5 * d5 - usq);
    fe[6] = r2 * (CT(1) + CT(3) * d6 + CT(4.5) * d6 * d6 - usq);
    fe[8] = r2 * (CT(1) - CT(3) * d6 + CT(4.5) * d6 * d6 - usq);
}

// Collision of the variants with a given force F: BGK (Eq 13), TRT or MRT, each
// relaxing part towards the equilibrium at u + F / (rho s) for its own rate s.
template <typename CT, int COLL>
__device__ __forceinline__ void collide_with_force(const LatticeArgs& A, const CT f[9], CT rho, CT jx, CT jy,
                                                   CT Fx, CT Fy, CT fs[9]) {
    const CT inv_rho = rcp(rho);
    const CT ux = jx * inv_rho, uy = jy * inv_rho, gx = Fx * inv_rho, gy = Fy * inv_rho;
    const CT tau = CT(A.tau), inv_tau = CT(A.inv_tau);
    if constexpr (COLL == COLLIDE_BGK) {
        CT fe[9];
        feq9<CT>(rho, ux + tau * gx, uy + tau * gy, fe);
#pragma unroll
        for (int i = 0; i < 9; ++i) fs[i] = f[i] - (f[i] - fe[i]) * inv_tau;
    } else if constexpr (COLL == COLLIDE_TRT) {
        const CT tm = CT(A.tau_minus), inv_tm = rcp(tm);
        CT fe[9], fo[9];
        feq9<CT>(rho, ux + tau * gx, uy + tau * gy, fe);  // the even part's equilibrium
        feq9<CT>(rho, ux + tm * gx, uy + tm * gy, fo);    // the odd part's
        constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int o = opp[i];
            const CT ev = CT(0.5) * ((f[i] + f[o]) - (fe[i] + fe[o]));
            const CT od = CT(0.5) * ((f[i] - f[o]) - (fo[i] - fo[o]));
            fs[i] = f[i] - ev * inv_tau - od * inv_tm;
        }
    } else {  // MRT, Lallemand-Luo moments; equilibrium moments in closed form
        const CT se = CT(A.s_e), sp = CT(A.s_eps), sq = CT(A.s_q);
        // velocities shifted for each rate: 1/tau (j, stress), s_e, s_eps, s_q
        const CT vx = ux + tau * gx, vy = uy + tau * gy;
        const CT ex = ux + gx * rcp(se), ey = uy + gy * rcp(se);
        const CT px = ux + gx * rcp(sp), py = uy + gy * rcp(sp);
        const CT qx = ux + gx * rcp(sq), qy = uy + gy * rcp(sq);
        const CT axis = (f[1] + f[2]) + (f[3] + f[4]), diag = (f[5] + f[6]) + (f[7] + f[8]);
        const CT m_e = CT(-4) * f[0] - axis + CT(2) * diag;
        const CT m_p = CT(4) * f[0] - CT(2) * axis + diag;
        const CT m_qx = CT(-2) * (f[1] - f[3]) + ((f[5] - f[6]) - (f[7] - f[8]));
        const CT m_qy = CT(-2) * (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
        const CT m_xx = (f[1] + f[3]) - (f[2] + f[4]);
        const CT m_xy = (f[5] + f[7]) - (f[6] + f[8]);
        // s_k (m_k - m_k^eq) / |row k|^2
        const CT de = se * (m_e - rho * (CT(-2) + CT(3) * (ex * ex + ey * ey))) * CT(1.0 / 36.0);
        const CT dp = sp * (m_p - rho * (CT(1) - CT(3) * (px * px + py * py))) * CT(1.0 / 36.0);
        const CT djx = -Fx * CT(1.0 / 6.0), djy = -Fy * CT(1.0 / 6.0);  // (1/tau)(j - rho (u + tau F/rho)) / 6
        const CT dqx = sq * (m_qx + rho * qx) * CT(1.0 / 12.0);
        const CT dqy = sq * (m_qy + rho * qy) * CT(1.0 / 12.0);
        const CT dxx = inv_tau * (m_xx - rho * (vx * vx - vy * vy)) * CT(0.25);
        const CT dxy = inv_tau * (m_xy - rho * vx * vy) * CT(0.25);
        // f* = f - M^T d, column by column of M
        fs[0] = f[0] - (CT(-4) * de + CT(4) * dp);
        fs[1] = f[1] - (((-de - CT(2) * dp) + (djx - CT(2) * dqx)) + dxx);
        fs[2] = f[2] - (((-de - CT(2) * dp) + (djy - CT(2) * dqy)) - dxx);
        fs[3] = f[3] - (((-de - CT(2) * dp) - (djx - CT(2) * dqx)) + dxx);
        fs[4] = f[4] - (((-de - CT(2) * dp) - (djy - CT(2) * dqy)) - dxx);
        const CT c = CT(2) * de + dp;
        fs[5] = f[5] - (c + ((djx + dqx) + (djy + dqy)) + dxy);
        fs[6] = f[6] - (c + (-(djx + dqx) + (djy + dqy)) - dxy);
        fs[7] = f[7] - (c - ((djx + dqx) + (djy + dqy)) + dxy);
        fs[8] = f[8] - (c + ((djx + dqx) - (djy + dqy)) - dxy);
    }
}

__device__ __forceinline__ int tile_of_block(int b, int nblk) {
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
    // band of tiles so that halos shared by neighbouring tiles stay in its L2.
    const int q = nblk >> 3, r = nblk & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// ---------------------------------------------------------------- the fused step
template <typename CT, int TY, int TX = TILE_X, bool PT = false>
struct TileLds {
    CT rs[TY + 4][TX + 4];  // density, tile + 2-node ring
    CT ms[TY + 2][TX + 2];  // chemical potential, tile + 1-node ring
};
// The pressure-tensor force also keeps P_xx, P_yy, P_xy on the tile + 1-node ring.
template <typename CT, int TY, int TX>
struct TileLds<CT, TY, TX, true> {
    CT rs[TY + 4][TX + 4];
    CT ms[TY + 2][TX + 2];
    CT ps[3][TY + 2][TX + 2];
};

// Ring slot q of a TX x TY tile's two-node density ring (2 (TX + 4) + 2 (TX + 4) +
// 2 TY + 2 TY slots: the two rows below, the two rows above, the two columns on
// the left, the two columns on the right) as its row r and column c in the
// (TY + 4) x (TX + 4) density tile.
template <int TY, int TX>
__device__ __forceinline__ void ring_slot(int q, int& r, int& c) {
    constexpr int RW = TX + 4;
    if (q < 2 * RW) {
        r = q / RW;
        c = q % RW;
    } else if (q < 4 * RW) {
        r = TY + 2 + (q - 2 * RW) / RW;
        c = (q - 2 * RW) % RW;
    } else if (q < 4 * RW + 2 * TY) {
        r = 2 + (q - 4 * RW) / 2;
        c = (q - 4 * RW) % 2;
    } else {
        r = 2 + (q - 4 * RW - 2 * TY) / 2;
        c = TX + 2 + (q - 4 * RW - 2 * TY) % 2;
    }
}

// Own-node pulls of a TX x TY tile: thread (lx, ly) pulls the nine distributions
// of its RPT nodes (column x0 + lx, rows y0 + ly + k TY/RPT).  All RPT pulls go
// out before any wait; every thread pulls a fluid node (rows clamped into the
// fluid range, columns wrapped), and what a thread does not own is dropped later.
template <typename ST, int TY, int TX, int RPT>
__device__ __forceinline__ void tile_pull(const LatticeArgs& A, const Planes<ST>& F, int x0, int y0,
                                          typename Codec<ST>::CT f[RPT][9]) {
    using CT = typename Codec<ST>::CT;
    constexpr int RS = TY / RPT;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int gxw = wrap_fast(x0 + lx, A.nx, A.nx < TX + 2);
    const int y_lo = A.bottom == BC_PERIODIC ? 0 : 1, y_hi = A.bottom == BC_PERIODIC ? A.ny - 1 : A.ny - 2;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int gy = y0 + ly + k * RS;
        // rows are uniform across a wave: TX is a multiple of the wave width
        pull9<ST, CT, TX % 64 == 0>(A, F, gxw, gy < y_lo ? y_lo : (gy > y_hi ? y_hi : gy), f[k]);
    }
}

// The rest of one tile of the step (MODE_STEP) or of the field output
// (MODE_FIELDS), from the own nodes' pulled distributions f: densities of the
// tile and its ring into LDS, chemical potential, force, collision and store.
// HOIST: the ring's pulls go out right after the own pulls, before the first wait
// (one memory round trip instead of two, at the cost of registers).  NTS: the
// stores of f*(t) are non-temporal (lattices larger than the caches).
template <typename ST, int EOS, int MODE, int TY, int TX, int RPT, bool HOIST = false, int FORCE = FORCE_CP,
          int COLL = COLLIDE_BGK, bool NTS = false>
__device__ __forceinline__ void tile_rest(const LatticeArgs& A, const Planes<ST>& F, ST* __restrict__ fout,
                                          const typename Codec<ST>::CT* __restrict__ mu_w,
                                          double* __restrict__ out, int x0, int y0,
                                          typename Codec<ST>::CT f[RPT][9],
                                          TileLds<typename Codec<ST>::CT, TY, TX, FORCE == FORCE_PTENSOR>& L) {
    using CT = typename Codec<ST>::CT;
    using C = Codec<ST>;
    constexpr int RW = TX + 4, MW = TX + 2;
    constexpr int NT = TX * TY / RPT;  // threads
    constexpr int RS = TY / RPT;       // row stride between a thread's nodes
    auto& rs = L.rs;
    auto& ms = L.ms;

    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const bool small_x = A.nx < TX + 2, small_y = A.ny < TY + 2;

    constexpr int RING = 2 * (TX + 4) * 2 + 2 * TY * 2;
    constexpr int RPR = HOIST ? (RING + NT - 1) / NT : 1;  // ring slots per thread
    CT fr[RPR][9];
    int rpos[RPR];     // r * RW + c of the slot; -1: a spare slot
    bool rfluid[RPR];  // the slot is a fluid node (its density is the sum of its pulls)
    if constexpr (HOIST) {
        const bool periodic = A.bottom == BC_PERIODIC;
        const int y_lo = periodic ? 0 : 1, y_hi = periodic ? A.ny - 1 : A.ny - 2;
#pragma unroll
        for (int j = 0; j < RPR; ++j) {
            const int q = threadIdx.x + j * NT;
            const bool live = q < RING;
            int r, c;
            ring_slot<TY, TX>(q, r, c);
            if (!live) {  // a spare slot loads a line that the bottom ring row fetches anyway
                r = 0;
                c = q % RW;
            }
            int gy = y0 - 2 + r;
            if (periodic) gy = wrap_fast(gy, A.ny, small_y);
            rfluid[j] = live && gy >= y_lo && gy <= y_hi;
            rpos[j] = live ? r * RW + c : -1;
            pull9<ST, CT>(A, F, wrap_fast(x0 - 2 + c, A.nx, small_x), gy < y_lo ? y_lo : (gy > y_hi ? y_hi : gy),
                          fr[j]);
        }
    }

    // 1. own nodes: density and momentum from the pulls, density into LDS
    CT jx[RPT], jy[RPT];
    const int gx_raw = x0 + lx;
    const int gxw = wrap_fast(gx_raw, A.nx, small_x);
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int gy = y0 + ly + k * RS;
        const bool own = gx_raw < A.nx && gy < A.ny && !solid_row(A, gy);
        CT r;
        if (own) {
            r = sum9(f[k]);
            momentum(f[k], jx[k], jy[k]);
        } else {
            r = node_rho<ST, CT>(A, F, gxw, gy, small_y);
        }
        rs[ly + k * RS + 2][lx + 2] = r;
    }

    // Wall chemical potentials (the surface value of Sec. IV, which enters the force of
    // Eq 12 through grad mu) of a CP wall row inside the chemical-potential
    // tile go out with the ring's pulls and land in LDS with the densities, so that
    // step 3 reads no global memory.
    const int mwb = 1 - y0, mwt = A.ny - y0;  // ms rows of y = 0 and y = ny - 1
    const bool cpb = A.bottom == BC_CPWALL && mwb >= 0;
    const bool cpt = A.top == BC_CPWALL && mwt <= TY + 1;
    constexpr int MWR = (2 * MW + NT - 1) / NT;
    CT mwv[MWR];
    if (cpb || cpt) {
#pragma unroll
        for (int j = 0; j < MWR; ++j) {
            const int q = threadIdx.x + j * NT, w = q / MW, c = q % MW;
            mwv[j] = (q < 2 * MW && (w == 0 ? cpb : cpt))
                         ? mu_w[(w == 0 ? 0 : A.pitch) + wrap_fast(x0 - 1 + c, A.nx, small_x)]
                         : CT(0);
        }
    }

    // 2. the two-node ring of densities around the tile (Eq 28 for solid rows)
    if constexpr (HOIST) {
        CT* rs_flat = &rs[0][0];
#pragma unroll
        for (int j = 0; j < RPR; ++j) {
            if (rpos[j] < 0) continue;
            CT r;
            if (rfluid[j]) {
                r = sum9(fr[j]);
            } else {
                const int rr = rpos[j] / RW, cc = rpos[j] % RW;
                r = node_rho<ST, CT>(A, F, wrap_fast(x0 - 2 + cc, A.nx, small_x), y0 - 2 + rr, small_y);
            }
            rs_flat[rpos[j]] = r;
        }
    } else {
        for (int q = threadIdx.x; q < RING; q += NT) {
            int r, c;
            ring_slot<TY, TX>(q, r, c);
            rs[r][c] = node_rho<ST, CT>(A, F, wrap_fast(x0 - 2 + c, A.nx, small_x), y0 - 2 + r, small_y);
        }
    }
    if (cpb || cpt) {
#pragma unroll
        for (int j = 0; j < MWR; ++j) {
            const int q = threadIdx.x + j * NT, w = q / MW, c = q % MW;
            if (q < 2 * MW && (w == 0 ? cpb : cpt)) ms[w == 0 ? mwb : mwt][c] = mwv[j];
        }
    }
    __syncthreads();

    // 3. chemical potential, Eq 8, on the tile and a one-node ring
    const CT kappa = CT(A.kappa);
    if constexpr (FORCE == FORCE_PTENSOR) {
        // the pressure tensor of Eq 9 on the tile and a one-node ring (periodic
        // lattices only), and the chemical potential for the field output
        for (int q = threadIdx.x; q < (TY + 2) * MW; q += NT) {
            const int r = q / MW, c = q % MW;
            const CT rho = rs[r + 1][c + 1];
            const CT lap = lap9<CT, RW>(rs, r + 1, c + 1);
            CT gx, gy;
            grad9<CT, RW>(rs, r + 1, c + 1, gx, gy);
            const CT pd = p_bulk<EOS, CT>(A.eos, rho) - kappa * rho * lap - CT(0.5) * kappa * (gx * gx + gy * gy);
            L.ps[0][r][c] = pd + kappa * gx * gx;
            L.ps[1][r][c] = pd + kappa * gy * gy;
            L.ps[2][r][c] = kappa * gx * gy;
            if (MODE == MODE_FIELDS) ms[r][c] = mu_node<EOS, ST>(A, rho) - kappa * lap;
        }
    } else
    for (int q = threadIdx.x; q < (TY + 2) * MW; q += NT) {
        const int r = q / MW, c = q % MW;
        const int y = y0 - 1 + r;
        CT m;
        if (A.bottom == BC_PERIODIC) {
            m = mu_node<EOS, ST>(A, rs[r + 1][c + 1]) - kappa * lap9<CT, RW>(rs, r + 1, c + 1);
        } else if (y <= 0 || y >= A.ny - 1) {
            if (y == 0 || y == A.ny - 1) {
                const int kind = y == 0 ? A.bottom : A.top;
                if (kind == BC_CPWALL) {
                    continue;  // in LDS since step 2
                } else {  // neutral wall: the chemical potential of the adjacent fluid node
                    const int rn = y == 0 ? r + 2 : r;
                    m = mu_node<EOS, ST>(A, rs[rn][c + 1]) - kappa * lap9<CT, RW>(rs, rn, c + 1);
                }
            } else {
                m = CT(0);  // outside the lattice: never read
            }
        } else {
            m = mu_node<EOS, ST>(A, rs[r + 1][c + 1]) - kappa * lap9<CT, RW>(rs, r + 1, c + 1);
        }
        ms[r][c] = m;
    }
    __syncthreads();

    // 4. force (Eq 12), collision (Eqs 13, 14, u_eq = u + tau F / rho), store
    const CT tau = CT(A.tau), inv_tau = CT(A.inv_tau);
    const CT b0 = CT(A.rho_ref) * Wt<CT>::w0, b1 = CT(A.rho_ref) * Wt<CT>::w1,
             b2 = CT(A.rho_ref) * Wt<CT>::w2;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ry = ly + k * RS;
        const int gy = y0 + ry;
        if (gx_raw >= A.nx || gy >= A.ny) continue;
        const bool solid = solid_row(A, gy);
        const CT rho = rs[ry + 2][lx + 2];
        if (MODE == MODE_FIELDS) {
            const long long o = (long long)gy * A.nx + gx_raw;
            const long long P = (long long)A.nx * A.ny;
            if (solid) {
                out[o] = double(rho);
                out[P + o] = 0.0;
                out[2 * P + o] = 0.0;
                out[3 * P + o] = double(ms[ry + 1][lx + 1]);
                continue;
            }
        } else if (solid) {
            continue;
        }
        CT gmx, gmy, grx, gry;
        grad9<CT, RW>(rs, ry + 2, lx + 2, grx, gry);
        if constexpr (FORCE == FORCE_PTENSOR) {
            // F = -div P + c_s^2 grad(rho), Eq 5; (gmx, gmy) carry div P
            CT dxx, dyx, dxy, dyy, dxn, dyn;
            grad9<CT, MW>(L.ps[0], ry + 1, lx + 1, dxx, dyx);
            grad9<CT, MW>(L.ps[2], ry + 1, lx + 1, dxy, dyy);
            grad9<CT, MW>(L.ps[1], ry + 1, lx + 1, dxn, dyn);
            gmx = dxx + dyy;
            gmy = dxy + dyn;
        } else {
            grad9<CT, MW>(ms, ry + 1, lx + 1, gmx, gmy);
        }
        constexpr CT third = CT(1) / CT(3);
        // the force: Eq 12 (-rho grad mu) or Eq 5 (-div P), plus c_s^2 grad(rho)
        auto force = [&](CT& Fx, CT& Fy) {
            if constexpr (FORCE == FORCE_PTENSOR) {
                Fx = -gmx + grx * third;
                Fy = -gmy + gry * third;
            } else {
                Fx = -rho * gmx + grx * third;
                Fy = -rho * gmy + gry * third;
            }
        };
        if (MODE == MODE_FIELDS) {
            CT Fx, Fy;
            force(Fx, Fy);
            const CT inv_rho = rcp(rho);
            const long long o = (long long)gy * A.nx + gx_raw;
            const long long P = (long long)A.nx * A.ny;
            out[o] = double(rho);
            out[P + o] = double(jx[k] * inv_rho + CT(0.5) * Fx * inv_rho);
            out[2 * P + o] = double(jy[k] * inv_rho + CT(0.5) * Fy * inv_rho);
            out[3 * P + o] = double(ms[ry + 1][lx + 1]);
            continue;
        }
        CT fs[9];
        if constexpr (FORCE == FORCE_CP && COLL == COLLIDE_BGK) {
            collide<CT>(f[k], rho, jx[k], jy[k], gmx, gmy, grx, gry, tau, inv_tau, fs);
        } else {
            CT Fx, Fy;
            force(Fx, Fy);
            collide_with_force<CT, COLL>(A, f[k], rho, jx[k], jy[k], Fx, Fy, fs);
        }
        const unsigned o = unsigned(gy) * unsigned(A.fpitch) + unsigned(gx_raw);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const CT base = i == 0 ? b0 : (i < 5 ? b1 : b2);
            if constexpr (NTS)
                C::stn(fout + (long long)i * A.plane, o, fs[i], base);
            else
                C::st(fout + (long long)i * A.plane, o, fs[i], base);
        }
    }
}

// One TX x TY tile of the step or of the field output, run by a workgroup of
// TX * TY / RPT threads, RPT nodes of one column per thread.
template <typename ST, int EOS, int MODE, int TY, int TX = TILE_X, int RPT = ROWS_PER_THREAD, bool HOIST = false,
          int FORCE = FORCE_CP, int COLL = COLLIDE_BGK, bool NTS = false>
__device__ __forceinline__ void step_tile(const LatticeArgs& A, const ST* __restrict__ fin,
                                          ST* __restrict__ fout,
                                          const typename Codec<ST>::CT* __restrict__ mu_w,
                                          double* __restrict__ out, int x0, int y0,
                                          TileLds<typename Codec<ST>::CT, TY, TX, FORCE == FORCE_PTENSOR>& L) {
    using CT = typename Codec<ST>::CT;
    Planes<ST> F;
#pragma unroll
    for (int i = 0; i < 9; ++i) F.p[i] = fin + (long long)i * A.plane;
    CT f[RPT][9];
    // On lattices beyond the caches the pulls go out at a raised wave priority, so
    // that a wave issuing its loads wins the SIMD's arbitration over waves in their
    // arithmetic and more bytes are in flight from HBM (4096^2 FP32: 217.9 -> 208.2 us;
    // a cache-resident 1024^2 lattice lost 4 % with it)
    if constexpr (NTS) __builtin_amdgcn_s_setprio(2);
    tile_pull<ST, TY, TX, RPT>(A, F, x0, y0, f);
    if constexpr (NTS) __builtin_amdgcn_s_setprio(0);
    tile_rest<ST, EOS, MODE, TY, TX, RPT, HOIST, FORCE, COLL, NTS>(A, F, fout, mu_w, out, x0, y0, f, L);
}

// One lattice: one workgroup per tile.
template <typename ST, int EOS, int MODE, int TY, int TX = TILE_X, int RPT = ROWS_PER_THREAD, bool HOIST = false,
          int FORCE = FORCE_CP, int COLL = COLLIDE_BGK, bool NTS = false>
__global__ __launch_bounds__(TX * TY / RPT) void step_kernel(LatticeArgs A, const ST* __restrict__ fin,
                                                            ST* __restrict__ fout,
                                                            const typename Codec<ST>::CT* __restrict__ mu_w,
                                                            double* __restrict__ out) {
    __shared__ TileLds<typename Codec<ST>::CT, TY, TX, FORCE == FORCE_PTENSOR> L;
    const int t = tile_of_block(blockIdx.x, gridDim.x);
    const int tiles_x = (A.nx + TX - 1) / TX;
    step_tile<ST, EOS, MODE, TY, TX, RPT, HOIST, FORCE, COLL, NTS>(A, fin, fout, mu_w, out, (t % tiles_x) * TX,
                                                              (t / tiles_x) * TY, L);
}

// The mixed schedule: a case narrower than BATCH_MIXED_WIDE columns runs 64 x 32 tiles,
// a wider one 256 x 8 tiles (the shape codes its descriptor carries); both shapes have
// 512 threads of 4 rows, so one launch takes both, with the LDS of the larger.
template <typename ST, bool NTS>
__global__ __launch_bounds__(512) void batch_step_mixed_kernel(const CaseDesc* __restrict__ cases,
                                                               const int2* __restrict__ tiles, int ntiles,
                                                               int parity) {
    using CT = typename Codec<ST>::CT;
    __shared__ union {
        TileLds<CT, 32, 64> small;
        TileLds<CT, 8, 256> wide;
    } L;
    const int chunk = tile_of_block(blockIdx.x, gridDim.x);
    const int begin = int((long long)ntiles * chunk / gridDim.x);
    const int end = int((long long)ntiles * (chunk + 1) / gridDim.x);
    constexpr int R = ROWS_PER_THREAD;
    constexpr int F = FORCE_CP, B = COLLIDE_BGK;
    for (int t = begin; t < end; ++t) {
        const int2 w = tiles[t];
        const CaseDesc& C = cases[w.x];
        const ST* fin = in_global(static_cast<const ST*>(C.f[parity]));
        ST* fout = in_global(static_cast<ST*>(C.f[parity ^ 1]));
        const CT* mw = in_global(static_cast<const CT*>(C.mu_w));
        if (C.A.tile_y == 32) {  // workgroup-uniform
            const int tiles_x = (C.A.nx + 63) / 64;
            const int x0 = (w.y % tiles_x) * 64, y0 = (w.y / tiles_x) * 32;
            switch (C.eos) {
            case EOS_VDW:
                step_tile<ST, EOS_VDW, MODE_STEP, 32, 64, R, false, F, B, NTS>(C.A, fin, fout, mw, nullptr, x0, y0,
                                                                              L.small);
                break;
            case EOS_CS:
                step_tile<ST, EOS_CS, MODE_STEP, 32, 64, R, false, F, B, NTS>(C.A, fin, fout, mw, nullptr, x0, y0,
                                                                             L.small);
                break;
            case EOS_PR:
                step_tile<ST, EOS_PR, MODE_STEP, 32, 64, R, false, F, B, NTS>(C.A, fin, fout, mw, nullptr, x0, y0,
                                                                             L.small);
                break;
            default:
                step_tile<ST, EOS_RK, MODE_STEP, 32, 64, R, false, F, B, NTS>(C.A, fin, fout, mw, nullptr, x0, y0,
                                                                             L.small);
                break;
            }
        } else {
            const int tiles_x = (C.A.nx + 255) / 256;
            const int x0 = (w.y % tiles_x) * 256, y0 = (w.y / tiles_x) * 8;
            switch (C.eos) {
            case EOS_VDW:
                step_tile<ST, EOS_VDW, MODE_STEP, 8, 256, R, false, F, B, NTS>(C.A, fin, fout, mw, nullptr, x0, y0,
                                                                              L.wide);
                break;
            case EOS_CS:
                step_tile<ST, EOS_CS, MODE_STEP, 8, 256, R, false, F, B, NTS>(C.A, fin, fout, mw, nullptr, x0, y0,
                                                                             L.wide);
                break;
            case EOS_PR:
                step_tile<ST, EOS_PR, MODE_STEP, 8, 256, R, false, F, B, NTS>(C.A, fin, fout, mw, nullptr, x0, y0,
                                                                             L.wide);
                break;
            default:
                step_tile<ST, EOS_RK, MODE_STEP, 8, 256, R, false, F, B, NTS>(C.A, fin, fout, mw, nullptr, x0, y0,
                                                                             L.wide);
                break;
            }
        }
        __syncthreads();  // the next tile reuses the LDS
    }
}

// Many lattices in one persistent launch: each workgroup walks a contiguous range
// of the (case, tile) list; the ranges of the workgroups on one XCD are adjacent.
template <typename ST, int TY, int TX = TILE_X, bool NTS = false>
__global__ __launch_bounds__(TX * TY / ROWS_PER_THREAD) void batch_step_kernel(
    const CaseDesc* __restrict__ cases, const int2* __restrict__ tiles, int ntiles, int parity) {
    using CT = typename Codec<ST>::CT;
    __shared__ TileLds<CT, TY, TX> L;
    const int chunk = tile_of_block(blockIdx.x, gridDim.x);
    const int begin = int((long long)ntiles * chunk / gridDim.x);
    const int end = int((long long)ntiles * (chunk + 1) / gridDim.x);
    for (int t = begin; t < end; ++t) {
        const int2 w = tiles[t];
        const CaseDesc& C = cases[w.x];
        const int tiles_x = (C.A.nx + TX - 1) / TX;
        const int x0 = (w.y % tiles_x) * TX, y0 = (w.y / tiles_x) * TY;
        const ST* fin = in_global(static_cast<const ST*>(C.f[parity]));
        ST* fout = in_global(static_cast<ST*>(C.f[parity ^ 1]));
        const CT* mw = in_global(static_cast<const CT*>(C.mu_w));
        constexpr int R = ROWS_PER_THREAD;
        switch (C.eos) {
        case EOS_VDW:
            step_tile<ST, EOS_VDW, MODE_STEP, TY, TX, R, false, FORCE_CP, COLLIDE_BGK, NTS>(C.A, fin, fout, mw, nullptr,
                                                                                         x0, y0, L);
            break;
        case EOS_CS:
            step_tile<ST, EOS_CS, MODE_STEP, TY, TX, R, false, FORCE_CP, COLLIDE_BGK, NTS>(C.A, fin, fout, mw, nullptr,
                                                                                        x0, y0, L);
            break;
        case EOS_PR:
            step_tile<ST, EOS_PR, MODE_STEP, TY, TX, R, false, FORCE_CP, COLLIDE_BGK, NTS>(C.A, fin, fout, mw, nullptr,
                                                                                        x0, y0, L);
            break;
        default:
            step_tile<ST, EOS_RK, MODE_STEP, TY, TX, R, false, FORCE_CP, COLLIDE_BGK, NTS>(C.A, fin, fout, mw, nullptr,
                                                                                        x0, y0, L);
            break;
        }
        __syncthreads();  // the next tile reuses the LDS
    }
}

// ---------------------------------------------------------------- column-marching step
// For large lattices a workgroup owns a strip of MARCH_OWN columns and a segment of
// rows, one lane per column plus two halo lanes on each side, and marches up the
// segment one row per iteration.  Iteration R pulls row R (its loads were issued one
// iteration earlier) and puts its density into an LDS ring of rows, evaluates the
// chemical potential of row R - 2 into a second ring, and collides row R - 3 from
// distributions it kept in registers.  Every (plane, row) of f*(t-1) is read once
// per strip, the only redundant work is the two halo lanes per side and four extra
// rows per segment, and one barrier per row orders the rings.  Loads and stores are
// raw buffer accesses: the lane's column is a fixed byte offset, plane and row a
// uniform one, so no per-load address arithmetic remains.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}

// ldr: the raw stored value; dec: the distribution it holds (deviation formats add
// w_i rho_ref back); st: encode and store.  Loads stay raw until their row is used,
// so that a row's loads are issued back to back.
template <typename ST>
struct RawIO;
template <>
struct RawIO<double> {
    using RT = double;
    static __device__ __forceinline__ RT ldr(__amdgpu_buffer_rsrc_t r, int v, int s) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
    }
    static __device__ __forceinline__ double dec(RT x, double) { return x; }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int v, int s, double x, double) {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, x), r, v, s, 0);
    }
};
template <>
struct RawIO<float> {
    using RT = float;
    static __device__ __forceinline__ RT ldr(__amdgpu_buffer_rsrc_t r, int v, int s) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
    }
    static __device__ __forceinline__ float dec(RT x, float) { return x; }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int v, int s, float x, float) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, 0);
    }
};
template <>
struct RawIO<__half> {
    using RT = unsigned short;
    static __device__ __forceinline__ RT ldr(__amdgpu_buffer_rsrc_t r, int v, int s) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0);
    }
    static __device__ __forceinline__ float dec(RT x, float base) {
        return __half2float(__builtin_bit_cast(__half, x)) + base;
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int v, int s, float x, float base) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2half_rn(x - base)), r, v,
                                              s, 0);
    }
};
template <>
struct RawIO<__hip_bfloat16> {
    using RT = unsigned short;
    static __device__ __forceinline__ RT ldr(__amdgpu_buffer_rsrc_t r, int v, int s) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0);
    }
    static __device__ __forceinline__ float dec(RT x, float base) {
        return __bfloat162float(__builtin_bit_cast(__hip_bfloat16, x)) + base;
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int v, int s, float x, float base) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2bfloat16(x - base)), r, v,
                                              s, 0);
    }
};

__device__ __forceinline__ int wrap_col(int x, int n) {
    x %= n;
    return x < 0 ? x + n : x;
}

template <typename ST, int EOS>
struct March {
    using CT = typename Codec<ST>::CT;
    using IO = RawIO<ST>;
    static constexpr int NT = MARCH_NT;
    static constexpr int LW = MARCH_NT + 2;  // ring row: one pad entry on each side
    static constexpr int SZ = int(sizeof(ST));
    // A byte offset no buffer reaches: raw buffer accesses beyond the buffer's size
    // are dropped (stores) or read zero (loads), which masks a lane without a branch.
    static constexpr int NOWHERE = int(0x80000000u);

    const LatticeArgs& A;
    CT (*rs)[LW];  // density ring, 8 rows
    CT (*ms)[LW];  // chemical-potential ring, 4 rows
    const CT* mu_w;
    __amdgpu_buffer_rsrc_t rin, rout;
    int l, ys, ye, xr, xw;  // lane, segment rows [ys, ye), raw and wrapped column
    int vc, vm, vp;         // byte offsets of the columns x, x - 1, x + 1
    int vs;                 // store offset: vc on owned lanes, NOWHERE elsewhere
    int PB, RB;             // bytes per plane, per row
    bool walled, live, mu_lane, owned;
    bool nr;  // the next lane holds a density of this strip
    CT b0, b1, b2, tau, inv_tau, kappa;
    typename IO::RT fr[9];  // raw values of row R + 1, in flight
    CT fd[4][9];            // distributions of rows R, R-1, R-2, R-3 (slot = phase)

    __device__ __forceinline__ CT* rrow(int R) const { return rs[R & 7] + 1; }
    __device__ __forceinline__ CT* mrow(int m) const { return ms[m & 3] + 1; }

    __device__ __forceinline__ int wrap_row(int r) const {
        while (r < 0) r += A.ny;
        while (r >= A.ny) r -= A.ny;
        return r;
    }
    __device__ __forceinline__ bool fluid_row(int R) const {
        return walled ? (R >= 1 && R <= A.ny - 2) : true;
    }
    __device__ __forceinline__ CT base(int i) const { return i == 0 ? b0 : (i < 5 ? b1 : b2); }

    // f_i of row r from rows rm (below) and rp (above) at the column whose own /
    // left / right byte offsets are cc / cm / cp (pull streaming; reflected
    // populations when the row below / above is solid, sm / sp).
    __device__ __forceinline__ void pull_rows(int r, int rm, int rp, bool sm, bool sp, typename IO::RT g[9],
                                              int cc, int cm, int cp) const {
        const int oc = r * RB, om = rm * RB, op = rp * RB;
        g[0] = IO::ldr(rin, cc, oc);
        g[1] = IO::ldr(rin, cm, PB + oc);
        g[3] = IO::ldr(rin, cp, 3 * PB + oc);
        if (sm) {
            g[2] = IO::ldr(rin, cc, 4 * PB + oc);
            g[5] = IO::ldr(rin, cc, 7 * PB + oc);
            g[6] = IO::ldr(rin, cc, 8 * PB + oc);
        } else {
            g[2] = IO::ldr(rin, cc, 2 * PB + om);
            g[5] = IO::ldr(rin, cm, 5 * PB + om);
            g[6] = IO::ldr(rin, cp, 6 * PB + om);
        }
        if (sp) {
            g[4] = IO::ldr(rin, cc, 2 * PB + oc);
            g[7] = IO::ldr(rin, cc, 5 * PB + oc);
            g[8] = IO::ldr(rin, cc, 6 * PB + oc);
        } else {
            g[4] = IO::ldr(rin, cc, 4 * PB + op);
            g[7] = IO::ldr(rin, cp, 7 * PB + op);
            g[8] = IO::ldr(rin, cm, 8 * PB + op);
        }
    }
    // f_i of fluid row R, any row of the lattice.
    __device__ __forceinline__ void pull_row(int R, typename IO::RT g[9], int cc, int cm, int cp) const {
        if (walled)
            pull_rows(R, R - 1, R + 1, R - 1 == 0, R + 1 == A.ny - 1, g, cc, cm, cp);
        else
            pull_rows(wrap_row(R), wrap_row(R - 1), wrap_row(R + 1), false, false, g, cc, cm, cp);
    }
    __device__ __forceinline__ void decode(const typename IO::RT g[9], CT d[9]) const {
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = IO::dec(g[i], base(i));
    }

    // Density of fluid row rf at the column next to this lane's (dx = -1 or +1).
    __device__ __forceinline__ CT side_rho(int rf, int dx) const {
        const int x = wrap_col(xw + dx, A.nx);
        typename IO::RT g[9];
        CT d[9];
        pull_row(rf, g, x * SZ, wrap_col(x - 1, A.nx) * SZ, wrap_col(x + 1, A.nx) * SZ);
        decode(g, d);
        return sum9(d);
    }

    // Eq 28: density of the solid row next to fluid row rf.
    __device__ __forceinline__ CT ghost(int rf) const {
        const CT* q = rrow(rf);
        const CT r0 = q[l];
        const CT rl = l > 0 ? q[l - 1] : side_rho(rf, -1);
        const CT rr = nr ? q[l + 1] : side_rho(rf, +1);
        return CT(2) / CT(3) * r0 + CT(1) / CT(6) * rl + CT(1) / CT(6) * rr;
    }

    __device__ __forceinline__ CT lap(const CT* a, const CT* b, const CT* c) const {
        const CT axis = (b[l - 1] + b[l + 1]) + (a[l] + c[l]);
        const CT diag = (a[l - 1] + a[l + 1]) + (c[l - 1] + c[l + 1]);
        return CT(2) / CT(3) * axis + CT(1) / CT(6) * diag - CT(10) / CT(3) * b[l];
    }
    __device__ __forceinline__ void grad(const CT* a, const CT* b, const CT* c, CT& gx, CT& gy) const {
        const CT ne = c[l + 1], nw = c[l - 1], se = a[l + 1], sw = a[l - 1];
        constexpr CT third = CT(1) / CT(3), twelfth = CT(1) / CT(12);
        gx = (b[l + 1] - b[l - 1]) * third + ((ne - nw) + (se - sw)) * twelfth;
        gy = (c[l] - a[l]) * third + ((ne + nw) - (se + sw)) * twelfth;
    }
    __device__ __forceinline__ CT mu_at(int m) const {
        return mu_node<EOS, ST>(A, rrow(m)[l]) - kappa * lap(rrow(m - 1), rrow(m), rrow(m + 1));
    }
    // Collision of row c with the distributions g, stored to f*(t) at store offset v.
    __device__ __forceinline__ void collide_row(int c, const CT g[9], int v) const {
        CT gmx, gmy, grx, gry, jx, jy;
        grad(mrow(c - 1), mrow(c), mrow(c + 1), gmx, gmy);
        grad(rrow(c - 1), rrow(c), rrow(c + 1), grx, gry);
        momentum(g, jx, jy);
        CT fs[9];
        collide<CT>(g, rrow(c)[l], jx, jy, gmx, gmy, grx, gry, tau, inv_tau, fs);
        const int oc = c * RB;
        // plain stores: non-temporal ones slowed the marching step down (FP16 at
        // 4096^2: 173 -> 200 us), unlike the tiles
#pragma unroll
        for (int i = 0; i < 9; ++i) IO::st(rout, v, i * PB + oc, fs[i], base(i));
    }

    // Any iteration: every row kind (periodic wrap, walls, Eq 28 ghosts, wall mu).
    template <int P>
    __device__ __forceinline__ void iter(int R) {
        constexpr int PC = (P + 1) % 4;         // slot of row R - 3
        R = __builtin_amdgcn_readfirstlane(R);  // uniform: keeps row offsets scalar
        // (a) density of row R (its loads were issued one iteration earlier)
        if (R <= ye + 1 && live) {
            if (fluid_row(R)) {
                decode(fr, fd[P]);
                rrow(R)[l] = sum9(fd[P]);
            } else if (walled && R == A.ny - 1) {
                rrow(R)[l] = ghost(R - 1);
            }
        }
        // (b) issue the loads of row R + 1; they complete under (c), the barrier and (d)
        if (R + 1 <= ye + 1 && live && fluid_row(R + 1)) pull_row(R + 1, fr, vc, vm, vp);
        // (c) chemical potential of row m = R - 2 (Eq 8; wall rows from Sec. IV / V)
        const int m = R - 2;
        if (m >= ys - 1 && m <= ye) {
            if (!walled || (m >= 1 && m <= A.ny - 2)) {
                if (mu_lane) {
                    const CT mu = mu_at(m);
                    mrow(m)[l] = mu;
                    if (walled && m == 1) {
                        CT w = mu;
                        if (A.bottom == BC_CPWALL) w = mu_w[xw];
                        mrow(0)[l] = w;
                    }
                }
            } else if (walled && m == 0) {
                if (live) rrow(0)[l] = ghost(1);
            } else if (walled && m == A.ny - 1) {
                if (mu_lane) {
                    CT mu;
                    if (A.top == BC_CPWALL) {
                        mu = mu_w[A.pitch + xw];
                    } else {
                        mu = mrow(m - 1)[l];
                    }
                    mrow(m)[l] = mu;
                }
            }
        }
        __syncthreads();
        // (d) collision of row c = R - 3, stored to f*(t)
        const int c = R - 3;
        if (c >= ys && c < ye && owned && fluid_row(c)) collide_row(c, fd[PC], vc);
    }

    // An interior iteration (rows R - 4 .. R + 2 are fluid rows inside the lattice,
    // no wrap, no wall): the same work with no branch, so the memory operations of
    // every iteration are the same and the loads of row R need not wait for the
    // stores issued after them.  Lanes outside the strip's columns compute values
    // nobody reads (the ring rows are padded) and store nowhere.
    template <int P>
    __device__ __forceinline__ void steady(int R) {
        constexpr int PC = (P + 1) % 4;
        R = __builtin_amdgcn_readfirstlane(R);
        decode(fr, fd[P]);
        rrow(R)[l] = sum9(fd[P]);
        pull_rows(R + 1, R, R + 2, false, false, fr, vc, vm, vp);
        mrow(R - 2)[l] = mu_at(R - 2);
        __syncthreads();
        collide_row(R - 3, fd[PC], vs);
    }

    __device__ __forceinline__ void run() {
        const int R0 = ys - 2, Rend = ye + 2;
        int R = R0;
        if (live && fluid_row(R)) pull_row(R, fr, vc, vm, vp);
        // interior iterations [S0, S1]; S0p: first iteration of a four-row block at
        // or after S0, so that the register rotation's phase there is zero
        const int S0 = walled ? max(ys + 3, 4) : ys + 3;
        const int S1 = min(ye, walled ? A.ny - 4 : A.ny - 3);
        const int S0p = R0 + 4 * ((S0 - R0 + 3) / 4);
        const int stop = min(S0p, Rend + 1);
        while (R < stop) {  // iterations past Rend do nothing
            iter<0>(R);
            iter<1>(R + 1);
            iter<2>(R + 2);
            iter<3>(R + 3);
            R += 4;
        }
        if (R == S0p && R + 3 <= S1) {
            __builtin_amdgcn_s_waitcnt(0);  // the interior loop starts with nothing in flight
            do {
                steady<0>(R);
                steady<1>(R + 1);
                steady<2>(R + 2);
                steady<3>(R + 3);
                R += 4;
            } while (R + 3 <= S1);
        }
        for (;;) {
            if (R > Rend) break;
            iter<0>(R);
            if (++R > Rend) break;
            iter<1>(R);
            if (++R > Rend) break;
            iter<2>(R);
            if (++R > Rend) break;
            iter<3>(R);
            ++R;
        }
    }
};

// One strip-segment per workgroup.  The lattice's columns are split evenly into
// `strips` strips of at most MARCH_OWN columns and its rows evenly into `segs`
// segments of at least 4 rows (so only the first segment touches the bottom wall
// rows).  The host keeps the nine planes of one buffer below 2 GiB (32-bit buffer
// offsets) and sizes the grid so that every workgroup is resident at once.
#ifndef MARCH_WAVES_PER_EU
#define MARCH_WAVES_PER_EU 4
#endif
template <typename ST, int EOS>
__global__ __launch_bounds__(MARCH_NT) __attribute__((amdgpu_waves_per_eu(MARCH_WAVES_PER_EU))) void march_kernel(
    LatticeArgs A, const ST* __restrict__ fin, ST* __restrict__ fout,
    const typename Codec<ST>::CT* __restrict__ mu_w, int strips, int segs) {
    using CT = typename Codec<ST>::CT;
    using M_t = March<ST, EOS>;
    __shared__ CT rs[8][MARCH_NT + 2];
    __shared__ CT ms[4][MARCH_NT + 2];
    const int t = tile_of_block(blockIdx.x, gridDim.x);
    const int s = t % strips, g = t / strips;
    M_t M{A};
    M.rs = rs;
    M.ms = ms;
    M.mu_w = in_global(mu_w);
    const int bytes = int(9LL * A.ny * A.pitch * (long long)sizeof(ST));
    M.rin = buffer_of(fin, bytes);
    M.rout = buffer_of(fout, bytes);
    M.l = threadIdx.x;
    M.ys = int((long long)g * A.ny / segs);
    M.ye = int((long long)(g + 1) * A.ny / segs);
    const int x0 = int((long long)s * A.nx / strips), x1 = int((long long)(s + 1) * A.nx / strips);
    const int xr = x0 - 2 + M.l;  // this lane's raw column
    M.xr = xr;
    M.xw = wrap_col(xr, A.nx);
    M.walled = A.bottom != BC_PERIODIC;
    M.live = xr < x1 + 2;
    M.mu_lane = M.l >= 1 && xr < x1 + 1;
    M.owned = M.l >= 2 && xr < x1;
    M.nr = M.live && M.l < MARCH_NT - 1 && xr + 1 < x1 + 2;
    // lanes past the strip's halo read nowhere (zero, no memory traffic)
    M.vc = M.live ? M.xw * int(sizeof(ST)) : M_t::NOWHERE;
    M.vm = M.live ? wrap_col(xr - 1, A.nx) * int(sizeof(ST)) : M_t::NOWHERE;
    M.vp = M.live ? wrap_col(xr + 1, A.nx) * int(sizeof(ST)) : M_t::NOWHERE;
    M.vs = M.owned ? M.vc : M_t::NOWHERE;
    M.PB = int(A.plane * (long long)sizeof(ST));
    M.RB = A.fpitch * int(sizeof(ST));
    M.b0 = CT(A.rho_ref) * Wt<CT>::w0;
    M.b1 = CT(A.rho_ref) * Wt<CT>::w1;
    M.b2 = CT(A.rho_ref) * Wt<CT>::w2;
    M.tau = CT(A.tau);
    M.inv_tau = CT(A.inv_tau);
    M.kappa = CT(A.kappa);
    M.run();
}

// ---------------------------------------------------------------- monitors
constexpr int MON_THREADS = 256;
constexpr int MON_BLOCKS_MAX = 1024;

int mon_blocks(const LatticeArgs& A) {
    const long long n = (long long)A.nx * A.ny;
    const long long nb = (n + MON_THREADS - 1) / MON_THREADS;
    return int(nb < MON_BLOCKS_MAX ? (nb < 1 ? 1 : nb) : MON_BLOCKS_MAX);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

// Densities of the current state; compare == 1 also accumulates the mass, the
// largest change since the last snapshot and the divergence flags per block.
template <typename ST, int COMPARE>
__global__ __launch_bounds__(MON_THREADS) void monitor_kernel(LatticeArgs A, const ST* __restrict__ fin,
                                                              typename Codec<ST>::CT* __restrict__ rho_mon,
                                                              double* __restrict__ partials) {
    using CT = typename Codec<ST>::CT;
    Planes<ST> F;
#pragma unroll
    for (int i = 0; i < 9; ++i) F.p[i] = fin + (long long)i * A.plane;
    double mass = 0.0, res = 0.0;
    int flags = 0;
    const long long n = (long long)A.nx * A.ny;
    for (long long c = (long long)blockIdx.x * MON_THREADS + threadIdx.x; c < n;
         c += (long long)gridDim.x * MON_THREADS) {
        const int y = int(c / A.nx), x = int(c % A.nx);
        if (solid_row(A, y)) continue;
        const CT r = fluid_rho<ST, CT>(A, F, x, y);
        const int o = y * A.pitch + x;
        if (COMPARE) {
            const double rd = double(r);
            mass += rd;
            const double d = fabs(rd - double(rho_mon[o]));
            res = d > res ? d : res;
            if (!(rd == rd) || isinf(rd)) flags |= 1;
            else if (rd <= 0.0) flags |= 2;
            else if (rd >= A.eos.rho_max) flags |= 4;
            if (!(d == d)) res = d;  // propagate NaN
        }
        rho_mon[o] = r;
    }
    if (!COMPARE) return;
    __shared__ double s_mass[MON_THREADS / 64], s_res[MON_THREADS / 64];
    __shared__ int s_flags[MON_THREADS / 64];
    mass = wave_sum(mass);
    res = wave_max(res);
    flags = wave_or(flags);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        s_mass[w] = mass;
        s_res[w] = res;
        s_flags[w] = flags;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0, rr = 0.0;
        int fl = 0;
        for (int i = 0; i < MON_THREADS / 64; ++i) {
            m += s_mass[i];
            rr = fmax(rr, s_res[i]);
            fl |= s_flags[i];
        }
        partials[3 * blockIdx.x] = m;
        partials[3 * blockIdx.x + 1] = rr;
        partials[3 * blockIdx.x + 2] = double(fl);
    }
}

// Fixed-order reduction of the per-block partials (deterministic).
__global__ __launch_bounds__(64) void monitor_reduce(const double* __restrict__ partials, int nblk,
                                                     double* __restrict__ mon) {
    double m = 0.0, r = 0.0;
    int fl = 0;
    for (int b = threadIdx.x; b < nblk; b += 64) {
        m += partials[3 * b];
        r = fmax(r, partials[3 * b + 1]);
        fl |= int(partials[3 * b + 2]);
    }
    m = wave_sum(m);
    r = wave_max(r);
    fl = wave_or(fl);
    if (threadIdx.x == 0) {
        mon[0] = m;
        mon[1] = r;
        mon[2] = double(fl);
    }
}

// Monitors of many lattices: one workgroup per (case, tile); per-tile partials, then
// one workgroup per case reduces its contiguous tile range in a fixed order.
// TY == 0: each case's own tile shape, from its shape code (the mixed schedule).
template <typename ST, int COMPARE, int TY_, int TX_ = TILE_X>
__global__ __launch_bounds__(MON_THREADS) void batch_monitor_kernel(const CaseDesc* __restrict__ cases,
                                                                    const int2* __restrict__ tiles, int parity,
                                                                    double* __restrict__ partials) {
    using CT = typename Codec<ST>::CT;
    const int2 w = tiles[blockIdx.x];
    const CaseDesc& C = cases[w.x];
    const LatticeArgs& A = C.A;
    const int TY = TY_ ? TY_ : tile_ty(A.tile_y), TX = TY_ ? TX_ : tile_tx(A.tile_y);
    Planes<ST> F;
    const ST* fin = in_global(static_cast<const ST*>(C.f[parity]));
#pragma unroll
    for (int i = 0; i < 9; ++i) F.p[i] = fin + (long long)i * A.plane;
    CT* rho_mon = in_global(static_cast<CT*>(C.rho_mon));
    const int tiles_x = (A.nx + TX - 1) / TX;
    const int x0 = (w.y % tiles_x) * TX, y0 = (w.y / tiles_x) * TY;
    double mass = 0.0, res = 0.0;
    int flags = 0;
    for (int i = threadIdx.x; i < TX * TY; i += MON_THREADS) {
        const int x = x0 + i % TX, y = y0 + i / TX;
        if (x >= A.nx || y >= A.ny || solid_row(A, y)) continue;
        const CT r = fluid_rho<ST, CT>(A, F, x, y);
        const unsigned o = unsigned(y) * unsigned(A.pitch) + unsigned(x);
        if (COMPARE) {
            const double rd = double(r);
            mass += rd;
            const double d = fabs(rd - double(rho_mon[o]));
            res = d > res ? d : res;
            if (!(rd == rd) || isinf(rd)) flags |= 1;
            else if (rd <= 0.0) flags |= 2;
            else if (rd >= A.eos.rho_max) flags |= 4;
            if (!(d == d)) res = d;
        }
        rho_mon[o] = r;
    }
    if (!COMPARE) return;
    __shared__ double s_mass[MON_THREADS / 64], s_res[MON_THREADS / 64];
    __shared__ int s_flags[MON_THREADS / 64];
    mass = wave_sum(mass);
    res = wave_max(res);
    flags = wave_or(flags);
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        s_mass[wv] = mass;
        s_res[wv] = res;
        s_flags[wv] = flags;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0, rr = 0.0;
        int fl = 0;
        for (int i = 0; i < MON_THREADS / 64; ++i) {
            m += s_mass[i];
            rr = fmax(rr, s_res[i]);
            fl |= s_flags[i];
        }
        partials[3 * blockIdx.x] = m;
        partials[3 * blockIdx.x + 1] = rr;
        partials[3 * blockIdx.x + 2] = double(fl);
    }
}

__global__ __launch_bounds__(64) void batch_monitor_reduce(const double* __restrict__ partials,
                                                           const int* __restrict__ case_tile_begin,
                                                           double* __restrict__ case_mon) {
    const int c = blockIdx.x;
    const int b0 = case_tile_begin[c], b1 = case_tile_begin[c + 1];
    if (b0 == b1) return;  // inactive case: keep its last values
    double m = 0.0, r = 0.0;
    int fl = 0;
    for (int b = b0 + int(threadIdx.x); b < b1; b += 64) {
        m += partials[3 * b];
        r = fmax(r, partials[3 * b + 1]);
        fl |= int(partials[3 * b + 2]);
    }
    m = wave_sum(m);
    r = wave_max(r);
    fl = wave_or(fl);
    if (threadIdx.x == 0) {
        case_mon[3 * c] = m;
        case_mon[3 * c + 1] = r;
        case_mon[3 * c + 2] = double(fl);
    }
}

// ---------------------------------------------------------------- state conversion
__device__ __forceinline__ double feq_d(int i, double rho, double ux, double uy) {
    constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const double w = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    const double eu = ex[i] * ux + ey[i] * uy;
    return w * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy));
}

// Storage value S_j(x) = f_j(x + e_j) if x + e_j is fluid, else f_opp(j)(x): the
// inverse of the pull, so that the next pull returns exactly f(t).
template <typename ST>
__global__ void init_kernel(LatticeArgs A, const double* __restrict__ rho0, const double* __restrict__ ux0,
                            const double* __restrict__ uy0, const double* __restrict__ f_in,
                            ST* __restrict__ fstore) {
    using CT = typename Codec<ST>::CT;
    constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    const long long n = (long long)A.nx * A.ny;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int y = int(c / A.nx), x = int(c % A.nx);
    const unsigned o = unsigned(y) * unsigned(A.fpitch) + unsigned(x);
    if (solid_row(A, y)) {
        for (int j = 0; j < 9; ++j) Codec<ST>::st(fstore + (long long)j * A.plane, o, CT(0), CT(0));
        return;
    }
    const double wr[3] = {A.rho_ref * 4.0 / 9.0, A.rho_ref / 9.0, A.rho_ref / 36.0};
    for (int j = 0; j < 9; ++j) {
        int xt = x + ex[j], yt = y + ey[j];
        xt = xt < 0 ? xt + A.nx : (xt >= A.nx ? xt - A.nx : xt);
        if (A.bottom == BC_PERIODIC) yt = yt < 0 ? yt + A.ny : (yt >= A.ny ? yt - A.ny : yt);
        int src_dir = j;
        long long src = (long long)yt * A.nx + xt;
        if (A.bottom != BC_PERIODIC && solid_row(A, yt)) {
            src_dir = opp[j];
            src = c;
        }
        double v;
        if (f_in) {
            v = f_in[(long long)src_dir * n + src];
        } else {
            v = feq_d(src_dir, rho0[src], ux0 ? ux0[src] : 0.0, uy0 ? uy0[src] : 0.0);
        }
        const CT base = CT(j == 0 ? wr[0] : (j < 5 ? wr[1] : wr[2]));
        Codec<ST>::st(fstore + (long long)j * A.plane, o, CT(v), base);
    }
}

template <typename ST>
__global__ void get_state_kernel(LatticeArgs A, const ST* __restrict__ fstore, double* __restrict__ f_out) {
    using CT = typename Codec<ST>::CT;
    const long long n = (long long)A.nx * A.ny;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int y = int(c / A.nx), x = int(c % A.nx);
    if (solid_row(A, y)) {
        for (int i = 0; i < 9; ++i) f_out[(long long)i * n + c] = 0.0;
        return;
    }
    Planes<ST> F;
    for (int i = 0; i < 9; ++i) F.p[i] = fstore + (long long)i * A.plane;
    CT f[9];
    pull9<ST, CT>(A, F, x, y, f);
    for (int i = 0; i < 9; ++i) f_out[(long long)i * n + c] = double(f[i]);
}

template <typename ST, int EOS, int MODE, int TY, int TX, int RPT, bool HOIST = false, int FORCE = FORCE_CP,
          int COLL = COLLIDE_BGK, bool NTS = false>
hipError_t step_launch(const LatticeArgs& A, const void* fin, void* fout, const void* mu_w, double* out,
                       hipStream_t s) {
    using CT = typename Codec<ST>::CT;
    const int tiles = ((A.nx + TX - 1) / TX) * ((A.ny + TY - 1) / TY);
    (void)hipGetLastError();  // drop any error left by earlier runtime calls
    hipLaunchKernelGGL((step_kernel<ST, EOS, MODE, TY, TX, RPT, HOIST, FORCE, COLL, NTS>), dim3(tiles),
                       dim3(TX * TY / RPT), 0, s, A, (const ST*)fin, (ST*)fout, (const CT*)mu_w, out);
    return hipGetLastError();
}

// The variants of the step (force of Eq 5, TRT / MRT collision): 64 x 16 tiles,
// FP64 and FP32 storage, with the non-temporal stores of the plain step where it
// takes them (so that the variants compare like with like).
template <typename ST, int EOS, int MODE, bool NTS>
hipError_t step_scheme_nt(const LatticeArgs& A, const void* fin, void* fout, const void* mu_w, double* out,
                          hipStream_t s) {
    static_assert(SCHEME_TILE_Y == 16, "the variants are instantiated for 64 x 16 tiles");
    switch (A.scheme) {
    case FORCE_CP | COLLIDE_TRT:
        return step_launch<ST, EOS, MODE, 16, 64, 4, false, FORCE_CP, COLLIDE_TRT, NTS>(A, fin, fout, mu_w, out, s);
    case FORCE_CP | COLLIDE_MRT:
        return step_launch<ST, EOS, MODE, 16, 64, 4, false, FORCE_CP, COLLIDE_MRT, NTS>(A, fin, fout, mu_w, out, s);
    case FORCE_PTENSOR | COLLIDE_BGK:
        return step_launch<ST, EOS, MODE, 16, 64, 4, false, FORCE_PTENSOR, COLLIDE_BGK, NTS>(A, fin, fout, mu_w, out,
                                                                                             s);
    case FORCE_PTENSOR | COLLIDE_TRT:
        return step_launch<ST, EOS, MODE, 16, 64, 4, false, FORCE_PTENSOR, COLLIDE_TRT, NTS>(A, fin, fout, mu_w, out,
                                                                                             s);
    case FORCE_PTENSOR | COLLIDE_MRT:
        return step_launch<ST, EOS, MODE, 16, 64, 4, false, FORCE_PTENSOR, COLLIDE_MRT, NTS>(A, fin, fout, mu_w, out,
                                                                                             s);
    default: return hipErrorInvalidValue;
    }
}

template <typename ST, int EOS, int MODE>
hipError_t step_scheme(const LatticeArgs& A, const void* fin, void* fout, const void* mu_w, double* out,
                       hipStream_t s) {
    if constexpr (sizeof(ST) < 4) {
        return hipErrorInvalidValue;
    } else {
        if constexpr (MODE == MODE_STEP) {
            if (A.nt_store) return step_scheme_nt<ST, EOS, MODE, true>(A, fin, fout, mu_w, out, s);
        }
        return step_scheme_nt<ST, EOS, MODE, false>(A, fin, fout, mu_w, out, s);
    }
}

template <typename ST, int EOS, int MODE, bool NTS>
hipError_t step_ty_nt(int tile_y, const LatticeArgs& A, const void* fin, void* fout, const void* mu_w, double* out,
                      hipStream_t s) {
    constexpr int F = FORCE_CP, B = COLLIDE_BGK;
    switch (tile_y) {
    case 8: return step_launch<ST, EOS, MODE, 8, 64, 4, false, F, B, NTS>(A, fin, fout, mu_w, out, s);
    case 16: return step_launch<ST, EOS, MODE, 16, 64, 4, false, F, B, NTS>(A, fin, fout, mu_w, out, s);
    case 32: return step_launch<ST, EOS, MODE, 32, 64, 4, false, F, B, NTS>(A, fin, fout, mu_w, out, s);
    case 12816: return step_launch<ST, EOS, MODE, 16, 128, 4, false, F, B, NTS>(A, fin, fout, mu_w, out, s);
    case 12832: return step_launch<ST, EOS, MODE, 32, 128, 8, false, F, B, NTS>(A, fin, fout, mu_w, out, s);
    case 25608: return step_launch<ST, EOS, MODE, 8, 256, 4, false, F, B, NTS>(A, fin, fout, mu_w, out, s);
    case 25616: return step_launch<ST, EOS, MODE, 16, 256, 8, false, F, B, NTS>(A, fin, fout, mu_w, out, s);
    case HOIST_BASE + 16: return step_launch<ST, EOS, MODE, 16, 64, 4, true, F, B, NTS>(A, fin, fout, mu_w, out, s);
    case HOIST_BASE + 32: return step_launch<ST, EOS, MODE, 32, 64, 4, true, F, B, NTS>(A, fin, fout, mu_w, out, s);
    default: return hipErrorInvalidValue;
    }
}

// Field output stores no distributions: one form.
template <typename ST, int EOS, int MODE>
hipError_t step_ty(int tile_y, const LatticeArgs& A, const void* fin, void* fout, const void* mu_w, double* out,
                   hipStream_t s) {
    if constexpr (MODE == MODE_STEP) {
        if (A.nt_store) return step_ty_nt<ST, EOS, MODE, true>(tile_y, A, fin, fout, mu_w, out, s);
    }
    return step_ty_nt<ST, EOS, MODE, false>(tile_y, A, fin, fout, mu_w, out, s);
}

// Column-marching launch with k resident workgroups per CU: the rows are split
// into as many segments as fill k workgroups per CU over all strips (one round).
template <typename ST, int EOS>
hipError_t march_launch(int k, const LatticeArgs& A, const void* fin, void* fout, const void* mu_w, hipStream_t s) {
    using CT = typename Codec<ST>::CT;
    if (k < 1 || k > MARCH_K_MAX || 9LL * A.ny * A.pitch * (long long)sizeof(ST) > MARCH_MAX_BYTES)
        return hipErrorInvalidValue;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    const long long strips = (A.nx + MARCH_OWN - 1) / MARCH_OWN;
    long long segs = (long long)k * cus / strips;
    segs = std::min<long long>(segs, A.ny / 4);
    segs = std::max<long long>(segs, 1);
    (void)hipGetLastError();
    hipLaunchKernelGGL((march_kernel<ST, EOS>), dim3(unsigned(strips * segs)), dim3(MARCH_NT), 0, s, A,
                       (const ST*)fin, (ST*)fout, (const CT*)mu_w, int(strips), int(segs));
    return hipGetLastError();
}

template <typename ST, int EOS>
hipError_t step_eos(int mode, int tile_y, const LatticeArgs& A, const void* fin, void* fout, const void* mu_w,
                    double* out, hipStream_t s) {
    if (A.scheme != 0)
        return mode == MODE_STEP ? step_scheme<ST, EOS, MODE_STEP>(A, fin, fout, mu_w, out, s)
                                 : step_scheme<ST, EOS, MODE_FIELDS>(A, fin, fout, mu_w, out, s);
    if (mode == MODE_STEP && tile_y < 0) return march_launch<ST, EOS>(-tile_y, A, fin, fout, mu_w, s);
    if (mode == MODE_STEP) return step_ty<ST, EOS, MODE_STEP>(tile_y, A, fin, fout, mu_w, out, s);
    return step_ty<ST, EOS, MODE_FIELDS>(16, A, fin, fout, mu_w, out, s);  // output uses one shape
}

template <typename ST>
hipError_t step_prec(int eos, int mode, int tile_y, const LatticeArgs& A, const void* fin, void* fout,
                     const void* mu_w, double* out, hipStream_t s) {
    switch (eos) {
    case EOS_VDW: return step_eos<ST, EOS_VDW>(mode, tile_y, A, fin, fout, mu_w, out, s);
    case EOS_CS: return step_eos<ST, EOS_CS>(mode, tile_y, A, fin, fout, mu_w, out, s);
    case EOS_PR: return step_eos<ST, EOS_PR>(mode, tile_y, A, fin, fout, mu_w, out, s);
    case EOS_RKS:
    case EOS_RK: return step_eos<ST, EOS_RK>(mode, tile_y, A, fin, fout, mu_w, out, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename ST>
hipError_t monitor_prec(int compare, const LatticeArgs& A, const void* fin, void* rho_mon, double* partials,
                        double* mon, hipStream_t s) {
    using CT = typename Codec<ST>::CT;
    const int nb = mon_blocks(A);
    (void)hipGetLastError();
    if (compare) {
        hipLaunchKernelGGL((monitor_kernel<ST, 1>), dim3(nb), dim3(MON_THREADS), 0, s, A, (const ST*)fin,
                           (CT*)rho_mon, partials);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(monitor_reduce, dim3(1), dim3(64), 0, s, partials, nb, mon);
    } else {
        hipLaunchKernelGGL((monitor_kernel<ST, 0>), dim3(nb), dim3(MON_THREADS), 0, s, A, (const ST*)fin,
                           (CT*)rho_mon, partials);
    }
    return hipGetLastError();
}

template <typename ST, int TY, int TX>
void batch_step_one(int grid, bool nt, const CaseDesc* cases, const int2* tiles, int ntiles, int parity,
                    hipStream_t s) {
    if (nt)
        hipLaunchKernelGGL((batch_step_kernel<ST, TY, TX, true>), dim3(grid), dim3(TX * TY / ROWS_PER_THREAD), 0, s,
                           cases, tiles, ntiles, parity);
    else
        hipLaunchKernelGGL((batch_step_kernel<ST, TY, TX, false>), dim3(grid), dim3(TX * TY / ROWS_PER_THREAD), 0, s,
                           cases, tiles, ntiles, parity);
}

// code: a 64-wide tile height (8, 16, 32) or a wide shape code (12816, 25608)
template <typename ST>
hipError_t batch_step_prec(int code, int nt, const CaseDesc* cases, const int2* tiles, int ntiles, int parity,
                           int grid, hipStream_t s) {
    (void)hipGetLastError();
    switch (code) {
    case BATCH_MIXED:
        if (nt)
            hipLaunchKernelGGL((batch_step_mixed_kernel<ST, true>), dim3(grid), dim3(512), 0, s, cases, tiles, ntiles,
                               parity);
        else
            hipLaunchKernelGGL((batch_step_mixed_kernel<ST, false>), dim3(grid), dim3(512), 0, s, cases, tiles, ntiles,
                               parity);
        break;
    case 8: batch_step_one<ST, 8, 64>(grid, nt, cases, tiles, ntiles, parity, s); break;
    case 16: batch_step_one<ST, 16, 64>(grid, nt, cases, tiles, ntiles, parity, s); break;
    case 32: batch_step_one<ST, 32, 64>(grid, nt, cases, tiles, ntiles, parity, s); break;
    case 12816: batch_step_one<ST, 16, 128>(grid, nt, cases, tiles, ntiles, parity, s); break;
    case 25608: batch_step_one<ST, 8, 256>(grid, nt, cases, tiles, ntiles, parity, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename ST, int COMPARE, int TY, int TX>
void batch_monitor_one(int ntiles, const CaseDesc* cases, const int2* tiles, int parity, double* partials,
                       hipStream_t s) {
    hipLaunchKernelGGL((batch_monitor_kernel<ST, COMPARE, TY, TX>), dim3(ntiles), dim3(MON_THREADS), 0, s, cases,
                       tiles, parity, partials);
}

template <typename ST, int COMPARE>
hipError_t batch_monitor_ty(int code, const CaseDesc* cases, const int2* tiles, int ntiles, int parity,
                            double* partials, hipStream_t s) {
    switch (code) {
    case BATCH_MIXED: batch_monitor_one<ST, COMPARE, 0, 0>(ntiles, cases, tiles, parity, partials, s); break;
    case 8: batch_monitor_one<ST, COMPARE, 8, 64>(ntiles, cases, tiles, parity, partials, s); break;
    case 16: batch_monitor_one<ST, COMPARE, 16, 64>(ntiles, cases, tiles, parity, partials, s); break;
    case 32: batch_monitor_one<ST, COMPARE, 32, 64>(ntiles, cases, tiles, parity, partials, s); break;
    case 12816: batch_monitor_one<ST, COMPARE, 16, 128>(ntiles, cases, tiles, parity, partials, s); break;
    case 25608: batch_monitor_one<ST, COMPARE, 8, 256>(ntiles, cases, tiles, parity, partials, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename ST>
hipError_t batch_monitor_prec(int compare, int tile_y, const CaseDesc* cases, const int2* tiles, int ntiles,
                              int parity, double* partials, const int* case_tile_begin, int ncases,
                              double* case_mon, hipStream_t s) {
    (void)hipGetLastError();
    if (ntiles == 0) return hipSuccess;
    hipError_t e = compare ? batch_monitor_ty<ST, 1>(tile_y, cases, tiles, ntiles, parity, partials, s)
                           : batch_monitor_ty<ST, 0>(tile_y, cases, tiles, ntiles, parity, partials, s);
    if (e != hipSuccess || !compare) return e;
    hipLaunchKernelGGL(batch_monitor_reduce, dim3(ncases), dim3(64), 0, s, partials, case_tile_begin, case_mon);
    return hipGetLastError();
}

template <typename ST>
int batch_occupancy(int code) {
    int n = 0;
    const int threads = code == BATCH_MIXED ? 512 : tile_tx(code) * tile_ty(code) / ROWS_PER_THREAD;
    const void* k = nullptr;
    switch (code) {
    case BATCH_MIXED: k = (const void*)batch_step_mixed_kernel<ST, false>; break;
    case 8: k = (const void*)batch_step_kernel<ST, 8, 64>; break;
    case 16: k = (const void*)batch_step_kernel<ST, 16, 64>; break;
    case 32: k = (const void*)batch_step_kernel<ST, 32, 64>; break;
    case 12816: k = (const void*)batch_step_kernel<ST, 16, 128>; break;
    default: k = (const void*)batch_step_kernel<ST, 8, 256>; break;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, threads, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

template <typename ST>
hipError_t init_prec(const LatticeArgs& A, const double* rho0, const double* ux0, const double* uy0,
                            const double* f_in, void* fstore, hipStream_t s) {
    const long long n = (long long)A.nx * A.ny;
    const int blocks = int((n + 255) / 256);
    (void)hipGetLastError();
    hipLaunchKernelGGL((init_kernel<ST>), dim3(blocks), dim3(256), 0, s, A, rho0, ux0, uy0, f_in, (ST*)fstore);
    return hipGetLastError();
}

template <typename ST>
hipError_t get_state_prec(const LatticeArgs& A, const void* fstore, double* f_out, hipStream_t s) {
    const long long n = (long long)A.nx * A.ny;
    const int blocks = int((n + 255) / 256);
    (void)hipGetLastError();
    hipLaunchKernelGGL((get_state_kernel<ST>), dim3(blocks), dim3(256), 0, s, A, (const ST*)fstore, f_out);
    return hipGetLastError();
}

}  // namespace

// Entry points of this translation unit, for one storage type (CPLBM_ST); the
// dispatch over storage types is in lbm_dispatch.cpp.
#define CPLBM_CAT2(a, b) a##_##b
#define CPLBM_CAT(a, b) CPLBM_CAT2(a, b)
#define CPLBM_FN(name) CPLBM_CAT(name, CPLBM_SUFFIX)

hipError_t CPLBM_FN(launch_step)(int eos, int mode, const LatticeArgs& A, const void* fin, void* fout,
                                 const void* mu_w, double* out, hipStream_t s) {
    return step_prec<CPLBM_ST>(eos, mode, A.tile_y, A, fin, fout, mu_w, out, s);
}

hipError_t CPLBM_FN(launch_monitor)(int compare, const LatticeArgs& A, const void* fin, void* rho_mon,
                                    double* partials, double* mon, hipStream_t s) {
    return monitor_prec<CPLBM_ST>(compare, A, fin, rho_mon, partials, mon, s);
}

hipError_t CPLBM_FN(launch_batch_step)(int tile_y, int nt, const CaseDesc* cases, const int2* tiles, int ntiles,
                                       int parity, int grid, hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    return batch_step_prec<CPLBM_ST>(tile_y, nt, cases, tiles, ntiles, parity, grid, s);
}

hipError_t CPLBM_FN(launch_batch_monitor)(int compare, int tile_y, const CaseDesc* cases, const int2* tiles,
                                          int ntiles, int parity, double* partials, const int* case_tile_begin,
                                          int ncases, double* case_mon, hipStream_t s) {
    return batch_monitor_prec<CPLBM_ST>(compare, tile_y, cases, tiles, ntiles, parity, partials, case_tile_begin,
                                        ncases, case_mon, s);
}

int CPLBM_FN(batch_blocks_per_cu)(int tile_y) { return batch_occupancy<CPLBM_ST>(tile_y); }

hipError_t CPLBM_FN(launch_init)(const LatticeArgs& A, const double* rho0, const double* ux0, const double* uy0,
                                 const double* f_in, void* fstore, hipStream_t s) {
    return init_prec<CPLBM_ST>(A, rho0, ux0, uy0, f_in, fstore, s);
}

hipError_t CPLBM_FN(launch_get_state)(const LatticeArgs& A, const void* fstore, double* f_out, hipStream_t s) {
    return get_state_prec<CPLBM_ST>(A, fstore, f_out, s);
}

}  // namespace cplbm
