// HIP kernels of the chemical-potential lattice Boltzmann step for CDNA4 (gfx950).
//
// Storage: nine direction planes f[i][y][x] (SoA, row pitch a multiple of 64
// elements) holding the post-collision distributions f*(t-1).  A step pulls
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

template <typename ST>
struct Codec;

template <>
struct Codec<double> {
    using CT = double;
    static __device__ __forceinline__ double ld(const double* p, unsigned o, double) { return *at(p, o); }
    static __device__ __forceinline__ void st(double* p, unsigned o, double v, double) { *at(p, o) = v; }
};
template <>
struct Codec<float> {
    using CT = float;
    static __device__ __forceinline__ float ld(const float* p, unsigned o, float) { return *at(p, o); }
    static __device__ __forceinline__ void st(float* p, unsigned o, float v, float) { *at(p, o) = v; }
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
template <typename ST, typename CT>
__device__ __forceinline__ void pull9(const LatticeArgs& A, const Planes<ST>& F, int gx, int gy,
                                      CT f[9]) {
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
    const unsigned pitch = unsigned(A.pitch), ux = unsigned(gx), uxm = unsigned(xm), uxp = unsigned(xp);
    const unsigned rc = unsigned(gy) * pitch, rm = unsigned(ym) * pitch, rp = unsigned(yp) * pitch;
    f[0] = C::ld(F.p[0], rc + ux, b0);
    f[1] = C::ld(F.p[1], rc + uxm, b1);
    f[3] = C::ld(F.p[3], rc + uxp, b1);
    if (sm) {  // links from the wall below return reversed (halfway bounce-back)
        f[2] = C::ld(F.p[4], rc + ux, b1);
        f[5] = C::ld(F.p[7], rc + ux, b2);
        f[6] = C::ld(F.p[8], rc + ux, b2);
    } else {
        f[2] = C::ld(F.p[2], rm + ux, b1);
        f[5] = C::ld(F.p[5], rm + uxm, b2);
        f[6] = C::ld(F.p[6], rm + uxp, b2);
    }
    if (sp) {
        f[4] = C::ld(F.p[2], rc + ux, b1);
        f[7] = C::ld(F.p[5], rc + ux, b2);
        f[8] = C::ld(F.p[6], rc + ux, b2);
    } else {
        f[4] = C::ld(F.p[4], rp + ux, b1);
        f[7] = C::ld(F.p[7], rp + uxp, b2);
        f[8] = C::ld(F.p[8], rp + uxm, b2);
    }
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
// Bulk chemical potential psi'(rho): Eq 18 (VdW), Eq 27 (CS), Eq 24 (PR), Eq 21 (RK, RKS).
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
            return rep - c1 * lg((s2 - CT(1) + br) * rcp(s2 + CT(1) - br)) -
                   a * rho * rcp(CT(1) + CT(2) * br - br * br);
        } else {  // RK, RKS
            return rep - c1 * lg(CT(1) + br) - a * rho * rcp(CT(1) + br);
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

__device__ __forceinline__ int tile_of_block(int b, int nblk) {
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
    // band of tiles so that halos shared by neighbouring tiles stay in its L2.
    const int q = nblk >> 3, r = nblk & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// ---------------------------------------------------------------- the fused step
template <typename CT, int TY>
struct TileLds {
    CT rs[TY + 4][TILE_X + 4];  // density, tile + 2-node ring
    CT ms[TY + 2][TILE_X + 2];  // chemical potential, tile + 1-node ring
};

// One TILE_X x TY tile of the step (MODE_STEP) or of the field output (MODE_FIELDS),
// run by a workgroup of TILE_X * TY / ROWS_PER_THREAD threads.
template <typename ST, int EOS, int MODE, int TY>
__device__ __forceinline__ void step_tile(const LatticeArgs& A, const ST* __restrict__ fin,
                                          ST* __restrict__ fout,
                                          const typename Codec<ST>::CT* __restrict__ mu_w,
                                          double* __restrict__ out, int x0, int y0,
                                          TileLds<typename Codec<ST>::CT, TY>& L) {
    using CT = typename Codec<ST>::CT;
    using C = Codec<ST>;
    constexpr int RW = TILE_X + 4, MW = TILE_X + 2;
    constexpr int NT = TILE_X * TY / ROWS_PER_THREAD;  // threads
    constexpr int RS = TY / ROWS_PER_THREAD;           // row stride between a thread's nodes
    auto& rs = L.rs;
    auto& ms = L.ms;

    Planes<ST> F;
#pragma unroll
    for (int i = 0; i < 9; ++i) F.p[i] = fin + (long long)i * A.plane;

    const int lx = threadIdx.x % TILE_X, ly = threadIdx.x / TILE_X;
    const bool small_x = A.nx < TILE_X + 2, small_y = A.ny < TY + 2;

    // 1. own nodes: pull, keep f, density into LDS
    CT f[ROWS_PER_THREAD][9];
    CT jx[ROWS_PER_THREAD], jy[ROWS_PER_THREAD];
    const int gx_raw = x0 + lx;
    const int gxw = wrap_fast(gx_raw, A.nx, small_x);
#pragma unroll
    for (int k = 0; k < ROWS_PER_THREAD; ++k) {
        const int gy = y0 + ly + k * RS;
        const bool own = gx_raw < A.nx && gy < A.ny && !solid_row(A, gy);
        CT r;
        if (own) {
            pull9<ST, CT>(A, F, gxw, gy, f[k]);
            r = sum9(f[k]);
            jx[k] = ((f[k][1] - f[k][3]) + (f[k][5] - f[k][6])) + (f[k][8] - f[k][7]);
            jy[k] = ((f[k][2] - f[k][4]) + (f[k][5] + f[k][6])) - (f[k][7] + f[k][8]);
        } else {
            r = node_rho<ST, CT>(A, F, gxw, gy, small_y);
        }
        rs[ly + k * RS + 2][lx + 2] = r;
    }

    // 2. the two-node ring of densities around the tile
    constexpr int RING = 2 * RW * 2 + 2 * TY * 2;
    for (int q = threadIdx.x; q < RING; q += NT) {
        int r, c;
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
            c = TILE_X + 2 + (q - 4 * RW - 2 * TY) % 2;
        }
        rs[r][c] = node_rho<ST, CT>(A, F, wrap_fast(x0 - 2 + c, A.nx, small_x), y0 - 2 + r, small_y);
    }
    __syncthreads();

    // 3. chemical potential, Eq 8, on the tile and a one-node ring
    const CT kappa = CT(A.kappa);
    for (int q = threadIdx.x; q < (TY + 2) * MW; q += NT) {
        const int r = q / MW, c = q % MW;
        const int y = y0 - 1 + r;
        CT m;
        if (A.bottom == BC_PERIODIC) {
            m = mu_bulk<EOS, CT>(A.eos, rs[r + 1][c + 1]) - kappa * lap9<CT, RW>(rs, r + 1, c + 1);
        } else if (y <= 0 || y >= A.ny - 1) {
            if (y == 0 || y == A.ny - 1) {
                const int kind = y == 0 ? A.bottom : A.top;
                if (kind == BC_CPWALL) {
                    m = mu_w[(y == 0 ? 0 : A.pitch) + wrap_fast(x0 - 1 + c, A.nx, small_x)];
                } else {  // neutral wall: the chemical potential of the adjacent fluid node
                    const int rn = y == 0 ? r + 2 : r;
                    m = mu_bulk<EOS, CT>(A.eos, rs[rn][c + 1]) - kappa * lap9<CT, RW>(rs, rn, c + 1);
                }
            } else {
                m = CT(0);  // outside the lattice: never read
            }
        } else {
            m = mu_bulk<EOS, CT>(A.eos, rs[r + 1][c + 1]) - kappa * lap9<CT, RW>(rs, r + 1, c + 1);
        }
        ms[r][c] = m;
    }
    __syncthreads();

    // 4. force (Eq 12), collision (Eqs 13, 14, u_eq = u + tau F / rho), store
    const CT tau = CT(A.tau), inv_tau = CT(A.inv_tau);
    const CT b0 = CT(A.rho_ref) * Wt<CT>::w0, b1 = CT(A.rho_ref) * Wt<CT>::w1,
             b2 = CT(A.rho_ref) * Wt<CT>::w2;
#pragma unroll
    for (int k = 0; k < ROWS_PER_THREAD; ++k) {
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
        grad9<CT, MW>(ms, ry + 1, lx + 1, gmx, gmy);
        grad9<CT, RW>(rs, ry + 2, lx + 2, grx, gry);
        constexpr CT third = CT(1) / CT(3);
        const CT Fx = -rho * gmx + grx * third;
        const CT Fy = -rho * gmy + gry * third;
        const CT inv_rho = rcp(rho);
        const CT ux = jx[k] * inv_rho, uy = jy[k] * inv_rho;
        if (MODE == MODE_FIELDS) {
            const long long o = (long long)gy * A.nx + gx_raw;
            const long long P = (long long)A.nx * A.ny;
            out[o] = double(rho);
            out[P + o] = double(ux + CT(0.5) * Fx * inv_rho);
            out[2 * P + o] = double(uy + CT(0.5) * Fy * inv_rho);
            out[3 * P + o] = double(ms[ry + 1][lx + 1]);
            continue;
        }
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
        const unsigned o = unsigned(gy) * unsigned(A.pitch) + unsigned(gx_raw);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const CT fs = f[k][i] - (f[k][i] - feq[i]) * inv_tau;
            const CT base = i == 0 ? b0 : (i < 5 ? b1 : b2);
            C::st(fout + (long long)i * A.plane, o, fs, base);
        }
    }
}

// One lattice: one workgroup per tile.
template <typename ST, int EOS, int MODE, int TY>
__global__ __launch_bounds__(TILE_X * TY / ROWS_PER_THREAD) void step_kernel(
    LatticeArgs A, const ST* __restrict__ fin, ST* __restrict__ fout,
    const typename Codec<ST>::CT* __restrict__ mu_w, double* __restrict__ out) {
    __shared__ TileLds<typename Codec<ST>::CT, TY> L;
    const int t = tile_of_block(blockIdx.x, gridDim.x);
    const int tiles_x = (A.nx + TILE_X - 1) / TILE_X;
    step_tile<ST, EOS, MODE, TY>(A, fin, fout, mu_w, out, (t % tiles_x) * TILE_X, (t / tiles_x) * TY, L);
}

// Many lattices in one persistent launch: each workgroup walks a contiguous range
// of the (case, tile) list; the ranges of the workgroups on one XCD are adjacent.
template <typename ST, int TY>
__global__ __launch_bounds__(TILE_X * TY / ROWS_PER_THREAD) void batch_step_kernel(
    const CaseDesc* __restrict__ cases, const int2* __restrict__ tiles, int ntiles, int parity) {
    using CT = typename Codec<ST>::CT;
    __shared__ TileLds<CT, TY> L;
    const int chunk = tile_of_block(blockIdx.x, gridDim.x);
    const int begin = int((long long)ntiles * chunk / gridDim.x);
    const int end = int((long long)ntiles * (chunk + 1) / gridDim.x);
    for (int t = begin; t < end; ++t) {
        const int2 w = tiles[t];
        const CaseDesc& C = cases[w.x];
        const int tiles_x = (C.A.nx + TILE_X - 1) / TILE_X;
        const int x0 = (w.y % tiles_x) * TILE_X, y0 = (w.y / tiles_x) * TY;
        const ST* fin = static_cast<const ST*>(C.f[parity]);
        ST* fout = static_cast<ST*>(C.f[parity ^ 1]);
        const CT* mw = static_cast<const CT*>(C.mu_w);
        switch (C.eos) {
        case EOS_VDW: step_tile<ST, EOS_VDW, MODE_STEP, TY>(C.A, fin, fout, mw, nullptr, x0, y0, L); break;
        case EOS_CS: step_tile<ST, EOS_CS, MODE_STEP, TY>(C.A, fin, fout, mw, nullptr, x0, y0, L); break;
        case EOS_PR: step_tile<ST, EOS_PR, MODE_STEP, TY>(C.A, fin, fout, mw, nullptr, x0, y0, L); break;
        default: step_tile<ST, EOS_RK, MODE_STEP, TY>(C.A, fin, fout, mw, nullptr, x0, y0, L); break;
        }
        __syncthreads();  // the next tile reuses the LDS
    }
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
template <typename ST, int COMPARE, int TY>
__global__ __launch_bounds__(MON_THREADS) void batch_monitor_kernel(const CaseDesc* __restrict__ cases,
                                                                    const int2* __restrict__ tiles, int parity,
                                                                    double* __restrict__ partials) {
    using CT = typename Codec<ST>::CT;
    const int2 w = tiles[blockIdx.x];
    const CaseDesc& C = cases[w.x];
    const LatticeArgs& A = C.A;
    Planes<ST> F;
    const ST* fin = static_cast<const ST*>(C.f[parity]);
#pragma unroll
    for (int i = 0; i < 9; ++i) F.p[i] = fin + (long long)i * A.plane;
    CT* rho_mon = static_cast<CT*>(C.rho_mon);
    const int tiles_x = (A.nx + TILE_X - 1) / TILE_X;
    const int x0 = (w.y % tiles_x) * TILE_X, y0 = (w.y / tiles_x) * TY;
    double mass = 0.0, res = 0.0;
    int flags = 0;
    for (int i = threadIdx.x; i < TILE_X * TY; i += MON_THREADS) {
        const int x = x0 + i % TILE_X, y = y0 + i / TILE_X;
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
    const int o = y * A.pitch + x;
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

template <typename ST, int EOS, int MODE>
hipError_t step_ty(int tile_y, const LatticeArgs& A, const void* fin, void* fout, const void* mu_w, double* out,
                   hipStream_t s) {
    using CT = typename Codec<ST>::CT;
    const int tiles = ((A.nx + TILE_X - 1) / TILE_X) * ((A.ny + tile_y - 1) / tile_y);
    (void)hipGetLastError();  // drop any error left by earlier runtime calls
    switch (tile_y) {
    case 8:
        hipLaunchKernelGGL((step_kernel<ST, EOS, MODE, 8>), dim3(tiles), dim3(TILE_X * 8 / ROWS_PER_THREAD), 0, s, A,
                           (const ST*)fin, (ST*)fout, (const CT*)mu_w, out);
        break;
    case 16:
        hipLaunchKernelGGL((step_kernel<ST, EOS, MODE, 16>), dim3(tiles), dim3(TILE_X * 16 / ROWS_PER_THREAD), 0, s,
                           A, (const ST*)fin, (ST*)fout, (const CT*)mu_w, out);
        break;
    case 32:
        hipLaunchKernelGGL((step_kernel<ST, EOS, MODE, 32>), dim3(tiles), dim3(TILE_X * 32 / ROWS_PER_THREAD), 0, s,
                           A, (const ST*)fin, (ST*)fout, (const CT*)mu_w, out);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename ST, int EOS>
hipError_t step_eos(int mode, int tile_y, const LatticeArgs& A, const void* fin, void* fout, const void* mu_w,
                    double* out, hipStream_t s) {
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

template <typename ST>
hipError_t batch_step_prec(int tile_y, const CaseDesc* cases, const int2* tiles, int ntiles, int parity, int grid,
                           hipStream_t s) {
    (void)hipGetLastError();
    switch (tile_y) {
    case 8:
        hipLaunchKernelGGL((batch_step_kernel<ST, 8>), dim3(grid), dim3(TILE_X * 8 / ROWS_PER_THREAD), 0, s, cases,
                           tiles, ntiles, parity);
        break;
    case 16:
        hipLaunchKernelGGL((batch_step_kernel<ST, 16>), dim3(grid), dim3(TILE_X * 16 / ROWS_PER_THREAD), 0, s,
                           cases, tiles, ntiles, parity);
        break;
    case 32:
        hipLaunchKernelGGL((batch_step_kernel<ST, 32>), dim3(grid), dim3(TILE_X * 32 / ROWS_PER_THREAD), 0, s,
                           cases, tiles, ntiles, parity);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename ST, int COMPARE>
hipError_t batch_monitor_ty(int tile_y, const CaseDesc* cases, const int2* tiles, int ntiles, int parity,
                            double* partials, hipStream_t s) {
    switch (tile_y) {
    case 8:
        hipLaunchKernelGGL((batch_monitor_kernel<ST, COMPARE, 8>), dim3(ntiles), dim3(MON_THREADS), 0, s, cases,
                           tiles, parity, partials);
        break;
    case 16:
        hipLaunchKernelGGL((batch_monitor_kernel<ST, COMPARE, 16>), dim3(ntiles), dim3(MON_THREADS), 0, s, cases,
                           tiles, parity, partials);
        break;
    case 32:
        hipLaunchKernelGGL((batch_monitor_kernel<ST, COMPARE, 32>), dim3(ntiles), dim3(MON_THREADS), 0, s, cases,
                           tiles, parity, partials);
        break;
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
int batch_occupancy(int tile_y) {
    int n = 0;
    const int threads = TILE_X * tile_y / ROWS_PER_THREAD;
    const void* k = tile_y == 8 ? (const void*)batch_step_kernel<ST, 8>
                  : (tile_y == 16 ? (const void*)batch_step_kernel<ST, 16> : (const void*)batch_step_kernel<ST, 32>);
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

hipError_t CPLBM_FN(launch_batch_step)(int tile_y, const CaseDesc* cases, const int2* tiles, int ntiles,
                                       int parity, int grid, hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    return batch_step_prec<CPLBM_ST>(tile_y, cases, tiles, ntiles, parity, grid, s);
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
