// HIP kernels of the chemical-potential lattice Boltzmann step on D3Q19 for CDNA4
// (gfx950): the method of Sec. II on a periodic box.  The state is nineteen
// direction planes f[i][z][y][x] (x pitch a multiple of 64) holding the
// post-collision f*(t-1); a step pulls f_i(x, t) = f*_i(x - e_i, t-1), so reads are
// shifted and writes aligned.
//
// Two launches per step.  The density pass pulls the nineteen values of every
// node and writes rho(t) (one value per node).  The step pass owns a 64 x 4 x 4
// block: it loads rho of the block and a two-node ring into LDS, evaluates the
// chemical potential of Eq 8 on the block and a one-node ring, then pulls the
// distributions again, forms the force of Eq 12, collides (Eqs 13, 14 with the
// equilibrium velocity u + tau F / rho) and stores.  In 3-D a ring of redundant
// pulls (the 2-D kernel's choice) would cost more than the density pass: the
// ring of a 64 x 4 x 4 block holds 3.25 times as many nodes as the block.
#include <hip/hip_runtime.h>

#include "lbm3d_internal.h"
#include "lbm_eos_device.h"

namespace cplbm {
namespace d3 {
namespace {

using eosd::rcp;

// Velocity set, in the order of the C ABI: rest; +x, -x, +y, -y, +z, -z; the
// twelve edges (+x+y, -x-y, +x-y, -x+y, +x+z, -x-z, +x-z, -x+z, +y+z, -y-z, +y-z, -y+z).
__constant__ int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__constant__ int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__constant__ int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

constexpr int TX = 64, TY = 4, TZ = 4, NT = 256;  // block of the step pass; 4 nodes (a z run) per thread

template <typename CT>
struct W3 {
    static constexpr CT w0 = CT(1) / CT(3), w1 = CT(1) / CT(18), w2 = CT(1) / CT(36);
};

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Workgroups are dealt round-robin to the 8 XCDs; renumbered so that each XCD gets a
// contiguous band of blocks, neighbouring blocks (which pull from each other's
// planes) share an L2 instead of fetching the same lines through eight of them.
__device__ __forceinline__ unsigned xcd_band(unsigned b, unsigned nblk) {
    const unsigned q = nblk >> 3, r = nblk & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Offset of node (x, y, z) in a plane.
__device__ __forceinline__ unsigned node(const Args3& A, int x, int y, int z) {
    return (unsigned(z) * unsigned(A.ny) + unsigned(y)) * unsigned(A.pitch) + unsigned(x);
}

// f_i(x, t) of node (x, y, z): the stored f*_i of node x - e_i.
template <typename ST, typename CT>
__device__ __forceinline__ void pull19(const Args3& A, const ST* __restrict__ fin, int x, int y, int z, CT f[19]) {
    const int xm = wrapi(x - 1, A.nx), xp = wrapi(x + 1, A.nx);
    const int ym = wrapi(y - 1, A.ny), yp = wrapi(y + 1, A.ny);
    const int zm = wrapi(z - 1, A.nz), zp = wrapi(z + 1, A.nz);
    const ST* p = fin;
    const long long P = A.plane;
    f[0] = CT(p[node(A, x, y, z)]);
    f[1] = CT(p[P + node(A, xm, y, z)]);
    f[2] = CT(p[2 * P + node(A, xp, y, z)]);
    f[3] = CT(p[3 * P + node(A, x, ym, z)]);
    f[4] = CT(p[4 * P + node(A, x, yp, z)]);
    f[5] = CT(p[5 * P + node(A, x, y, zm)]);
    f[6] = CT(p[6 * P + node(A, x, y, zp)]);
    f[7] = CT(p[7 * P + node(A, xm, ym, z)]);
    f[8] = CT(p[8 * P + node(A, xp, yp, z)]);
    f[9] = CT(p[9 * P + node(A, xm, yp, z)]);
    f[10] = CT(p[10 * P + node(A, xp, ym, z)]);
    f[11] = CT(p[11 * P + node(A, xm, y, zm)]);
    f[12] = CT(p[12 * P + node(A, xp, y, zp)]);
    f[13] = CT(p[13 * P + node(A, xm, y, zp)]);
    f[14] = CT(p[14 * P + node(A, xp, y, zm)]);
    f[15] = CT(p[15 * P + node(A, x, ym, zm)]);
    f[16] = CT(p[16 * P + node(A, x, yp, zp)]);
    f[17] = CT(p[17 * P + node(A, x, ym, zp)]);
    f[18] = CT(p[18 * P + node(A, x, yp, zm)]);
}

template <typename CT>
__device__ __forceinline__ CT sum19(const CT f[19]) {
    CT s = f[0];
#pragma unroll
    for (int i = 1; i < 19; ++i) s += f[i];
    return s;
}

// Density pass: rho(t) of every node.
template <typename ST, typename CT>
__global__ __launch_bounds__(256) void density_kernel(Args3 A, const ST* __restrict__ fin, CT* __restrict__ rho) {
    const unsigned n = unsigned(A.nx) * unsigned(A.ny) * unsigned(A.nz);
    const unsigned c = xcd_band(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
    if (c >= n) return;
    const unsigned x = c % unsigned(A.nx), yz = c / unsigned(A.nx);
    const unsigned y = yz % unsigned(A.ny), z = yz / unsigned(A.ny);
    CT f[19];
    pull19<ST, CT>(A, fin, int(x), int(y), int(z), f);
    rho[node(A, int(x), int(y), int(z))] = sum19(f);
}

// Weighted neighbour sums of a field held in an LDS box with row stride SX and
// plane stride SYX: the isotropic Laplacian 6 sum_i w_i (phi_i - phi_0) and the
// gradient 3 sum_i w_i e_i phi_i of the D3Q19 weights.
template <typename CT, int SX, int SYX>
__device__ __forceinline__ CT lap19(const CT* s, int o) {
    const CT axis = ((s[o + 1] + s[o - 1]) + (s[o + SX] + s[o - SX])) + (s[o + SYX] + s[o - SYX]);
    const CT exy = (s[o + 1 + SX] + s[o - 1 - SX]) + (s[o + 1 - SX] + s[o - 1 + SX]);
    const CT exz = (s[o + 1 + SYX] + s[o - 1 - SYX]) + (s[o + 1 - SYX] + s[o - 1 + SYX]);
    const CT eyz = (s[o + SX + SYX] + s[o - SX - SYX]) + (s[o + SX - SYX] + s[o - SX + SYX]);
    return CT(1) / CT(3) * axis + CT(1) / CT(6) * ((exy + exz) + eyz) - CT(4) * s[o];
}

template <typename CT, int SX, int SYX>
__device__ __forceinline__ void grad19(const CT* s, int o, CT& gx, CT& gy, CT& gz) {
    constexpr CT a = CT(1) / CT(6), e = CT(1) / CT(12);
    gx = (s[o + 1] - s[o - 1]) * a +
         (((s[o + 1 + SX] - s[o - 1 - SX]) + (s[o + 1 - SX] - s[o - 1 + SX])) +
          ((s[o + 1 + SYX] - s[o - 1 - SYX]) + (s[o + 1 - SYX] - s[o - 1 + SYX]))) * e;
    gy = (s[o + SX] - s[o - SX]) * a +
         (((s[o + 1 + SX] - s[o - 1 - SX]) - (s[o + 1 - SX] - s[o - 1 + SX])) +
          ((s[o + SX + SYX] - s[o - SX - SYX]) + (s[o + SX - SYX] - s[o - SX + SYX]))) * e;
    gz = (s[o + SYX] - s[o - SYX]) * a +
         (((s[o + 1 + SYX] - s[o - 1 - SYX]) - (s[o + 1 - SYX] - s[o - 1 + SYX])) +
          ((s[o + SX + SYX] - s[o - SX - SYX]) - (s[o + SX - SYX] - s[o - SX + SYX]))) * e;
}

template <typename CT>
struct Lds3 {
    CT rs[(TZ + 4) * (TY + 4) * (TX + 4)];  // density, block + 2-node ring
    CT ms[(TZ + 2) * (TY + 2) * (TX + 2)];  // chemical potential, block + 1-node ring
};

constexpr int RX = TX + 4, RYX = (TY + 4) * RX;   // strides of rs
constexpr int MX = TX + 2, MYX = (TY + 2) * MX;   // strides of ms

// Step pass (MODE 0) or field output (MODE 1: out = [5][nz][ny][nx] doubles rho,
// vx, vy, vz, mu with v = u + F / (2 rho)).
// NTS: the stores of f*(t) are non-temporal (boxes larger than the caches).
template <typename ST, typename CT, int EOS, int MODE, bool NTS = false>
__global__ __launch_bounds__(NT) void step3_kernel(Args3 A, const ST* __restrict__ fin, const CT* __restrict__ rho_g,
                                                   ST* __restrict__ fout, double* __restrict__ out) {
    __shared__ Lds3<CT> L;
    const int bx = (A.nx + TX - 1) / TX, by = (A.ny + TY - 1) / TY;
    const int b = int(xcd_band(blockIdx.x, gridDim.x));
    const int x0 = (b % bx) * TX, y0 = ((b / bx) % by) * TY, z0 = (b / (bx * by)) * TZ;
    // 1. density of the block and its two-node ring (periodic wrap)
    for (int q = threadIdx.x; q < (TZ + 4) * RYX; q += NT) {
        const int cz = q / RYX, r = q % RYX, cy = r / RX, cx = r % RX;
        int x = x0 - 2 + cx, y = y0 - 2 + cy, z = z0 - 2 + cz;
        x = ((x % A.nx) + A.nx) % A.nx;
        y = ((y % A.ny) + A.ny) % A.ny;
        z = ((z % A.nz) + A.nz) % A.nz;
        L.rs[q] = rho_g[node(A, x, y, z)];
    }
    __syncthreads();
    // 2. chemical potential, Eq 8, on the block and a one-node ring
    const CT kappa = CT(A.kappa);
    for (int q = threadIdx.x; q < (TZ + 2) * MYX; q += NT) {
        const int mz = q / MYX, r = q % MYX, my = r / MX, mx = r % MX;
        const int o = ((mz + 1) * (TY + 4) + (my + 1)) * RX + (mx + 1);
        L.ms[q] = eosd::mu_bulk<EOS, CT>(A.eos, L.rs[o]) - kappa * lap19<CT, RX, RYX>(L.rs, o);
    }
    __syncthreads();
    // 3. own nodes: pull, force (Eq 12), collision (Eqs 13, 14), store
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= A.nx || y >= A.ny) return;
    const CT tau = CT(A.tau), inv_tau = CT(A.inv_tau);
    constexpr CT third = CT(1) / CT(3);
    for (int k = 0; k < TZ; ++k) {
        const int z = z0 + k;
        if (z >= A.nz) break;
        CT f[19];
        pull19<ST, CT>(A, fin, x, y, z, f);
        const int ro = ((k + 2) * (TY + 4) + (ly + 2)) * RX + (lx + 2);
        const int mo = ((k + 1) * (TY + 2) + (ly + 1)) * MX + (lx + 1);
        const CT rho = L.rs[ro];
        CT gmx, gmy, gmz, grx, gry, grz;
        grad19<CT, MX, MYX>(L.ms, mo, gmx, gmy, gmz);
        grad19<CT, RX, RYX>(L.rs, ro, grx, gry, grz);
        const CT Fx = -rho * gmx + grx * third, Fy = -rho * gmy + gry * third, Fz = -rho * gmz + grz * third;
        CT jx = CT(0), jy = CT(0), jz = CT(0);
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            jx += CT(CX[i]) * f[i];
            jy += CT(CY[i]) * f[i];
            jz += CT(CZ[i]) * f[i];
        }
        const CT inv_rho = rcp(rho);
        if constexpr (MODE == 1) {
            const long long n = (long long)A.nx * A.ny * A.nz;
            const long long c = ((long long)z * A.ny + y) * A.nx + x;
            out[c] = double(rho);
            out[n + c] = double((jx + CT(0.5) * Fx) * inv_rho);
            out[2 * n + c] = double((jy + CT(0.5) * Fy) * inv_rho);
            out[3 * n + c] = double((jz + CT(0.5) * Fz) * inv_rho);
            out[4 * n + c] = double(L.ms[mo]);
            continue;
        }
        const CT ux = (jx + tau * Fx) * inv_rho, uy = (jy + tau * Fy) * inv_rho, uz = (jz + tau * Fz) * inv_rho;
        const CT usq = CT(1.5) * ((ux * ux + uy * uy) + uz * uz);
        const unsigned o = node(A, x, y, z);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const CT w = i == 0 ? W3<CT>::w0 : (i <= 6 ? W3<CT>::w1 : W3<CT>::w2);
            const CT eu = (CT(CX[i]) * ux + CT(CY[i]) * uy) + CT(CZ[i]) * uz;
            const CT feq = w * rho * (CT(1) + CT(3) * eu + CT(4.5) * eu * eu - usq);
            const ST v = ST(f[i] - (f[i] - feq) * inv_tau);
            if constexpr (NTS)
                __builtin_nontemporal_store(v, &fout[i * A.plane + o]);
            else
                fout[i * A.plane + o] = v;
        }
    }
}

// Initial storage: S_i(x) = f_i(x + e_i) with f = f_eq(rho0, 0) (init) or the given
// post-streaming f (set_state), so that the first pull returns f.
template <typename ST>
__global__ void init3_kernel(Args3 A, const double* __restrict__ rho0, const double* __restrict__ f_in,
                             ST* __restrict__ fs) {
    const unsigned n = unsigned(A.nx) * unsigned(A.ny) * unsigned(A.nz);
    const unsigned c = blockIdx.x * 256u + threadIdx.x;
    if (c >= n) return;
    const int x = int(c % unsigned(A.nx)), yz = int(c / unsigned(A.nx));
    const int y = yz % A.ny, z = yz / A.ny;
    for (int i = 0; i < 19; ++i) {
        const int xs = wrapi(x + CX[i], A.nx), ys = wrapi(y + CY[i], A.ny), zs = wrapi(z + CZ[i], A.nz);
        const long long src = ((long long)zs * A.ny + ys) * A.nx + xs;
        double v;
        if (f_in) {
            v = f_in[(long long)i * n + src];
        } else {
            const double w = i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
            v = w * rho0[src];
        }
        fs[i * A.plane + node(A, x, y, z)] = ST(v);
    }
}

// Post-streaming f(t) [19][nz][ny][nx] from the storage.
template <typename ST>
__global__ void state3_kernel(Args3 A, const ST* __restrict__ fs, double* __restrict__ f_out) {
    const unsigned n = unsigned(A.nx) * unsigned(A.ny) * unsigned(A.nz);
    const unsigned c = blockIdx.x * 256u + threadIdx.x;
    if (c >= n) return;
    const int x = int(c % unsigned(A.nx)), yz = int(c / unsigned(A.nx));
    const int y = yz % A.ny, z = yz / A.ny;
    double f[19];
    pull19<ST, double>(A, fs, x, y, z, f);
    for (int i = 0; i < 19; ++i) f_out[(long long)i * n + c] = f[i];
}

template <typename ST, int EOS>
hipError_t step_eos(int mode, const Args3& A, const void* fin, void* rho, void* fout, double* out, hipStream_t s) {
    using CT = ST;  // FP64 storage computes in FP64, FP32 in FP32
    const unsigned n = unsigned(A.nx) * unsigned(A.ny) * unsigned(A.nz);
    (void)hipGetLastError();
    hipLaunchKernelGGL((density_kernel<ST, CT>), dim3((n + 255) / 256), dim3(256), 0, s, A, (const ST*)fin, (CT*)rho);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned blocks = unsigned((A.nx + TX - 1) / TX) * unsigned((A.ny + TY - 1) / TY) *
                            unsigned((A.nz + TZ - 1) / TZ);
    // non-temporal stores when the two distribution buffers exceed the 256 MB Infinity Cache
    const bool nt = 2 * 19 * A.plane * (long long)sizeof(ST) > (256LL << 20);
    if (mode == 0 && nt)
        hipLaunchKernelGGL((step3_kernel<ST, CT, EOS, 0, true>), dim3(blocks), dim3(NT), 0, s, A, (const ST*)fin,
                           (const CT*)rho, (ST*)fout, out);
    else if (mode == 0)
        hipLaunchKernelGGL((step3_kernel<ST, CT, EOS, 0>), dim3(blocks), dim3(NT), 0, s, A, (const ST*)fin,
                           (const CT*)rho, (ST*)fout, out);
    else
        hipLaunchKernelGGL((step3_kernel<ST, CT, EOS, 1>), dim3(blocks), dim3(NT), 0, s, A, (const ST*)fin,
                           (const CT*)rho, (ST*)fout, out);
    return hipGetLastError();
}

template <typename ST>
hipError_t step_prec(int eos, int mode, const Args3& A, const void* fin, void* rho, void* fout, double* out,
                     hipStream_t s) {
    switch (eos) {
    case EOS_VDW: return step_eos<ST, EOS_VDW>(mode, A, fin, rho, fout, out, s);
    case EOS_CS: return step_eos<ST, EOS_CS>(mode, A, fin, rho, fout, out, s);
    case EOS_PR: return step_eos<ST, EOS_PR>(mode, A, fin, rho, fout, out, s);
    case EOS_RKS:
    case EOS_RK: return step_eos<ST, EOS_RK>(mode, A, fin, rho, fout, out, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_step3(int prec, int eos, int mode, const Args3& A, const void* fin, void* rho, void* fout,
                        double* out, hipStream_t s) {
    if (prec == PREC_F64) return step_prec<double>(eos, mode, A, fin, rho, fout, out, s);
    if (prec == PREC_F32) return step_prec<float>(eos, mode, A, fin, rho, fout, out, s);
    return hipErrorInvalidValue;
}

hipError_t launch_init3(int prec, const Args3& A, const double* rho0, const double* f_in, void* fs, hipStream_t s) {
    const unsigned n = unsigned(A.nx) * unsigned(A.ny) * unsigned(A.nz);
    (void)hipGetLastError();
    if (prec == PREC_F64)
        hipLaunchKernelGGL(init3_kernel<double>, dim3((n + 255) / 256), dim3(256), 0, s, A, rho0, f_in, (double*)fs);
    else if (prec == PREC_F32)
        hipLaunchKernelGGL(init3_kernel<float>, dim3((n + 255) / 256), dim3(256), 0, s, A, rho0, f_in, (float*)fs);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_state3(int prec, const Args3& A, const void* fs, double* f_out, hipStream_t s) {
    const unsigned n = unsigned(A.nx) * unsigned(A.ny) * unsigned(A.nz);
    (void)hipGetLastError();
    if (prec == PREC_F64)
        hipLaunchKernelGGL(state3_kernel<double>, dim3((n + 255) / 256), dim3(256), 0, s, A, (const double*)fs, f_out);
    else if (prec == PREC_F32)
        hipLaunchKernelGGL(state3_kernel<float>, dim3((n + 255) / 256), dim3(256), 0, s, A, (const float*)fs, f_out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace d3
}  // namespace cplbm
