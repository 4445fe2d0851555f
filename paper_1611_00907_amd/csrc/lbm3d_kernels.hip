// HIP kernels of the chemical-potential lattice Boltzmann step on D3Q19 for CDNA4
// (gfx950): the method of Sec. II on a periodic box.  The state is nineteen
// direction planes f[i][z][y][x] (x pitch a multiple of 64) holding the
// post-collision f*(t-1); a step pulls f_i(x, t) = f*_i(x - e_i, t-1), so reads are
// shifted and writes aligned.
//
// One launch per step (march3_kernel): a workgroup marches a 64 x 8 column of the
// box through a run of planes in z, pulling each node once; the densities and
// chemical potentials its stencils need sit in LDS rings of planes.  The field
// output keeps the two-pass form: a density pass writes rho(t), and a blocked
// kernel evaluates the chemical potential of Eq 8 and the force of Eq 12 from it.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbm3d_internal.h"
#include "lbm_eos_device.h"

namespace cplbm {
namespace d3 {
namespace {

using eosd::rcp;

// Velocity set, in the order of the C ABI: rest; +x, -x, +y, -y, +z, -z; the
// twelve edges (+x+y, -x-y, +x-y, -x+y, +x+z, -x-z, +x-z, -x+z, +y+z, -y-z, +y-z, -y+z).
constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

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

// Field output: out = [5][nz][ny][nx] doubles rho, vx, vy, vz, mu with
// v = u + F / (2 rho), from the density pass's rho and a pull of the state.
template <typename ST, typename CT, int EOS>
__global__ __launch_bounds__(NT) void fields3_kernel(Args3 A, const ST* __restrict__ fin, const CT* __restrict__ rho_g,
                                                     double* __restrict__ out) {
    __shared__ Lds3<CT> L;
    const int bx = (A.nx + TX - 1) / TX, by = (A.ny + TY - 1) / TY;
    const int b = int(blockIdx.x);
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
    // 3. own nodes: pull, force (Eq 12), moments
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= A.nx || y >= A.ny) return;
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
        const long long n = (long long)A.nx * A.ny * A.nz;
        const long long c = ((long long)z * A.ny + y) * A.nx + x;
        out[c] = double(rho);
        out[n + c] = double((jx + CT(0.5) * Fx) * inv_rho);
        out[2 * n + c] = double((jy + CT(0.5) * Fy) * inv_rho);
        out[3 * n + c] = double((jz + CT(0.5) * Fz) * inv_rho);
        out[4 * n + c] = double(L.ms[mo]);
    }
}

// ---------------------------------------------------------------------------
// One-pass step: a workgroup owns a 64 x 8 column of the box in (x, y) and marches
// a run of planes in z.  Plane z + 2 is pulled once.  Its nineteen values stay in
// registers until its own collision two planes later, and its density goes into
// an LDS ring of five planes (the column plus a two-node ring in x and y).  The
// ring nodes' densities come from their own pulls: those nodes belong to the
// neighbouring columns, which pull the same lines at about the same time, so L2
// serves most of the re-reads.  The chemical potential (Eq 8) of plane z + 1 goes
// into an LDS ring of three planes (column plus a one-node ring), and then plane z
// has all that the force of Eq 12 and the collision need.  Per node and plane: one
// pull of the distributions, one store, no density pass.
constexpr int MY = 8, MNT = TX * MY;                   // 64 x 8 column, one node per thread
constexpr int MARCH_WGS = 512;                         // two resident workgroups per compute unit
constexpr int PX = TX + 4, PP = PX * (MY + 4);         // density plane with its two-node ring
constexpr int QX = TX + 2, QP = QX * (MY + 2);         // chemical-potential plane with its one-node ring
constexpr int NRING = PP - MNT;                        // ring nodes of a density plane
static_assert(NRING <= MNT, "at most one ring node per thread");

template <typename CT>
struct LdsMarch {
    CT r[5][PP];
    CT m[3][QP];
};

// In-plane byte offsets of a node's column and row and of their periodic
// neighbours; the nineteen pulls read at sums of one x and one y part.
struct Cols {
    unsigned xc, xm, xp, yc, ym, yp;
};

template <typename ST>
__device__ __forceinline__ Cols cols_of(const Args3& A, int x, int y) {
    const unsigned R = unsigned(A.pitch) * unsigned(sizeof(ST)), S = unsigned(sizeof(ST));
    return Cols{unsigned(x) * S, unsigned(wrapi(x - 1, A.nx)) * S, unsigned(wrapi(x + 1, A.nx)) * S,
                unsigned(y) * R, unsigned(wrapi(y - 1, A.ny)) * R, unsigned(wrapi(y + 1, A.ny)) * R};
}

// Direction i's slice of plane z (uniform: one base per workgroup), and the value
// at byte offset off in it (32-bit offsets: a slice holds less than 4 GiB).
template <typename T>
__device__ __forceinline__ T* slice(T* f, const Args3& A, int i, int z) {
    return f + (i * A.plane + (long long)z * A.ny * A.pitch);
}

template <typename T>
__device__ __forceinline__ T* at_byte(T* base, unsigned off) {
    return (T*)((const char*)base + off);
}

template <typename ST>
__device__ __forceinline__ ST ld(const ST* base, unsigned off) {
    return *at_byte(base, off);
}

// f_i(x, t) of the node whose in-plane sources are k, on plane z (zm, zp: its
// periodic neighbours).
template <typename ST, typename CT>
__device__ __forceinline__ void pull19z(const Args3& A, const ST* __restrict__ fin, const Cols& k, int z, int zm,
                                        int zp, CT f[19]) {
    const unsigned c = k.yc + k.xc, xm = k.yc + k.xm, xp = k.yc + k.xp, ym = k.ym + k.xc, yp = k.yp + k.xc;
    f[0] = CT(ld<ST>(slice(fin, A, 0, z), c));
    f[1] = CT(ld<ST>(slice(fin, A, 1, z), xm));
    f[2] = CT(ld<ST>(slice(fin, A, 2, z), xp));
    f[3] = CT(ld<ST>(slice(fin, A, 3, z), ym));
    f[4] = CT(ld<ST>(slice(fin, A, 4, z), yp));
    f[5] = CT(ld<ST>(slice(fin, A, 5, zm), c));
    f[6] = CT(ld<ST>(slice(fin, A, 6, zp), c));
    f[7] = CT(ld<ST>(slice(fin, A, 7, z), k.ym + k.xm));
    f[8] = CT(ld<ST>(slice(fin, A, 8, z), k.yp + k.xp));
    f[9] = CT(ld<ST>(slice(fin, A, 9, z), k.yp + k.xm));
    f[10] = CT(ld<ST>(slice(fin, A, 10, z), k.ym + k.xp));
    f[11] = CT(ld<ST>(slice(fin, A, 11, zm), xm));
    f[12] = CT(ld<ST>(slice(fin, A, 12, zp), xp));
    f[13] = CT(ld<ST>(slice(fin, A, 13, zp), xm));
    f[14] = CT(ld<ST>(slice(fin, A, 14, zm), xp));
    f[15] = CT(ld<ST>(slice(fin, A, 15, zm), ym));
    f[16] = CT(ld<ST>(slice(fin, A, 16, zp), yp));
    f[17] = CT(ld<ST>(slice(fin, A, 17, zp), ym));
    f[18] = CT(ld<ST>(slice(fin, A, 18, zm), yp));
}

// The D3Q19 Laplacian and gradient of the stencils above, on three LDS planes
// (below, centre, above) of row stride SX.
template <typename CT, int SX>
__device__ __forceinline__ CT lap19p(const CT* m, const CT* c, const CT* p, int o) {
    const CT axis = ((c[o + 1] + c[o - 1]) + (c[o + SX] + c[o - SX])) + (p[o] + m[o]);
    const CT exy = (c[o + 1 + SX] + c[o - 1 - SX]) + (c[o + 1 - SX] + c[o - 1 + SX]);
    const CT exz = (p[o + 1] + m[o - 1]) + (m[o + 1] + p[o - 1]);
    const CT eyz = (p[o + SX] + m[o - SX]) + (m[o + SX] + p[o - SX]);
    return CT(1) / CT(3) * axis + CT(1) / CT(6) * ((exy + exz) + eyz) - CT(4) * c[o];
}

template <typename CT, int SX>
__device__ __forceinline__ void grad19p(const CT* m, const CT* c, const CT* p, int o, CT& gx, CT& gy, CT& gz) {
    constexpr CT a = CT(1) / CT(6), e = CT(1) / CT(12);
    gx = (c[o + 1] - c[o - 1]) * a +
         (((c[o + 1 + SX] - c[o - 1 - SX]) + (c[o + 1 - SX] - c[o - 1 + SX])) +
          ((p[o + 1] - m[o - 1]) + (m[o + 1] - p[o - 1]))) * e;
    gy = (c[o + SX] - c[o - SX]) * a +
         (((c[o + 1 + SX] - c[o - 1 - SX]) - (c[o + 1 - SX] - c[o - 1 + SX])) +
          ((p[o + SX] - m[o - SX]) + (m[o + SX] - p[o - SX]))) * e;
    gz = (p[o] - m[o]) * a +
         (((p[o + 1] - m[o - 1]) - (m[o + 1] - p[o - 1])) + ((p[o + SX] - m[o - SX]) - (m[o + SX] - p[o - SX]))) * e;
}

// Per-thread state of the march: the thread's own node and, for the first NRING
// threads, one node of the density ring.
struct MarchPos {
    Cols own, ring;
    int ro;        // own node in a density plane
    int qo;        // own node in a chemical-potential plane
    int rr;        // ring node in a density plane (-1: none)
    bool store;    // own node lies in the box
};

template <typename ST, typename CT>
struct March3 {
    const Args3& A;
    const ST* __restrict__ fin;
    ST* __restrict__ fout;
    LdsMarch<CT>& L;
    const MarchPos& P;
    int zs;  // first plane of the run

    __device__ __forceinline__ int wz(int z) const { return ((z % A.nz) + A.nz) % A.nz; }

    // Pull plane z (relative index t = z - zs + 2 picks the density slot): own
    // node into f, densities of the own and the ring node into the ring.  On boxes
    // beyond the caches (NTS) the own pulls go out at a raised wave priority, so that
    // a wave issuing them wins the SIMD over the other workgroup's arithmetic (256^3
    // FP32: 661 -> 645 us; the ring's pulls at that priority as well: 652 us).
    template <bool NTS>
    __device__ __forceinline__ void lead(int z, CT f[19]) {
        const int zc = wz(z), zm = wz(zc - 1), zp = wz(zc + 1);
        CT* r = L.r[(z - zs + 2) % 5];
        if constexpr (NTS) __builtin_amdgcn_s_setprio(2);
        pull19z<ST, CT>(A, fin, P.own, zc, zm, zp, f);
        if constexpr (NTS) __builtin_amdgcn_s_setprio(0);
        if (P.rr >= 0) {
            CT h[19];
            pull19z<ST, CT>(A, fin, P.ring, zc, zm, zp, h);
            r[P.rr] = sum19(h);
        }
        r[P.ro] = sum19(f);
    }

    // Chemical potential of plane z (Eq 8) on the column and its one-node ring.
    template <int EOS>
    __device__ __forceinline__ void mu(int z) {
        const int t = z - zs + 2;
        const CT *rm = L.r[(t - 1) % 5], *rc = L.r[t % 5], *rp = L.r[(t + 1) % 5];
        CT* m = L.m[(t - 1) % 3];
        const CT kappa = CT(A.kappa);
        for (int q = threadIdx.x; q < QP; q += MNT) {
            const int o = (q / QX + 1) * PX + (q % QX + 1);
            m[q] = eosd::mu_bulk<EOS, CT>(A.eos, rc[o]) - kappa * lap19p<CT, PX>(rm, rc, rp, o);
        }
    }

    // Force (Eq 12) and collision (Eqs 13, 14) of the own node on plane z.
    template <bool NTS>
    __device__ __forceinline__ void collide(int z, const CT f[19]) {
        const int t = z - zs + 2;
        const CT *rm = L.r[(t - 1) % 5], *rc = L.r[t % 5], *rp = L.r[(t + 1) % 5];
        const CT *mm = L.m[(t - 2) % 3], *mc = L.m[(t - 1) % 3], *mp = L.m[t % 3];
        const int qo = P.qo;
        const CT rho = rc[P.ro];
        CT gmx, gmy, gmz, grx, gry, grz;
        grad19p<CT, QX>(mm, mc, mp, qo, gmx, gmy, gmz);
        grad19p<CT, PX>(rm, rc, rp, P.ro, grx, gry, grz);
        constexpr CT third = CT(1) / CT(3);
        const CT Fx = -rho * gmx + grx * third, Fy = -rho * gmy + gry * third, Fz = -rho * gmz + grz * third;
        CT jx = CT(0), jy = CT(0), jz = CT(0);
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            jx += CT(CX[i]) * f[i];
            jy += CT(CY[i]) * f[i];
            jz += CT(CZ[i]) * f[i];
        }
        const CT tau = CT(A.tau), inv_tau = CT(A.inv_tau), inv_rho = rcp(rho);
        const CT ux = (jx + tau * Fx) * inv_rho, uy = (jy + tau * Fy) * inv_rho, uz = (jz + tau * Fz) * inv_rho;
        const CT usq = CT(1.5) * ((ux * ux + uy * uy) + uz * uz);
        if (!P.store) return;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const CT w = i == 0 ? W3<CT>::w0 : (i <= 6 ? W3<CT>::w1 : W3<CT>::w2);
            const CT eu = (CT(CX[i]) * ux + CT(CY[i]) * uy) + CT(CZ[i]) * uz;
            const CT feq = w * rho * (CT(1) + CT(3) * eu + CT(4.5) * eu * eu - usq);
            const ST v = ST(f[i] - (f[i] - feq) * inv_tau);
            ST* dst = at_byte(slice(fout, A, i, z), P.own.yc + P.own.xc);
            if constexpr (NTS)
                __builtin_nontemporal_store(v, dst);
            else
                *dst = v;
        }
    }

    // Plane z: pull z + 2 into fc, chemical potential of z + 1, collide fa (plane z).
    template <int EOS, bool NTS>
    __device__ __forceinline__ void plane(int z, const CT fa[19], CT fc[19]) {
        lead<NTS>(z + 2, fc);
        __syncthreads();
        mu<EOS>(z + 1);
        __syncthreads();
        collide<NTS>(z, fa);
    }
};

// Launch: blocks = ceil(nx / 64) * ceil(ny / 8) * runs, each run `zrun` planes
// (the last one shorter); 512 threads.  FP32 is held to 128 registers so that two
// workgroups share a compute unit (a few values spill): at one workgroup per unit,
// or with fewer distributions held in registers, the march is slower.
template <typename ST, typename CT, int EOS, bool NTS>
__global__ __launch_bounds__(MNT) __attribute__((amdgpu_waves_per_eu(sizeof(ST) == 4 ? 4 : 1)))
void march3_kernel(Args3 A, int zrun, const ST* __restrict__ fin, ST* __restrict__ fout) {
    __shared__ LdsMarch<CT> L;
    const int bx = (A.nx + TX - 1) / TX, by = (A.ny + MY - 1) / MY;
    const int b = int(xcd_band(blockIdx.x, gridDim.x));
    const int x0 = (b % bx) * TX, y0 = ((b / bx) % by) * MY, zs = (b / (bx * by)) * zrun;
    const int len = min(zrun, A.nz - zs);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    // Every position of the column and its ring holds the node it wraps to, so a
    // ragged column computes the right neighbours for its nodes in the box.
    auto wrap = [](int v, int n) { return ((v % n) + n) % n; };
    MarchPos P;
    P.own = cols_of<ST>(A, wrap(x0 + lx, A.nx), wrap(y0 + ly, A.ny));
    P.ro = (ly + 2) * PX + (lx + 2);
    P.qo = (ly + 1) * QX + (lx + 1);
    P.store = x0 + lx < A.nx && y0 + ly < A.ny;
    P.rr = -1;
    if (int(threadIdx.x) < NRING) {
        int k = int(threadIdx.x), hx, hy;
        if (k < 4 * PX) {                 // rows -2, -1, MY, MY + 1
            const int row = k / PX;
            hy = row < 2 ? row - 2 : MY + row - 2;
            hx = k % PX - 2;
        } else {                          // columns -2, -1, TX, TX + 1 of rows 0 .. MY - 1
            k -= 4 * PX;
            const int c = k % 4;
            hy = k / 4;
            hx = c < 2 ? c - 2 : TX + c - 2;
        }
        P.ring = cols_of<ST>(A, wrap(x0 + hx, A.nx), wrap(y0 + hy, A.ny));
        P.rr = (hy + 2) * PX + (hx + 2);
    } else {
        P.ring = P.own;
    }
    March3<ST, CT> M{A, fin, fout, L, P, zs};
    // prologue: densities of planes zs - 2 .. zs + 1, chemical potentials of zs - 1, zs
    CT f0[19], f1[19], f2[19];
    M.template lead<NTS>(zs - 2, f2);
    M.template lead<NTS>(zs - 1, f2);
    M.template lead<NTS>(zs, f0);
    M.template lead<NTS>(zs + 1, f1);
    __syncthreads();
    M.template mu<EOS>(zs - 1);
    M.template mu<EOS>(zs);
    __syncthreads();
    // the three register sets rotate with the plane
    for (int k = 0; k < len; k += 3) {
        M.template plane<EOS, NTS>(zs + k, f0, f2);
        if (k + 1 >= len) break;
        M.template plane<EOS, NTS>(zs + k + 1, f1, f0);
        if (k + 2 >= len) break;
        M.template plane<EOS, NTS>(zs + k + 2, f2, f1);
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
    // non-temporal stores when the two distribution buffers exceed the 256 MB Infinity Cache
    const bool nt = 2 * 19 * A.plane * (long long)sizeof(ST) > (256LL << 20);
    (void)hipGetLastError();
    if (mode == 0) {
        // runs of planes (at least 4 planes each): the count that finishes first when
        // MARCH_WGS workgroups run at a time, each run taking a time proportional to
        // its length
        const long long cols = (long long)((A.nx + TX - 1) / TX) * ((A.ny + MY - 1) / MY);
        long long best = 1, best_t = -1;
        for (long long r = 1; r <= std::min(4096, std::max(1, A.nz / 4)); ++r) {
            const long long t = (cols * r + MARCH_WGS - 1) / MARCH_WGS * ((A.nz + r - 1) / r);
            if (best_t < 0 || t < best_t) best = r, best_t = t;
        }
        const int zrun = int((A.nz + best - 1) / best);
        const unsigned blocks = unsigned(cols * ((A.nz + zrun - 1) / zrun));
        if (nt)
            hipLaunchKernelGGL((march3_kernel<ST, CT, EOS, true>), dim3(blocks), dim3(MNT), 0, s, A, zrun,
                               (const ST*)fin, (ST*)fout);
        else
            hipLaunchKernelGGL((march3_kernel<ST, CT, EOS, false>), dim3(blocks), dim3(MNT), 0, s, A, zrun,
                               (const ST*)fin, (ST*)fout);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((density_kernel<ST, CT>), dim3((n + 255) / 256), dim3(256), 0, s, A, (const ST*)fin, (CT*)rho);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned blocks = unsigned((A.nx + TX - 1) / TX) * unsigned((A.ny + TY - 1) / TY) *
                            unsigned((A.nz + TZ - 1) / TZ);
    hipLaunchKernelGGL((fields3_kernel<ST, CT, EOS>), dim3(blocks), dim3(NT), 0, s, A, (const ST*)fin, (const CT*)rho,
                       out);
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
