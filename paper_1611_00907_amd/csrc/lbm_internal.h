// Internal interface between the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace cplbm {

enum Eos : int { EOS_VDW = 0, EOS_CS = 1, EOS_PR = 2, EOS_RKS = 3, EOS_RK = 4 };
enum Prec : int { PREC_F64 = 0, PREC_F32 = 1, PREC_F16DEV = 2, PREC_BF16DEV = 3 };
enum Bc : int { BC_PERIODIC = 0, BC_CPWALL = 1, BC_NEUTRAL = 2 };

// Tile of the fused step: TILE_X x tile_y nodes per workgroup of TILE_X * tile_y /
// ROWS_PER_THREAD threads; each thread owns ROWS_PER_THREAD nodes of one column.
// tile_y is one of TILE_Y_CHOICES (picked per lattice by the tuner; default 16).
constexpr int TILE_X = 64;
constexpr int ROWS_PER_THREAD = 4;
constexpr int TILE_Y_DEFAULT = 16;
constexpr int TILE_Y_CHOICES[3] = {8, 16, 32};
// Wider tiles of the single-lattice step, as shape codes 100 * width + height:
// 128 x 16 and 256 x 8 (4 rows per thread), 128 x 32 and 256 x 16 (8 rows per
// thread), each run by 512 threads.  A wider tile pulls a smaller fraction of
// redundant ring nodes.
constexpr int WIDE_TILE_CODES[4] = {12816, 12832, 25608, 25616};
// Batches take the 64-wide heights of TILE_Y_CHOICES and these wide shape codes
// (128 x 16 and 256 x 8, 4 rows per thread, 512 threads).
constexpr int BATCH_WIDE_CODES[2] = {12816, 25608};
// Batch schedule with a tile shape per size class, in one launch: cases narrower than
// BATCH_MIXED_WIDE columns take 64 x 32 tiles, the others 256 x 8 (both 512 threads).
constexpr int BATCH_MIXED = 1;
constexpr int BATCH_MIXED_WIDE = 256;
constexpr int batch_case_code(int schedule_code, int nx) {
    return schedule_code != BATCH_MIXED ? schedule_code : (nx < BATCH_MIXED_WIDE ? 32 : 25608);
}
// Columns and rows of a tile with shape code `code` (a 64-wide height or 100 * width + height).
constexpr int tile_tx(int code) { return code >= 10000 ? code / 100 : TILE_X; }
constexpr int tile_ty(int code) { return code >= 10000 ? code % 100 : code; }
// 64-wide tiles whose ring pulls go out with the own pulls (one memory round trip
// instead of two, more registers), as shape codes 1000000 + height.
constexpr int HOIST_BASE = 1000000;
constexpr int HOIST_CODES[2] = {HOIST_BASE + 16, HOIST_BASE + 32};

// Column-marching shape: a workgroup of MARCH_NT lanes owns a strip of at most
// MARCH_OWN columns (two halo lanes per side) and marches up a segment of rows.  A
// lattice's shape code (LatticeArgs::tile_y) is the tile height for tiles, or -k
// for marching with k resident workgroups per CU (1 <= k <= MARCH_K_MAX): the rows
// are split into as many segments as fill that many workgroups per CU.  Marching
// needs the nine planes of one buffer below 2 GiB (32-bit buffer offsets).
constexpr int MARCH_NT = 256;
constexpr int MARCH_OWN = MARCH_NT - 4;
constexpr int MARCH_K_MAX = 8;
constexpr long long MARCH_MAX_BYTES = (1LL << 31) - 1;

// Constants of the bulk chemical potential, precomputed on the host in FP64.
struct EosConst {
    double RT;       // R * T
    double a;        // a (VdW, CS) or a * alpha(T) (RK, RKS, PR)
    double b;
    double c1;       // PR: a alpha / (2 sqrt 2 b); RK/RKS: a alpha / b; CS: b / 4
    double rho_max;  // EOS pole: 1/b (4/b for CS)
};

// Everything a kernel needs about one lattice; passed by value.
struct LatticeArgs {
    int nx, ny;
    int pitch;            // elements per row of the density-shaped arrays (>= nx)
    int bottom, top;      // Bc of rows 0 and ny-1
    int tile_y;           // shape code: tile height (64-wide tiles), a wide-tile code, or -k (marching)
    long long plane;      // distributions: elements from direction i to direction i + 1 of one node
                          // (pitch in the row-interleaved layout, ny * pitch in the plane layout)
    double tau, inv_tau, kappa;
    double rho_ref;       // deviation base of the half/bf16 storage
    double sp_lo, sp_hi;  // spinodal band: the 16-bit storage types evaluate psi' in FP64
                          // for sp_lo < rho < sp_hi (empty band: both 0)
    EosConst eos;
    int scheme;           // force (bits 0-3) | collision (bits 4-7); 0 = Eq 12 with BGK
    int fpitch;           // distributions: elements from row y to row y + 1 of one direction
                          // (9 * pitch row-interleaved, pitch in the plane layout)
    int nt_store;         // 1: the step stores f*(t) non-temporally (working sets beyond the caches)
    int pad_;
    double tau_minus;     // TRT: relaxation time of the odd part
    double s_e, s_eps, s_q;  // MRT rates of e, epsilon and the heat-flux moments
};

enum Scheme : int { FORCE_CP = 0, FORCE_PTENSOR = 1, COLLIDE_BGK = 0, COLLIDE_TRT = 16, COLLIDE_MRT = 32 };
// The tile shape that runs the schemes other than 0.
constexpr int SCHEME_TILE_Y = 16;

enum StepMode : int { MODE_STEP = 0, MODE_FIELDS = 1 };

// One lattice of a batch, as the batched kernels see it.
struct CaseDesc {
    LatticeArgs A;
    int eos;
    int pad_;
    void* f[2];         // the two distribution buffers (storage type of the batch)
    const void* mu_w;   // [2][pitch] wall chemical potentials, compute type
    void* rho_mon;      // density snapshot, compute type
};

// Fused step (or field output) over the whole lattice.
// fin: storage of the post-collision distributions f*(t-1) (pulled to give f(t));
// fout: f*(t) (MODE_STEP).  mu_w: [2][pitch] wall chemical potentials in the compute
// type.  out: MODE_FIELDS only, [4][ny][nx] doubles rho, vx, vy, mu.
hipError_t launch_step(int prec, int eos, int mode, const LatticeArgs& A, const void* fin,
                       void* fout, const void* mu_w, double* out, hipStream_t s);

// Monitors of the state in fin: snapshot (compare == 0) writes rho to rho_mon;
// compare == 1 also writes per-block partials (mass, max |drho|, flags) and reduces
// them into mon[0..2] (mass, residual, flags as double).
hipError_t launch_monitor(int prec, int eos, int compare, const LatticeArgs& A, const void* fin,
                          void* rho_mon, double* partials, double* mon, hipStream_t s);

// All cases of a batch advance one step: tiles is the (case, tile) list of the active
// cases, grid the number of persistent workgroups, parity selects f[parity] -> f[parity^1],
// nt: non-temporal stores of f*(t) (a batch larger than the caches).
hipError_t launch_batch_step(int prec, int tile_y, int nt, const CaseDesc* cases, const int2* tiles, int ntiles,
                             int parity, int grid, hipStream_t s);
// Batched monitors over the same tile list: partials [3][ntiles]; compare == 1 reduces each
// case's tile range [case_tile_begin[c], case_tile_begin[c+1]) into case_mon[3 c .. 3 c + 2].
hipError_t launch_batch_monitor(int prec, int compare, int tile_y, const CaseDesc* cases, const int2* tiles,
                                int ntiles, int parity, double* partials, const int* case_tile_begin, int ncases,
                                double* case_mon, hipStream_t s);
// Resident workgroups per CU of the batched step kernel (for the persistent grid).
int batch_blocks_per_cu(int prec, int tile_y);

// f_i(t) from f_eq(rho0, u0) (init, u may be null) or from given f (set_state): writes the
// storage form f*(t-1) such that streaming reproduces f(t).  rho0/ux0/uy0/f_in are device
// doubles [ny][nx] / [9][ny][nx].
hipError_t launch_init(int prec, const LatticeArgs& A, const double* rho0, const double* ux0,
                       const double* uy0, const double* f_in, void* fstore, hipStream_t s);

// f_i(t) [9][ny][nx] doubles from the storage (zero on solid rows).
hipError_t launch_get_state(int prec, const LatticeArgs& A, const void* fstore, double* f_out,
                            hipStream_t s);

// Plain device copy of bytes (a multiple of 16) from src to dst.
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

size_t storage_bytes(int prec);
size_t compute_bytes(int prec);

// Whether the column-marching shapes may run on this lattice and storage type.
inline bool march_allowed(const LatticeArgs& A, int prec) {
    return 9LL * A.ny * A.pitch * (long long)storage_bytes(prec) <= MARCH_MAX_BYTES;
}

}  // namespace cplbm
