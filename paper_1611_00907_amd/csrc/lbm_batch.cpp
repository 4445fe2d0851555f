// C ABI of the batched solver: many independent lattices (uneven sizes, EOS, wall
// chemical potential) advanced together by one persistent launch per step.
#include <hip/hip_runtime.h>

#include <iterator>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "lbm_common.h"

using namespace cplbm;
using namespace cplbm::host;

struct lbm_batch {
    int n = 0;
    int prec = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* ws = nullptr;
    bool own_ws = false;
    std::vector<lbm_params> p;
    std::vector<LatticeArgs> A;
    std::vector<thermo::Fluid> fluid;
    std::vector<CaseDesc> desc;
    std::vector<std::vector<double>> mu_w_host;  // per case [2][nx]
    std::vector<int> tiles_of;                   // tiles per case
    // device tables
    CaseDesc* d_cases = nullptr;
    int2* d_tiles = nullptr;
    int* d_case_begin = nullptr;
    double* d_partials = nullptr;
    double* d_case_mon = nullptr;
    double* h_case_mon = nullptr;  // pinned [3][n]
    int total_tiles = 0;
    int ntiles = 0;  // active tiles
    // schedule
    int tile_y = TILE_Y_DEFAULT;
    int blocks_per_cu = -1;  // -1: one workgroup per (case, tile) entry; 0: the occupancy limit
    int grid = 0;
    int64_t step = 0;
    std::vector<int32_t> state;  // 0 active, 1 converged, 2 diverged
    std::vector<int64_t> steps;
    std::vector<double> residual, mass;
    std::vector<int32_t> flags;
    hipGraphExec_t graph = nullptr;
};

namespace {

constexpr int BATCH_GRAPH_STEPS = 16;  // even

struct BatchLayout {
    std::vector<size_t> f0, f1, mon, muw;
    size_t cases, tiles, begin, partials, case_mon, total;
    int total_tiles;
};

// Tiles of one case for the tile shape code (a 64-wide height or a wide code).
int tiles_for(const lbm_params& p, int code) {
    const int tx = tile_tx(code), ty = tile_ty(code);
    return ((p.nx + tx - 1) / tx) * ((p.ny + ty - 1) / ty);
}

// Tile lists are sized for the smallest tile height, so that any tuned shape fits.
BatchLayout batch_layout(const lbm_params* cases, int n) {
    BatchLayout B;
    size_t o = 0;
    B.total_tiles = 0;
    for (int i = 0; i < n; ++i) {
        const Layout L = layout_of(cases[i]);
        const size_t sb = storage_bytes(cases[i].prec), cb = compute_bytes(cases[i].prec);
        const size_t fbytes = align256(9 * size_t(L.plane) * sb);
        B.f0.push_back(o);
        o += fbytes;
        B.f1.push_back(o);
        o += fbytes;
        B.mon.push_back(o);
        o += align256(size_t(L.plane) * cb);
        B.muw.push_back(o);
        o += align256(2 * size_t(L.pitch) * cb);
        B.total_tiles += tiles_for(cases[i], 8);
    }
    B.cases = o;
    o += align256(n * sizeof(CaseDesc));
    B.tiles = o;
    o += align256(size_t(B.total_tiles) * sizeof(int2));
    B.begin = o;
    o += align256((n + 1) * sizeof(int));
    B.partials = o;
    o += align256(3 * size_t(B.total_tiles) * sizeof(double));
    B.case_mon = o;
    o += align256(3 * size_t(n) * sizeof(double));
    B.total = o;
    return B;
}

lbm_status validate_batch(const lbm_params* cases, int n) {
    if (!cases || n < 1) return LBM_EINVAL;
    for (int i = 0; i < n; ++i) {
        const lbm_status st = validate(&cases[i]);
        if (st != LBM_OK) return st;
        if (cases[i].prec != cases[0].prec) return LBM_EINVAL;
        if (cases[i].scheme != 0) return LBM_EINVAL;  // the variants run on single lattices only
    }
    return LBM_OK;
}

void drop_graph(lbm_batch* b) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

void release(lbm_batch* b) {
    if (!b) return;
    drop_graph(b);
    if (b->own_ws && b->ws) (void)hipFree(b->ws);
    if (b->h_case_mon) (void)hipHostFree(b->h_case_mon);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

// Rebuilds the (case, tile) list of the active cases and the per-case tile ranges.
lbm_status upload_tiles(lbm_batch* b) {
    std::vector<int2> tiles;
    std::vector<int> begin(b->n + 1, 0);
    for (int i = 0; i < b->n; ++i) {
        begin[i] = (int)tiles.size();
        if (b->state[i] != 0) continue;
        const int nt = tiles_for(b->p[i], batch_case_code(b->tile_y, b->p[i].nx));
        for (int t = 0; t < nt; ++t) tiles.push_back(make_int2(i, t));
    }
    begin[b->n] = (int)tiles.size();
    b->ntiles = (int)tiles.size();
    if (b->blocks_per_cu < 0) b->grid = std::max(1, b->ntiles);  // one workgroup per entry
    if (!tiles.empty())
        HIP_TRY(hipMemcpyAsync(b->d_tiles, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice,
                               b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_case_begin, begin.data(), begin.size() * sizeof(int), hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    drop_graph(b);
    return LBM_OK;
}

lbm_status upload_desc(lbm_batch* b) {
    for (int i = 0; i < b->n; ++i) b->desc[i].A.tile_y = batch_case_code(b->tile_y, b->p[i].nx);
    HIP_TRY(hipMemcpyAsync(b->d_cases, b->desc.data(), b->n * sizeof(CaseDesc), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return LBM_OK;
}

lbm_status set_schedule(lbm_batch* b, int tile_y, int blocks_per_cu) {
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
    const int occ = batch_blocks_per_cu(b->prec, tile_y);
    b->tile_y = tile_y;
    b->blocks_per_cu = blocks_per_cu;
    b->grid = std::max(1, cus * (blocks_per_cu > 0 ? std::min(blocks_per_cu, occ) : occ));  // -1: upload_tiles
    lbm_status st = upload_desc(b);
    if (st != LBM_OK) return st;
    return upload_tiles(b);
}

lbm_status one_step(lbm_batch* b) {
    HIP_TRY(launch_batch_step(b->prec, b->tile_y, b->A[0].nt_store, b->d_cases, b->d_tiles, b->ntiles, int(b->step & 1), b->grid,
                              b->stream));
    ++b->step;
    for (int i = 0; i < b->n; ++i)
        if (b->state[i] == 0) b->steps[i] = b->step;
    return LBM_OK;
}

// Captures and instantiates BATCH_GRAPH_STEPS batched steps from parity 0 (no work
// runs); a no-op when the batch already holds the graph.
lbm_status capture_graph(lbm_batch* b) {
    if (!b->graph) {
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int s = 0; s < BATCH_GRAPH_STEPS && e == hipSuccess; ++s)
            e = launch_batch_step(b->prec, b->tile_y, b->A[0].nt_store, b->d_cases, b->d_tiles, b->ntiles, s & 1, b->grid, b->stream);
        hipError_t e2 = hipStreamEndCapture(b->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_status(e != hipSuccess ? e : e2, "batch graph capture");
        }
        e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->graph = nullptr;
            return hip_status(e, "hipGraphInstantiate(batch)");
        }
        // uploaded now, so that the first replay does not carry the upload
        HIP_TRY(hipGraphUpload(b->graph, b->stream));
    }
    return LBM_OK;
}

lbm_status run_graph(lbm_batch* b) {
    const lbm_status st = capture_graph(b);
    if (st != LBM_OK) return st;
    HIP_TRY(hipGraphLaunch(b->graph, b->stream));
    b->step += BATCH_GRAPH_STEPS;
    for (int i = 0; i < b->n; ++i)
        if (b->state[i] == 0) b->steps[i] = b->step;
    return LBM_OK;
}

lbm_status advance(lbm_batch* b, int64_t n) {
    while (n > 0) {
        if (b->ntiles == 0) return LBM_OK;
        lbm_status st;
        if (n >= BATCH_GRAPH_STEPS && (b->step & 1) == 0) {
            st = run_graph(b);
            n -= BATCH_GRAPH_STEPS;
        } else {
            st = one_step(b);
            --n;
        }
        if (st != LBM_OK) return st;
    }
    return LBM_OK;
}

lbm_status monitor(lbm_batch* b, int compare) {
    HIP_TRY(launch_batch_monitor(b->prec, compare, b->tile_y, b->d_cases, b->d_tiles, b->ntiles, int(b->step & 1),
                                 b->d_partials, b->d_case_begin, b->n, b->d_case_mon, b->stream));
    if (!compare) return LBM_OK;
    HIP_TRY(hipMemcpyAsync(b->h_case_mon, b->d_case_mon, 3 * b->n * sizeof(double), hipMemcpyDeviceToHost,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(const lbm_params* cases, int32_t n) {
    if (validate_batch(cases, n) != LBM_OK) return 0;
    return batch_layout(cases, n).total;
}

lbm_status lbm_batch_init(const lbm_params* cases, int32_t n, const double* const* rho0,
                          const double* mu_w_bottom, void* dev_workspace, size_t workspace_bytes, void* hip_stream,
                          lbm_batch** out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    lbm_status st = validate_batch(cases, n);
    if (st != LBM_OK) return st;
    if (!rho0) return LBM_EINVAL;
    std::vector<thermo::Fluid> fl(n);
    for (int i = 0; i < n; ++i) {
        fl[i] = thermo::make_fluid(cases[i].eos, cases[i].a, cases[i].b, cases[i].R, cases[i].Tr, cases[i].omega);
        if (!(std::isfinite(fl[i].T) && fl[i].T > 0 && std::isfinite(fl[i].alpha))) return LBM_EINVAL;
        if (mu_w_bottom && !std::isfinite(mu_w_bottom[i])) return LBM_EINVAL;
        st = check_initial(cases[i], rho0[i], nullptr, nullptr);
        if (st != LBM_OK) return st;
    }
    const BatchLayout B = batch_layout(cases, n);
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_ENOMEM;
    b->n = n;
    b->prec = cases[0].prec;
    b->p.assign(cases, cases + n);
    b->fluid = fl;
    b->stream = (hipStream_t)hip_stream;
    b->total_tiles = B.total_tiles;
    if (hipError_t e = hipGetDevice(&b->device); e != hipSuccess) {
        note_error(e, "hipGetDevice");
        release(b);
        return LBM_EHIP;
    }
    if (!b->stream) {
        if (hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking); e != hipSuccess) {
            note_error(e, "hipStreamCreateWithFlags");
            b->stream = nullptr;
            release(b);
            return LBM_EHIP;
        }
        b->own_stream = true;
    }
    if (dev_workspace) {
        if (workspace_bytes < B.total || (reinterpret_cast<uintptr_t>(dev_workspace) & 255)) {
            release(b);
            return workspace_bytes < B.total ? LBM_ENOMEM : LBM_EINVAL;
        }
        b->ws = static_cast<char*>(dev_workspace);
    } else {
        if (hipMalloc(&b->ws, B.total) != hipSuccess) {
            release(b);
            return LBM_ENOMEM;
        }
        b->own_ws = true;
    }
    if (hipError_t e = hipHostMalloc(&b->h_case_mon, 3 * n * sizeof(double), hipHostMallocDefault); e != hipSuccess) {
        note_error(e, "hipHostMalloc");
        release(b);
        return LBM_EHIP;
    }
    if (hipError_t e = hipMemsetAsync(b->ws, 0, B.total, b->stream); e != hipSuccess) {
        note_error(e, "hipMemsetAsync(batch workspace)");
        release(b);
        return LBM_EHIP;
    }
    b->d_cases = reinterpret_cast<CaseDesc*>(b->ws + B.cases);
    b->d_tiles = reinterpret_cast<int2*>(b->ws + B.tiles);
    b->d_case_begin = reinterpret_cast<int*>(b->ws + B.begin);
    b->d_partials = reinterpret_cast<double*>(b->ws + B.partials);
    b->d_case_mon = reinterpret_cast<double*>(b->ws + B.case_mon);
    b->A.resize(n);
    b->desc.resize(n);
    b->mu_w_host.resize(n);
    b->state.assign(n, 0);
    b->steps.assign(n, 0);
    b->residual.assign(n, NAN);
    b->mass.assign(n, NAN);
    b->flags.assign(n, 0);
    // non-temporal stores when the batch's distributions together exceed the caches
    long long fbytes_all = 0;
    for (int i = 0; i < n; ++i) fbytes_all += 2 * 9 * layout_of(cases[i]).plane * (long long)storage_bytes(cases[i].prec);
    for (int i = 0; i < n; ++i) {
        const Layout L = layout_of(cases[i]);
        b->A[i] = lattice_args(cases[i], fl[i], L);
        b->A[i].nt_store = nt_store_for(fbytes_all);
        CaseDesc& d = b->desc[i];
        d.A = b->A[i];
        d.eos = cases[i].eos;
        d.f[0] = b->ws + B.f0[i];
        d.f[1] = b->ws + B.f1[i];
        d.mu_w = b->ws + B.muw[i];
        d.rho_mon = b->ws + B.mon[i];
        st = init_state(cases[i], b->A[i], rho0[i], nullptr, nullptr, d.f[0], b->stream);
        if (st != LBM_OK) {
            release(b);
            return st;
        }
        b->mu_w_host[i].assign(2 * (size_t)cases[i].nx, 0.0);
        if (mu_w_bottom && cases[i].bc_bottom == LBM_BC_CPWALL)
            std::fill(b->mu_w_host[i].begin(), b->mu_w_host[i].begin() + cases[i].nx, mu_w_bottom[i]);
        st = upload_mu_w(cases[i], L.pitch, b->mu_w_host[i].data(), const_cast<void*>(d.mu_w), b->stream);
        if (st != LBM_OK) {
            release(b);
            return st;
        }
    }
    st = set_schedule(b, TILE_Y_DEFAULT, -1);  // one workgroup per entry until tuned
    if (st != LBM_OK) {
        release(b);
        return st;
    }
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t n) {
    if (!b || n < 0) return LBM_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return LBM_EHIP;
    return advance(b, n);
}

lbm_status lbm_batch_run(lbm_batch* b, int64_t max_steps, int32_t check_every, int32_t window, double tol,
                         int64_t* steps_run) {
    if (!b || max_steps < 0 || check_every < 1 || window < 1 || window > check_every || !(tol >= 0))
        return LBM_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return LBM_EHIP;
    const int64_t start = b->step;
    while (b->step - start < max_steps && b->ntiles > 0) {
        const int64_t left = max_steps - (b->step - start);
        const int64_t chunk = std::min<int64_t>(check_every, left);
        if (chunk < window) {
            lbm_status st = advance(b, chunk);
            if (st != LBM_OK) return st;
            break;
        }
        lbm_status st = advance(b, chunk - window);
        if (st != LBM_OK) return st;
        st = monitor(b, 0);  // snapshot `window` steps before the check
        if (st != LBM_OK) return st;
        st = advance(b, window);
        if (st != LBM_OK) return st;
        st = monitor(b, 1);
        if (st != LBM_OK) return st;
        bool changed = false;
        for (int i = 0; i < b->n; ++i) {
            if (b->state[i] != 0) continue;
            b->mass[i] = b->h_case_mon[3 * i];
            b->residual[i] = b->h_case_mon[3 * i + 1] / window;
            b->flags[i] = (int32_t)b->h_case_mon[3 * i + 2];
            if (b->flags[i] || !std::isfinite(b->residual[i])) {
                b->state[i] = 2;
                changed = true;
            } else if (b->residual[i] < tol) {
                b->state[i] = 1;
                changed = true;
            }
        }
        if (changed) {
            st = upload_tiles(b);
            if (st != LBM_OK) return st;
        }
    }
    if (steps_run) *steps_run = b->step - start;
    return LBM_OK;
}

lbm_status lbm_batch_stop(lbm_batch* b, const int32_t* cases, int32_t count) {
    if (!b || count < 0 || (count > 0 && !cases)) return LBM_EINVAL;
    for (int32_t k = 0; k < count; ++k)
        if (cases[k] < 0 || cases[k] >= b->n) return LBM_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return LBM_EHIP;
    bool changed = false;
    for (int32_t k = 0; k < count; ++k) {
        if (b->state[cases[k]] != 0) continue;  // converged, diverged or stopped already
        b->state[cases[k]] = 3;
        changed = true;
    }
    // the list of active cases shrinks: rebuild it (and drop the captured graph)
    return changed ? upload_tiles(b) : LBM_OK;
}

lbm_status lbm_batch_status(lbm_batch* b, int32_t* state, int64_t* steps, double* residual, double* mass,
                            int32_t* flags) {
    if (!b) return LBM_EINVAL;
    for (int i = 0; i < b->n; ++i) {
        if (state) state[i] = b->state[i];
        if (steps) steps[i] = b->steps[i];
        if (residual) residual[i] = b->residual[i];
        if (mass) mass[i] = b->mass[i];
        if (flags) flags[i] = b->flags[i];
    }
    return LBM_OK;
}

lbm_status lbm_batch_get_fields(lbm_batch* b, int32_t i, double* rho, double* vx, double* vy, double* mu) {
    if (!b || i < 0 || i >= b->n) return LBM_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return LBM_EHIP;
    const lbm_params& p = b->p[i];
    const size_t n = (size_t)p.nx * p.ny;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, 4 * n * sizeof(double)));
    const CaseDesc& C = b->desc[i];
    hipError_t e = launch_step(p.prec, p.eos, MODE_FIELDS, C.A, C.f[b->steps[i] & 1], nullptr, C.mu_w, d, b->stream);
    double* outs[4] = {rho, vx, vy, mu};
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
        if (outs[k]) e = hipMemcpyAsync(outs[k], d + k * n, n * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(d);
    return hip_status(e, "lbm_batch_get_fields");
}

lbm_status lbm_batch_get_state(lbm_batch* b, int32_t i, double* f) {
    if (!b || !f || i < 0 || i >= b->n) return LBM_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return LBM_EHIP;
    const lbm_params& p = b->p[i];
    const size_t n = 9 * (size_t)p.nx * p.ny;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, n * sizeof(double)));
    const CaseDesc& C = b->desc[i];
    hipError_t e = launch_get_state(p.prec, C.A, C.f[b->steps[i] & 1], d, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d, n * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(d);
    return hip_status(e, "lbm_batch_get_state");
}

lbm_status lbm_batch_tune(lbm_batch* b, int32_t trial_steps, int32_t* tile_y, int32_t* blocks_per_cu,
                          double* best_ms) {
    if (!b || trial_steps < 1) return LBM_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return LBM_EHIP;
    const int parity = int(b->step & 1);
    double best = 1e300;
    int best_ty = b->tile_y, best_bpc = b->blocks_per_cu;
    struct Events {  // destroyed on every return path
        hipEvent_t a = nullptr, b = nullptr;
        ~Events() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    hipEvent_t e0 = ev.a, e1 = ev.b;
    constexpr int NCODES = int(std::size(TILE_Y_CHOICES) + std::size(BATCH_WIDE_CODES)) + 1;
    int codes[NCODES], nc = 0;
    for (int ty : TILE_Y_CHOICES) codes[nc++] = ty;
    for (int code : BATCH_WIDE_CODES) codes[nc++] = code;
    codes[nc++] = BATCH_MIXED;
    for (int ty : codes) {
        for (int bpc : {0, 1, 2, 4, -1}) {
            lbm_status st = set_schedule(b, ty, bpc);
            if (st != LBM_OK) return st;
            if (b->ntiles == 0) break;
            // the state is only read: every trial launch maps f[parity] -> f[parity ^ 1]
            for (int w = 0; w < 2; ++w)
                HIP_TRY(launch_batch_step(b->prec, ty, b->A[0].nt_store, b->d_cases, b->d_tiles, b->ntiles, parity, b->grid, b->stream));
            HIP_TRY(hipEventRecord(e0, b->stream));
            for (int s = 0; s < trial_steps; ++s)
                HIP_TRY(launch_batch_step(b->prec, ty, b->A[0].nt_store, b->d_cases, b->d_tiles, b->ntiles, parity, b->grid, b->stream));
            HIP_TRY(hipEventRecord(e1, b->stream));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                best_ty = ty;
                best_bpc = bpc;
            }
        }
    }
    lbm_status st = set_schedule(b, best_ty, best_bpc);
    if (st != LBM_OK) return st;
    if (tile_y) *tile_y = best_ty;
    // 0 stands for "as many as fit"; report how many that is (-1: one per entry)
    if (blocks_per_cu) *blocks_per_cu = best_bpc != 0 ? best_bpc : batch_blocks_per_cu(b->prec, best_ty);
    if (best_ms) *best_ms = best / trial_steps;
    return LBM_OK;
}

lbm_status lbm_batch_set_schedule(lbm_batch* b, int32_t tile_y, int32_t blocks_per_cu) {
    if (!b || blocks_per_cu < -1 || blocks_per_cu > 64) return LBM_EINVAL;
    bool ok = false;
    for (int ty : TILE_Y_CHOICES) ok = ok || ty == tile_y;
    for (int code : BATCH_WIDE_CODES) ok = ok || code == tile_y;
    ok = ok || tile_y == BATCH_MIXED;
    if (!ok) return LBM_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return LBM_EHIP;
    return set_schedule(b, tile_y, blocks_per_cu);
}

lbm_status lbm_batch_step_timed(lbm_batch* b, int64_t n, double* ms) {
    if (!b || n < 0 || !ms) return LBM_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return LBM_EHIP;
    // capture before the first event: capture and instantiation are not timed
    if (n >= BATCH_GRAPH_STEPS && b->ntiles > 0) {
        const lbm_status cs = capture_graph(b);
        if (cs != LBM_OK) return cs;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    lbm_status st = LBM_OK;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
    if (e == hipSuccess) st = advance(b, n);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_status(e, "lbm_batch_step_timed");
    *ms = t;
    return st;
}

int64_t lbm_batch_fluid_nodes(lbm_batch* b, int32_t active_only) {
    if (!b) return -1;
    int64_t s = 0;
    for (int i = 0; i < b->n; ++i) {
        if (active_only && b->state[i] != 0) continue;
        s += (int64_t)b->p[i].nx * (b->p[i].ny - (walled(b->p[i]) ? 2 : 0));
    }
    return s;
}

void lbm_batch_destroy(lbm_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    release(b);
}

}  // extern "C"
