// C ABI of the chemical-potential lattice Boltzmann library (declared in lbm.h).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <iterator>
#include <mutex>
#include <vector>

#include "lbm_common.h"

using namespace cplbm;

struct lbm_ctx {
    lbm_params p;
    LatticeArgs A;
    thermo::Fluid fluid;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    hipGraphExec_t graph = nullptr;  // GRAPH_STEPS fused steps from parity 0, captured on demand
    char* ws = nullptr;
    bool own_ws = false;
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    void* rho_mon = nullptr;
    void* mu_w = nullptr;
    double* partials = nullptr;
    double* mon_dev = nullptr;
    double* mon_host = nullptr;  // pinned
    int64_t step = 0;
    int64_t snap_step = -1;
    double mass = NAN, residual = NAN;
    int64_t mon_step = -1;
    int32_t flags = 0;
    std::vector<double> mu_w_host;  // [2][nx]
};

namespace cplbm {
namespace host {

thread_local char g_last_error[256] = "";

void note_error(hipError_t e, const char* where) {
    std::snprintf(g_last_error, sizeof g_last_error, "%s: %s (%d)", where, hipGetErrorName(e), (int)e);
}

lbm_status hip_status(hipError_t e, const char* where) {
    if (e == hipSuccess) return LBM_OK;
    note_error(e, where);
    return LBM_EHIP;
}

lbm_status validate(const lbm_params* p) {
    if (!p) return LBM_EINVAL;
    if (p->nx < 1 || p->ny < 1) return LBM_EINVAL;
    if (p->bc_bottom < 0 || p->bc_bottom > 2 || p->bc_top < 0 || p->bc_top > 2) return LBM_EINVAL;
    if ((p->bc_bottom == LBM_BC_PERIODIC) != (p->bc_top == LBM_BC_PERIODIC)) return LBM_EINVAL;
    if (walled(*p) && p->ny < 3) return LBM_EINVAL;
    if (p->eos < 0 || p->eos > 4 || p->prec < 0 || p->prec > 3) return LBM_EINVAL;
    const double vals[] = {p->a, p->b, p->R, p->omega, p->Tr, p->tau, p->kappa, p->rho_ref};
    for (double v : vals)
        if (!std::isfinite(v)) return LBM_EINVAL;
    if (p->a < 0 || p->b <= 0 || p->R <= 0 || p->Tr <= 0 || p->tau <= 0.5 || p->kappa < 0) return LBM_EINVAL;
    if (p->monitor_every < 0) return LBM_EINVAL;
    const int force = p->scheme & 15, coll = p->scheme & ~15;
    if (force > LBM_FORCE_PTENSOR || (coll != LBM_COLLIDE_BGK && coll != LBM_COLLIDE_TRT && coll != LBM_COLLIDE_MRT))
        return LBM_EINVAL;
    if (p->scheme != 0 && p->prec != LBM_F64 && p->prec != LBM_F32) return LBM_EINVAL;
    if (force == LBM_FORCE_PTENSOR && walled(*p)) return LBM_EINVAL;
    const double rates[] = {p->trt_lambda, p->mrt_s_e, p->mrt_s_eps, p->mrt_s_q};
    for (double v : rates)
        if (!std::isfinite(v) || v < 0) return LBM_EINVAL;
    if (p->mrt_s_e >= 2 || p->mrt_s_eps >= 2 || p->mrt_s_q >= 2) return LBM_EINVAL;  // rates in (0, 2)
    const long long pitch = ((long long)p->nx + PITCH_ALIGN - 1) / PITCH_ALIGN * PITCH_ALIGN;
    if (pitch * (long long)p->ny > INT_MAX) return LBM_EINVAL;  // in-plane offsets are 32-bit
    // kernels address each direction plane with a 32-bit byte offset
    if (pitch * (long long)p->ny * (long long)storage_bytes(p->prec) >= (1LL << 32)) return LBM_EINVAL;
    return LBM_OK;
}

Layout layout_of(const lbm_params& p) {
    Layout L{};
    L.pitch = (p.nx + PITCH_ALIGN - 1) / PITCH_ALIGN * PITCH_ALIGN;
    L.plane = (long long)L.pitch * p.ny;
    const size_t sb = storage_bytes(p.prec), cb = compute_bytes(p.prec);
    const size_t fbytes = align256(9 * size_t(L.plane) * sb);
    size_t o = 0;
    L.f0 = o;
    o += fbytes;
    L.f1 = o;
    o += fbytes;
    L.rho_mon = o;
    o += align256(size_t(L.plane) * cb);
    L.mu_w = o;
    o += align256(2 * size_t(L.pitch) * cb);
    L.partials = o;
    o += align256(3 * 1024 * sizeof(double));
    L.mon = o;
    o += align256(4 * sizeof(double));
    L.total = o;
    return L;
}

LatticeArgs lattice_args(const lbm_params& p, const thermo::Fluid& fl, const Layout& L) {
    LatticeArgs A{};
    A.nx = p.nx;
    A.ny = p.ny;
    A.pitch = L.pitch;
    A.bottom = p.bc_bottom;
    A.top = p.bc_top;
    // 128 x 16 tiles where a lattice is at least that wide: the fastest tile at the
    // sizes measured, before any tuning
    A.tile_y = p.nx >= 128 ? 12816 : TILE_Y_DEFAULT;
    A.scheme = p.scheme;
    if (p.scheme != 0) A.tile_y = SCHEME_TILE_Y;  // the one shape the variants run
    {
        const double lambda = p.trt_lambda > 0 ? p.trt_lambda : 0.25;
        A.tau_minus = 0.5 + lambda / (p.tau - 0.5);
        const double sn = 1.0 / p.tau;
        A.s_e = p.mrt_s_e > 0 ? p.mrt_s_e : 1.0;
        A.s_eps = p.mrt_s_eps > 0 ? p.mrt_s_eps : 1.0;
        A.s_q = p.mrt_s_q > 0 ? p.mrt_s_q : 8.0 * (2.0 - sn) / (8.0 - sn);
    }
    // Distributions row-interleaved, f[y][i][x], where every offset of one buffer
    // fits the kernels' 32-bit byte offsets: the nine rows a node's pull reads and the
    // nine it writes then lie in one contiguous stretch, so a tile's reads and writes
    // are two streams through memory instead of eighteen (measured on the bare pull
    // pattern at 4096^2 FP32: 13 % faster than nine planes).  Larger lattices keep
    // the plane layout f[i][y][x].
    if (9LL * L.plane * (long long)storage_bytes(p.prec) < (1LL << 32)) {
        A.plane = L.pitch;
        A.fpitch = 9 * L.pitch;
    } else {
        A.plane = L.plane;
        A.fpitch = L.pitch;
    }
    A.nt_store = nt_store_for(2 * 9 * L.plane * (long long)storage_bytes(p.prec));
    A.tau = p.tau;
    A.inv_tau = 1.0 / p.tau;
    A.kappa = p.kappa;
    A.rho_ref = (p.prec == LBM_F16DEV || p.prec == LBM_BF16DEV) ? p.rho_ref : 0.0;
    A.sp_lo = A.sp_hi = 0.0;
    if (p.prec == LBM_F16DEV || p.prec == LBM_BF16DEV) {
        double lo, hi;
        if (thermo::spinodal(fl, &lo, &hi)) {
            A.sp_lo = lo;
            A.sp_hi = hi;
        }
    }
    EosConst& E = A.eos;
    E.RT = fl.R * fl.T;
    E.b = fl.b;
    E.rho_max = thermo::rho_pole(fl.eos, fl.b);
    switch (fl.eos) {
    case LBM_EOS_VDW:
        E.a = fl.a;
        E.c1 = 0.0;
        break;
    case LBM_EOS_CS:
        E.a = fl.a;
        E.c1 = fl.b / 4.0;
        break;
    case LBM_EOS_PR:
        E.a = fl.a * fl.alpha;
        E.c1 = fl.a * fl.alpha / (2.0 * std::sqrt(2.0) * fl.b);
        break;
    default:
        E.a = fl.a * fl.alpha;
        E.c1 = fl.a * fl.alpha / fl.b;
    }
    return A;
}

lbm_status check_initial(const lbm_params& p, const double* rho0, const double* ux0, const double* uy0) {
    if (!rho0) return LBM_EINVAL;
    const double pole = thermo::rho_pole(p.eos, p.b);
    for (int y = 0; y < p.ny; ++y) {
        if (is_solid_row(p, y)) continue;
        for (int x = 0; x < p.nx; ++x) {
            const size_t i = (size_t)y * p.nx + x;
            const double r = rho0[i];
            if (!(std::isfinite(r) && r > 0.0 && r < pole)) return LBM_EDOMAIN;
            if ((ux0 && !std::isfinite(ux0[i])) || (uy0 && !std::isfinite(uy0[i]))) return LBM_EDOMAIN;
        }
    }
    return LBM_OK;
}

lbm_status init_state(const lbm_params& p, const LatticeArgs& A, const double* rho0, const double* ux0,
                      const double* uy0, void* fstore, hipStream_t s) {
    const size_t n = (size_t)p.nx * p.ny;
    double* staging = nullptr;
    const size_t sbytes = n * sizeof(double);
    const char* where = "hipMalloc(staging)";
    hipError_t e = hipMalloc(&staging, 3 * sbytes);
    if (e == hipSuccess) e = hipMemcpyAsync(staging, rho0, sbytes, hipMemcpyHostToDevice, s), where = "copy rho0";
    if (e == hipSuccess && ux0) e = hipMemcpyAsync(staging + n, ux0, sbytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && uy0) e = hipMemcpyAsync(staging + 2 * n, uy0, sbytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_init(p.prec, A, staging, ux0 ? staging + n : nullptr, uy0 ? staging + 2 * n : nullptr, nullptr,
                        fstore, s),
        where = "init kernel";
    if (e == hipSuccess) e = hipStreamSynchronize(s), where = "hipStreamSynchronize(init)";
    if (staging) (void)hipFree(staging);
    return hip_status(e, where);
}

lbm_status upload_mu_w(const lbm_params& p, int pitch, const double* mu_w_host, void* mu_w_dev, hipStream_t s) {
    const int nx = p.nx;
    if (p.prec == LBM_F64) {
        std::vector<double> buf(2 * (size_t)pitch, 0.0);
        for (int w = 0; w < 2; ++w)
            for (int x = 0; x < nx; ++x) buf[(size_t)w * pitch + x] = mu_w_host[(size_t)w * nx + x];
        HIP_TRY(hipMemcpyAsync(mu_w_dev, buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        std::vector<float> buf(2 * (size_t)pitch, 0.0f);
        for (int w = 0; w < 2; ++w)
            for (int x = 0; x < nx; ++x) buf[(size_t)w * pitch + x] = (float)mu_w_host[(size_t)w * nx + x];
        HIP_TRY(hipMemcpyAsync(mu_w_dev, buf.data(), buf.size() * sizeof(float), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return LBM_OK;
}

}  // namespace host
}  // namespace cplbm

using namespace cplbm::host;

namespace {

// Fused steps per captured HIP graph (even, so a replay returns to buffer 0).
constexpr int GRAPH_STEPS = 32;

// Monitor pass over the current state; compare == 1 also reads the results back.
lbm_status run_monitor(lbm_ctx* c, int compare) {
    HIP_TRY(launch_monitor(c->p.prec, c->p.eos, compare, c->A, c->f[c->cur], c->rho_mon, c->partials,
                           c->mon_dev, c->stream));
    c->snap_step = c->step;
    if (!compare) return LBM_OK;
    HIP_TRY(hipMemcpyAsync(c->mon_host, c->mon_dev, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->mass = c->mon_host[0];
    c->residual = c->mon_host[1];
    c->flags = (int32_t)c->mon_host[2];
    c->mon_step = c->step;
    return c->flags ? LBM_EDIVERGED : LBM_OK;
}

// Captures and instantiates GRAPH_STEPS fused steps starting from parity 0 (no
// work runs); a no-op when the context already holds the graph.
lbm_status capture_graph(lbm_ctx* c) {
    if (!c->graph) {
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int s = 0; s < GRAPH_STEPS && e == hipSuccess; ++s)
            e = launch_step(c->p.prec, c->p.eos, MODE_STEP, c->A, c->f[s & 1], c->f[(s & 1) ^ 1], c->mu_w, nullptr,
                            c->stream);
        hipError_t e2 = hipStreamEndCapture(c->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_status(e != hipSuccess ? e : e2, "graph capture");
        }
        e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->graph = nullptr;
            return hip_status(e, "hipGraphInstantiate");
        }
        // the graph's first launch would otherwise carry its upload to the device
        // (about 1 ms), inside whatever interval is being timed
        HIP_TRY(hipGraphUpload(c->graph, c->stream));
    }
    return LBM_OK;
}

// Replays (capturing on first use) GRAPH_STEPS fused steps starting from parity 0;
// GRAPH_STEPS is even, so the state ends in buffer 0 again.
lbm_status run_graph(lbm_ctx* c) {
    const lbm_status st = capture_graph(c);
    if (st != LBM_OK) return st;
    HIP_TRY(hipGraphLaunch(c->graph, c->stream));
    c->step += GRAPH_STEPS;
    return LBM_OK;
}

lbm_status one_step(lbm_ctx* c) {
    HIP_TRY(launch_step(c->p.prec, c->p.eos, MODE_STEP, c->A, c->f[c->cur], c->f[c->cur ^ 1], c->mu_w, nullptr,
                        c->stream));
    c->cur ^= 1;
    ++c->step;
    return LBM_OK;
}

lbm_status upload_mu_w(lbm_ctx* c) {
    return cplbm::host::upload_mu_w(c->p, c->A.pitch, c->mu_w_host.data(), c->mu_w, c->stream);
}

void drop_graph(lbm_ctx* c) {
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
}

void release(lbm_ctx* c) {
    if (!c) return;
    drop_graph(c);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->mon_host) (void)hipHostFree(c->mon_host);
    delete c;
}

}  // namespace

// Staging of lbm_get_fields_noalloc: the four FP64 fields of at most
// LBM_NOALLOC_MAX_NODES nodes.  Every device the library runs on holds its own copy
// for the life of the process.  Host code never passes this name to a kernel or a
// copy (on the host it is only a stand-in symbol): it uses the device address that
// hipGetSymbolAddress returns for the current device, kept per device below.
static __device__ __align__(256) double scratch[4 * (size_t)LBM_NOALLOC_MAX_NODES];

namespace {

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mutex;
double* g_scratch[SCRATCH_DEVICES] = {};

// Device address of device dev's copy of `scratch`; dev must be the current device.
// Looked up on the first call per device and kept.
lbm_status scratch_on_device(int dev, double** out) {
    if (dev < 0 || dev >= SCRATCH_DEVICES) return LBM_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_status(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch[dev];
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_params* p) {
    if (validate(p) != LBM_OK) return 0;
    return layout_of(*p).total;
}

lbm_status lbm_init(const lbm_params* p, const double* rho0, const double* ux0, const double* uy0,
                    void* dev_workspace, size_t workspace_bytes, void* hip_stream, lbm_ctx** out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    lbm_status st = validate(p);
    if (st != LBM_OK) return st;
    if (!rho0) return LBM_EINVAL;
    const thermo::Fluid fl = thermo::make_fluid(p->eos, p->a, p->b, p->R, p->Tr, p->omega);
    if (!(std::isfinite(fl.T) && fl.T > 0 && std::isfinite(fl.alpha))) return LBM_EINVAL;
    st = check_initial(*p, rho0, ux0, uy0);
    if (st != LBM_OK) return st;
    const Layout L = layout_of(*p);
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_ENOMEM;
    c->p = *p;
    c->fluid = fl;
    c->stream = (hipStream_t)hip_stream;
    if (hipError_t e0 = hipGetDevice(&c->device); e0 != hipSuccess) {
        note_error(e0, "hipGetDevice");
        release(c);
        return LBM_EHIP;
    }
    if (!c->stream) {  // a stream of our own (default priority), so that steps can be graph-captured
        if (hipError_t e0 = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking); e0 != hipSuccess) {
            note_error(e0, "hipStreamCreateWithFlags");
            c->stream = nullptr;
            release(c);
            return LBM_EHIP;
        }
        c->own_stream = true;
    }
    if (dev_workspace) {
        if (workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(dev_workspace) & 255)) {
            release(c);
            return workspace_bytes < L.total ? LBM_ENOMEM : LBM_EINVAL;
        }
        c->ws = static_cast<char*>(dev_workspace);
    } else {
        if (hipMalloc(&c->ws, L.total) != hipSuccess) {
            release(c);
            return LBM_ENOMEM;
        }
        c->own_ws = true;
    }
    if (hipError_t e0 = hipHostMalloc(&c->mon_host, 4 * sizeof(double), hipHostMallocDefault); e0 != hipSuccess) {
        note_error(e0, "hipHostMalloc");
        release(c);
        return LBM_EHIP;
    }
    c->f[0] = c->ws + L.f0;
    c->f[1] = c->ws + L.f1;
    c->rho_mon = c->ws + L.rho_mon;
    c->mu_w = c->ws + L.mu_w;
    c->partials = reinterpret_cast<double*>(c->ws + L.partials);
    c->mon_dev = reinterpret_cast<double*>(c->ws + L.mon);
    c->A = lattice_args(*p, fl, L);
    c->mu_w_host.assign(2 * (size_t)p->nx, 0.0);

    // f(0) = f_eq(rho0, u0), stored in the pulled form.
    if (hipError_t e = hipMemsetAsync(c->ws, 0, L.total, c->stream); e != hipSuccess) {
        note_error(e, "hipMemsetAsync(workspace)");
        release(c);
        return LBM_EHIP;
    }
    st = init_state(*p, c->A, rho0, ux0, uy0, c->f[0], c->stream);
    if (st != LBM_OK) {
        release(c);
        return st;
    }
    st = upload_mu_w(c);
    if (st != LBM_OK) {
        release(c);
        return st;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
    if (!c || n < 0) return LBM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    const int m = c->p.monitor_every;
    int64_t left = n;
    while (left > 0) {
        if (m > 0 && (c->step + 1) % m == 0 && c->snap_step != c->step) {
            lbm_status st = run_monitor(c, 0);  // snapshot one step before a monitor point
            if (st != LBM_OK) return st;
        }
        // steps that can run before the next monitor event (snapshot or compare)
        int64_t run = left;
        if (m > 0) {
            int64_t to_event = (m - 1 - c->step % m) % m;
            if (to_event == 0) to_event = 1;
            run = std::min(run, to_event);
        }
        lbm_status st;
        if (run >= GRAPH_STEPS && c->cur == 0) {
            st = run_graph(c);
            left -= GRAPH_STEPS;
        } else {
            st = one_step(c);
            --left;
        }
        if (st != LBM_OK) return st;
        if (m > 0 && c->step % m == 0) {
            st = run_monitor(c, 1);
            if (st != LBM_OK) return st;
        }
    }
    return LBM_OK;
}

lbm_status lbm_step_timed(lbm_ctx* c, int64_t n, double* ms) {
    if (!c || n < 0 || !ms) return LBM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a));
    if (hipError_t e = hipEventCreate(&b); e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_status(e, "hipEventCreate");
    }
    // the graph that the steps will replay is captured before the first event, so
    // that capture and instantiation stay outside the timed interval
    lbm_status st = n >= GRAPH_STEPS ? capture_graph(c) : LBM_OK;
    if (st != LBM_OK) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return st;
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipEventRecord(a, c->stream);
    if (e == hipSuccess) st = lbm_step(c, n);
    if (e == hipSuccess) e = hipEventRecord(b, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_status(e, "lbm_step_timed");
    *ms = t;
    return st;
}

lbm_status lbm_tune(lbm_ctx* c, int32_t trial_steps, int32_t* tile_y, double* best_ms) {
    if (!c || trial_steps < 1) return LBM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipError_t e = hipEventCreate(&e1); e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_status(e, "hipEventCreate");
    }
    double best = 1e300;
    int best_ty = c->A.tile_y;
    hipError_t e = hipSuccess;
    constexpr size_t MAX_SHAPES = std::size(TILE_Y_CHOICES) + std::size(WIDE_TILE_CODES) + std::size(HOIST_CODES) +
                                  MARCH_K_MAX;
    int shapes[MAX_SHAPES], nshapes = 0;
    if (c->A.scheme != 0) {
        shapes[nshapes++] = SCHEME_TILE_Y;
    } else {
        for (int ty : TILE_Y_CHOICES) shapes[nshapes++] = ty;
        for (int code : WIDE_TILE_CODES) shapes[nshapes++] = code;
        for (int code : HOIST_CODES) shapes[nshapes++] = code;
        if (march_allowed(c->A, c->p.prec))
            for (int k = 1; k <= MARCH_K_MAX; ++k) shapes[nshapes++] = -k;
    }
    for (int k = 0; k < nshapes; ++k) {
        const int ty = shapes[k];
        LatticeArgs A = c->A;
        A.tile_y = ty;
        // trial launches only read the state: each maps f[cur] -> f[cur ^ 1]
        for (int w = 0; w < 2 && e == hipSuccess; ++w)
            e = launch_step(c->p.prec, c->p.eos, MODE_STEP, A, c->f[c->cur], c->f[c->cur ^ 1], c->mu_w, nullptr,
                            c->stream);
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int s = 0; s < trial_steps && e == hipSuccess; ++s)
            e = launch_step(c->p.prec, c->p.eos, MODE_STEP, A, c->f[c->cur], c->f[c->cur ^ 1], c->mu_w, nullptr,
                            c->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        if (ms < best) {
            best = ms;
            best_ty = ty;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_status(e, "lbm_tune");
    if (best_ty != c->A.tile_y) {
        c->A.tile_y = best_ty;
        drop_graph(c);
    }
    if (tile_y) *tile_y = best_ty;
    if (best_ms) *best_ms = best / trial_steps;
    return LBM_OK;
}

lbm_status lbm_set_tile(lbm_ctx* c, int32_t tile_y) {
    if (!c) return LBM_EINVAL;
    bool ok = false;
    if (c->A.scheme != 0) {
        if (tile_y != SCHEME_TILE_Y) return LBM_EINVAL;
        return LBM_OK;
    }
    for (int ty : TILE_Y_CHOICES) ok = ok || ty == tile_y;
    for (int code : WIDE_TILE_CODES) ok = ok || code == tile_y;
    for (int code : HOIST_CODES) ok = ok || code == tile_y;
    if (march_allowed(c->A, c->p.prec))
        ok = ok || (tile_y < 0 && -tile_y <= MARCH_K_MAX);
    if (!ok) return LBM_EINVAL;
    if (tile_y != c->A.tile_y) {
        c->A.tile_y = tile_y;
        drop_graph(c);
    }
    return LBM_OK;
}

lbm_status lbm_monitor_step(lbm_ctx* c) {
    if (!c) return LBM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    lbm_status st = run_monitor(c, 0);
    if (st != LBM_OK) return st;
    st = one_step(c);
    if (st != LBM_OK) return st;
    return run_monitor(c, 1);
}

lbm_status lbm_get_fields(lbm_ctx* c, double* rho, double* vx, double* vy, double* mu) {
    if (!c) return LBM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    const size_t n = (size_t)c->p.nx * c->p.ny;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, 4 * n * sizeof(double)));
    hipError_t e = launch_step(c->p.prec, c->p.eos, MODE_FIELDS, c->A, c->f[c->cur], nullptr, c->mu_w, d, c->stream);
    double* outs[4] = {rho, vx, vy, mu};
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
        if (outs[k]) e = hipMemcpyAsync(outs[k], d + k * n, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    return hip_status(e, "lbm_get_fields");
}

lbm_status lbm_get_fields_noalloc(lbm_ctx* c, double* rho, double* vx, double* vy, double* mu) {
    if (!c) return LBM_EINVAL;
    const size_t n = (size_t)c->p.nx * c->p.ny;
    if (n > (size_t)LBM_NOALLOC_MAX_NODES) {
        std::snprintf(g_last_error, sizeof g_last_error,
                      "lbm_get_fields_noalloc: %zu nodes exceed the %d-node staging array", n,
                      (int)LBM_NOALLOC_MAX_NODES);
        return LBM_EINVAL;
    }
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    double* d = nullptr;
    const lbm_status st = scratch_on_device(c->device, &d);
    if (st != LBM_OK) return st;
    // the field kernel writes all four fields of every node, so nothing left in the
    // array by an earlier call is read
    hipError_t e = launch_step(c->p.prec, c->p.eos, MODE_FIELDS, c->A, c->f[c->cur], nullptr, c->mu_w, d, c->stream);
    double* outs[4] = {rho, vx, vy, mu};
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
        if (outs[k]) e = hipMemcpyAsync(outs[k], d + k * n, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_status(e, "lbm_get_fields_noalloc");
}

lbm_status lbm_set_wall_mu(lbm_ctx* c, int32_t wall, const double* mu_w, int32_t count) {
    if (!c || !mu_w || (wall != 0 && wall != 1)) return LBM_EINVAL;
    const int kind = wall == 0 ? c->p.bc_bottom : c->p.bc_top;
    if (kind != LBM_BC_CPWALL) return LBM_EINVAL;
    if (count != 1 && count != c->p.nx) return LBM_EINVAL;
    for (int i = 0; i < count; ++i)
        if (!std::isfinite(mu_w[i])) return LBM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    for (int x = 0; x < c->p.nx; ++x) c->mu_w_host[(size_t)wall * c->p.nx + x] = mu_w[count == 1 ? 0 : x];
    return upload_mu_w(c);
}

lbm_status lbm_get_monitors(lbm_ctx* c, double* mass, double* residual, int64_t* step, int32_t* flags) {
    if (!c) return LBM_EINVAL;
    if (mass) *mass = c->mass;
    if (residual) *residual = c->residual;
    if (step) *step = c->mon_step;
    if (flags) *flags = c->flags;
    return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx* c, double* f, int64_t* step) {
    if (!c || !f) return LBM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    const size_t n = 9 * (size_t)c->p.nx * c->p.ny;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, n * sizeof(double)));
    hipError_t e = launch_get_state(c->p.prec, c->A, c->f[c->cur], d, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e == hipSuccess && step) *step = c->step;
    return hip_status(e, "lbm_get_state");
}

lbm_status lbm_set_state(lbm_ctx* c, const double* f, int64_t step) {
    if (!c || !f || step < 0) return LBM_EINVAL;
    const size_t plane = (size_t)c->p.nx * c->p.ny;
    const size_t n = 9 * plane;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(f[i])) return LBM_EDOMAIN;
    if (hipSetDevice(c->device) != hipSuccess) return LBM_EHIP;
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, n * sizeof(double)));
    hipError_t e = hipMemcpyAsync(d, f, n * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_init(c->p.prec, c->A, nullptr, nullptr, nullptr, d, c->f[c->cur], c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_status(e, "lbm_set_state");
    c->step = step;
    c->snap_step = -1;
    return LBM_OK;
}

lbm_status lbm_get_temperature(lbm_ctx* c, double* T, double* alpha) {
    if (!c) return LBM_EINVAL;
    if (T) *T = c->fluid.T;
    if (alpha) *alpha = c->fluid.alpha;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    release(c);
}

const char* lbm_last_error(void) { return g_last_error; }

lbm_status lbm_copy_bandwidth(size_t bytes, int32_t iters, double* gbps) {
    if (bytes < 16 || (bytes & 15) || iters < 1 || !gbps) return LBM_EINVAL;
    void *a = nullptr, *b = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&a, bytes);
    if (e == hipSuccess) e = hipMalloc(&b, bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemsetAsync(a, 0, bytes, s);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_copy(a, b, bytes, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int i = 0; i < iters && e == hipSuccess; ++i) e = launch_copy((i & 1) ? b : a, (i & 1) ? a : b, bytes, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e != hipSuccess) return hip_status(e, "lbm_copy_bandwidth");
    *gbps = 2.0 * double(bytes) * iters / (ms * 1e-3) / 1e9;
    return LBM_OK;
}

const char* lbm_strerror(lbm_status s) {
    switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_EDOMAIN: return "density outside the equation-of-state domain";
    case LBM_EDIVERGED: return "simulation diverged (non-finite or out-of-domain density)";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ENOMEM: return "out of device memory or workspace too small";
    case LBM_ESTATE: return "invalid state";
    }
    return "unknown status";
}

lbm_status lbm_critical_point(int32_t eos, double a, double b, double R, double* Tc, double* rho_c, double* p_c) {
    if (eos < 0 || eos > 4 || !(a > 0) || !(b > 0) || !(R > 0)) return LBM_EINVAL;
    double t, r, pc;
    thermo::critical_point(eos, a, b, R, &t, &r, &pc);
    if (Tc) *Tc = t;
    if (rho_c) *rho_c = r;
    if (p_c) *p_c = pc;
    return LBM_OK;
}

lbm_status lbm_coexistence(const lbm_params* p, double* rho_g, double* rho_l, double* p_sat, double* mu_sat) {
    lbm_params q;
    if (!p) return LBM_EINVAL;
    q = *p;
    q.nx = q.ny = 3;  // lattice size is irrelevant here
    q.bc_bottom = q.bc_top = LBM_BC_PERIODIC;
    if (validate(&q) != LBM_OK || !(p->a > 0)) return LBM_EINVAL;
    if (!(p->Tr < 1.0)) return LBM_EDOMAIN;
    const thermo::Fluid fl = thermo::make_fluid(p->eos, p->a, p->b, p->R, p->Tr, p->omega);
    double g, l, ps, ms;
    if (!thermo::coexistence(fl, &g, &l, &ps, &ms)) return LBM_EDOMAIN;
    if (rho_g) *rho_g = g;
    if (rho_l) *rho_l = l;
    if (p_sat) *p_sat = ps;
    if (mu_sat) *mu_sat = ms;
    return LBM_OK;
}

lbm_status lbm_spinodal(const lbm_params* p, double* lo, double* hi) {
    if (!p || !lo || !hi) return LBM_EINVAL;
    lbm_params q = *p;
    q.nx = q.ny = 3;
    q.bc_bottom = q.bc_top = LBM_BC_PERIODIC;
    if (validate(&q) != LBM_OK) return LBM_EINVAL;
    const thermo::Fluid fl = thermo::make_fluid(p->eos, p->a, p->b, p->R, p->Tr, p->omega);
    *lo = *hi = 0.0;
    if (!thermo::spinodal(fl, lo, hi)) *lo = *hi = 0.0;
    return LBM_OK;
}

lbm_status lbm_eos_eval(const lbm_params* p, int64_t n, const double* rho, double* mu_b, double* p0) {
    if (!p || n < 0 || (n > 0 && !rho)) return LBM_EINVAL;
    lbm_params q = *p;
    q.nx = q.ny = 3;
    q.bc_bottom = q.bc_top = LBM_BC_PERIODIC;
    if (validate(&q) != LBM_OK) return LBM_EINVAL;
    const thermo::Fluid fl = thermo::make_fluid(p->eos, p->a, p->b, p->R, p->Tr, p->omega);
    for (int64_t i = 0; i < n; ++i) {
        if (mu_b) mu_b[i] = thermo::mu_b(fl, rho[i]);
        if (p0) p0[i] = thermo::p0(fl, rho[i]);
    }
    return LBM_OK;
}

lbm_status lbm_contact_angle(const double* rho, int32_t nx, int32_t ny, int32_t base_row, double surface_y,
                             double rho_mid, double* theta_deg, double* L, double* H) {
    if (!rho || !std::isfinite(rho_mid) || !std::isfinite(surface_y)) return LBM_EINVAL;
    const int r = thermo::contact_angle(rho, nx, ny, base_row, surface_y, rho_mid, theta_deg, L, H);
    return r == -1 ? LBM_EINVAL : (r == -2 ? LBM_EDOMAIN : LBM_OK);
}

}  // extern "C"
