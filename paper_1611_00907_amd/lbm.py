"""Python binding of the C ABI in ``include/lbm.h`` (argument marshalling only).

Every step of the method runs in the HIP library ``liblbm.so``; this module
only converts numpy arrays to pointers and turns status codes into exceptions.
There is no fallback: if the library is missing, loading fails loudly.

Device memory: by default the library allocates its workspace and uses the
null stream.  ``workspace="torch"`` takes the workspace from PyTorch and runs on
PyTorch's current stream instead; that needs PyTorch imported *before* this
library is loaded, so that both use PyTorch's HIP runtime (a process must not
hold two HIP runtimes, and PyTorch ships its own).
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm.so")

# lbm_status
LBM_OK, LBM_EINVAL, LBM_EDOMAIN, LBM_EDIVERGED, LBM_EHIP, LBM_ENOMEM, LBM_ESTATE = 0, -1, -2, -3, -4, -5, -6
# lbm_eos
LBM_EOS_VDW, LBM_EOS_CS, LBM_EOS_PR, LBM_EOS_RKS, LBM_EOS_RK = 0, 1, 2, 3, 4
# lbm_prec
LBM_F64, LBM_F32, LBM_F16DEV, LBM_BF16DEV = 0, 1, 2, 3
# lbm_bc
LBM_BC_PERIODIC, LBM_BC_CPWALL, LBM_BC_NEUTRAL = 0, 1, 2
# nodes of the largest lattice lbm_get_fields_noalloc serves (LBM_NOALLOC_MAX_NODES)
NOALLOC_MAX_NODES = 2097152

EXPORTED = ["lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_step_timed", "lbm_get_fields",
            "lbm_get_fields_noalloc", "lbm3d_init", "lbm3d_step", "lbm3d_step_timed", "lbm3d_get_fields",
            "lbm3d_get_state", "lbm3d_destroy",
            "lbm_set_wall_mu", "lbm_tune", "lbm_set_tile",
            "lbm_batch_workspace_bytes", "lbm_batch_init", "lbm_batch_step", "lbm_batch_step_timed",
            "lbm_batch_run", "lbm_batch_stop", "lbm_batch_status", "lbm_batch_get_fields", "lbm_batch_get_state",
            "lbm_batch_tune", "lbm_batch_set_schedule", "lbm_batch_fluid_nodes", "lbm_batch_destroy", "lbm_copy_bandwidth",
            "sur_create", "sur_param_count", "sur_set_params", "sur_get_params", "sur_forward", "sur_gradients",
            "sur_set_dataset", "sur_train", "sur_trace", "sur_read", "sur_destroy",
            "lbm_get_monitors", "lbm_monitor_step", "lbm_get_state", "lbm_set_state",
            "lbm_get_temperature", "lbm_destroy", "lbm_strerror", "lbm_last_error", "lbm_critical_point",
            "lbm_coexistence", "lbm_spinodal", "lbm_eos_eval", "lbm_contact_angle", "lbm_warm_cap",
            "lbm_warm_phase", "lbm_warm_density", "lbm_warm_smooth", "lbm_warm_bulk_phases"]


class LbmParams(C.Structure):
    """Mirror of ``lbm_params``."""

    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("bc_bottom", C.c_int32), ("bc_top", C.c_int32),
                ("eos", C.c_int32), ("prec", C.c_int32), ("a", C.c_double), ("b", C.c_double),
                ("R", C.c_double), ("omega", C.c_double), ("Tr", C.c_double), ("tau", C.c_double),
                ("kappa", C.c_double), ("rho_ref", C.c_double), ("monitor_every", C.c_int32),
                ("scheme", C.c_int32), ("trt_lambda", C.c_double), ("mrt_s_e", C.c_double),
                ("mrt_s_eps", C.c_double), ("mrt_s_q", C.c_double)]


# lbm_params.scheme: force | collision
LBM_FORCE_CP, LBM_FORCE_PTENSOR = 0, 1
LBM_COLLIDE_BGK, LBM_COLLIDE_TRT, LBM_COLLIDE_MRT = 0, 16, 32


def make_params(nx, ny, eos, a, b, Tr, tau, kappa, R=1.0, omega=0.0, prec=LBM_F32,
                bc_bottom=LBM_BC_PERIODIC, bc_top=LBM_BC_PERIODIC, rho_ref=1.0,
                monitor_every=0, scheme=0, trt_lambda=0.0, mrt_s_e=0.0, mrt_s_eps=0.0,
                mrt_s_q=0.0) -> LbmParams:
    return LbmParams(int(nx), int(ny), int(bc_bottom), int(bc_top), int(eos), int(prec), float(a),
                     float(b), float(R), float(omega), float(Tr), float(tau), float(kappa),
                     float(rho_ref), int(monitor_every), int(scheme), float(trt_lambda), float(mrt_s_e),
                     float(mrt_s_eps), float(mrt_s_q))


class LbmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = ""
        if status == LBM_EHIP:
            try:
                detail = " [" + load_library().lbm_last_error().decode() + "]"
            except RuntimeError:
                pass
        super().__init__("%s: %s (%d)%s" % (where, strerror(status), status, detail))


class LbmDiverged(LbmError):
    pass


_lib = None
_torch_runtime = False   # True when PyTorch's HIP runtime was in the process first


def load_library():
    """Loads liblbm.so; raises if it has not been built (no CPU fallback exists)."""
    global _lib, _torch_runtime
    if _lib is not None:
        return _lib
    _torch_runtime = "torch" in sys.modules
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblbm.so is not built: run `python -m paper_1611_00907_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER(LbmParams)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    lib.lbm_workspace_bytes.argtypes = [P]
    lib.lbm_workspace_bytes.restype = C.c_size_t
    lib.lbm_init.argtypes = [P, vp, vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.lbm_step.argtypes = [vp, C.c_int64]
    lib.lbm_step_timed.argtypes = [vp, C.c_int64, dp]
    lib.lbm_get_fields.argtypes = [vp, vp, vp, vp, vp]
    lib.lbm_get_fields_noalloc.argtypes = [vp, vp, vp, vp, vp]
    lib.lbm_set_wall_mu.argtypes = [vp, C.c_int32, vp, C.c_int32]
    lib.lbm_get_monitors.argtypes = [vp, dp, dp, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    lib.lbm_monitor_step.argtypes = [vp]
    lib.lbm_get_state.argtypes = [vp, vp, C.POINTER(C.c_int64)]
    lib.lbm_set_state.argtypes = [vp, vp, C.c_int64]
    lib.lbm_get_temperature.argtypes = [vp, dp, dp]
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_destroy.restype = None
    lib.lbm_strerror.argtypes = [C.c_int]
    lib.lbm_strerror.restype = C.c_char_p
    lib.lbm_last_error.argtypes = []
    lib.lbm_last_error.restype = C.c_char_p
    lib.lbm_tune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), dp]
    lib.lbm_set_tile.argtypes = [vp, C.c_int32]
    lib.lbm_batch_workspace_bytes.argtypes = [P, C.c_int32]
    lib.lbm_batch_workspace_bytes.restype = C.c_size_t
    lib.lbm_batch_init.argtypes = [P, C.c_int32, vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.lbm_batch_step.argtypes = [vp, C.c_int64]
    lib.lbm_batch_step_timed.argtypes = [vp, C.c_int64, dp]
    lib.lbm_batch_run.argtypes = [vp, C.c_int64, C.c_int32, C.c_int32, C.c_double, C.POINTER(C.c_int64)]
    lib.lbm_batch_stop.argtypes = [vp, vp, C.c_int32]
    lib.lbm_batch_status.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.lbm_batch_get_fields.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    lib.lbm_batch_get_state.argtypes = [vp, C.c_int32, vp]
    lib.lbm_batch_tune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp]
    lib.lbm_batch_set_schedule.argtypes = [vp, C.c_int32, C.c_int32]
    lib.lbm_batch_fluid_nodes.argtypes = [vp, C.c_int32]
    lib.lbm_batch_fluid_nodes.restype = C.c_int64
    lib.lbm_batch_destroy.argtypes = [vp]
    lib.lbm_batch_destroy.restype = None
    lib.lbm_copy_bandwidth.argtypes = [C.c_size_t, C.c_int32, dp]
    lib.sur_create.argtypes = [C.c_int32, C.c_int32, C.POINTER(vp)]
    lib.sur_param_count.argtypes = [vp]
    lib.sur_param_count.restype = C.c_int64
    lib.sur_set_params.argtypes = [vp, vp]
    lib.sur_get_params.argtypes = [vp, vp]
    lib.sur_forward.argtypes = [vp, vp, C.c_int32, vp]
    lib.sur_gradients.argtypes = [vp, vp, vp, C.c_int32, vp, dp]
    lib.sur_set_dataset.argtypes = [vp, vp, vp, C.c_int32]
    lib.sur_train.argtypes = [vp, C.c_int32, C.c_int32, C.c_float, C.c_uint64, vp]
    lib.sur_trace.argtypes = [vp, C.c_int32]
    lib.sur_read.argtypes = [vp, C.c_char_p, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.sur_destroy.argtypes = [vp]
    lib.sur_destroy.restype = None
    lib.lbm3d_init.argtypes = [P, C.c_int32, vp, C.POINTER(vp)]
    lib.lbm3d_step.argtypes = [vp, C.c_int64]
    lib.lbm3d_step_timed.argtypes = [vp, C.c_int64, dp]
    lib.lbm3d_get_fields.argtypes = [vp] + [vp] * 5
    lib.lbm3d_get_state.argtypes = [vp, vp, C.POINTER(C.c_int64)]
    lib.lbm3d_destroy.argtypes = [vp]
    lib.lbm3d_destroy.restype = None
    lib.lbm_critical_point.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, dp, dp, dp]
    lib.lbm_coexistence.argtypes = [P, dp, dp, dp, dp]
    lib.lbm_spinodal.argtypes = [P, dp, dp]
    lib.lbm_eos_eval.argtypes = [P, C.c_int64, vp, vp, vp]
    lib.lbm_contact_angle.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                      dp, dp, dp]
    d = C.c_double
    lib.lbm_warm_cap.argtypes = [C.c_int32, C.c_int32, d, d, d, d, d, d, vp]
    lib.lbm_warm_phase.argtypes = [C.c_int64, vp, d, d, vp]
    lib.lbm_warm_density.argtypes = [C.c_int64, vp, d, d, vp]
    lib.lbm_warm_smooth.argtypes = [C.c_int32, C.c_int32, vp, C.c_float, C.c_float, vp]
    lib.lbm_warm_bulk_phases.argtypes = [C.c_int32, C.c_int32, vp, dp, dp]
    for name in EXPORTED:
        if name not in ("lbm_workspace_bytes", "lbm_destroy", "lbm_strerror", "lbm_last_error",
                        "lbm_batch_workspace_bytes", "lbm_batch_fluid_nodes", "lbm_batch_destroy",
                        "sur_param_count", "sur_destroy", "lbm3d_destroy"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def strerror(status: int) -> str:
    try:
        return load_library().lbm_strerror(int(status)).decode()
    except RuntimeError:
        return "status %d" % status


def _check(status: int, where: str):
    if status == LBM_EDIVERGED:
        raise LbmDiverged(status, where)
    if status != LBM_OK:
        raise LbmError(status, where)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- host tools
def lbm_critical_point(eos: int, a: float, b: float, R: float = 1.0):
    lib = load_library()
    out = [C.c_double() for _ in range(3)]
    _check(lib.lbm_critical_point(int(eos), float(a), float(b), float(R), *[C.byref(o) for o in out]),
           "lbm_critical_point")
    return tuple(o.value for o in out)


def lbm_coexistence(p: LbmParams):
    """(rho_g, rho_l, p_sat, mu_sat) of the fluid in p (Maxwell equal area)."""
    lib = load_library()
    out = [C.c_double() for _ in range(4)]
    _check(lib.lbm_coexistence(C.byref(p), *[C.byref(o) for o in out]), "lbm_coexistence")
    return tuple(o.value for o in out)


def lbm_spinodal(p: LbmParams):
    """(lo, hi): dp0/drho < 0 for lo < rho < hi; (0, 0) at or above Tc."""
    lib = load_library()
    lo, hi = C.c_double(), C.c_double()
    _check(lib.lbm_spinodal(C.byref(p), C.byref(lo), C.byref(hi)), "lbm_spinodal")
    return lo.value, hi.value


def lbm_eos_eval(p: LbmParams, rho):
    lib = load_library()
    rho = _f64(rho).ravel()
    mu, p0 = np.empty_like(rho), np.empty_like(rho)
    _check(lib.lbm_eos_eval(C.byref(p), rho.size, _p(rho), _p(mu), _p(p0)), "lbm_eos_eval")
    return mu, p0


def lbm_contact_angle(rho, rho_mid: float, base_row: int = 1, surface_y=None):
    """(theta_deg, L, H) of the drop on base_row of rho[ny][nx] (Sec. V formula)."""
    lib = load_library()
    rho = _f64(rho)
    ny, nx = rho.shape
    sy = float(base_row) if surface_y is None else float(surface_y)
    out = [C.c_double() for _ in range(3)]
    _check(lib.lbm_contact_angle(_p(rho), nx, ny, int(base_row), sy, float(rho_mid),
                                 *[C.byref(o) for o in out]), "lbm_contact_angle")
    return tuple(o.value for o in out)


def warm_cap(nx: int, ny: int, rho_in: float, rho_out: float, radius: float, cx: float, cy: float,
             width: float = 4.0):
    """Drop of rho_in in rho_out with a tanh interface (lbm_warm_cap): [ny][nx] doubles."""
    out = np.empty((ny, nx))
    _check(load_library().lbm_warm_cap(int(nx), int(ny), float(rho_in), float(rho_out), float(radius), float(cx),
                                       float(cy), float(width), _p(out)), "lbm_warm_cap")
    return out


def warm_phase(rho, rho_g: float, rho_l: float):
    """ln(rho / rho_g) / ln(rho_l / rho_g) as float32 (lbm_warm_phase)."""
    rho = _f64(rho)
    out = np.empty(rho.shape, np.float32)
    _check(load_library().lbm_warm_phase(rho.size, _p(rho), float(rho_g), float(rho_l), _p(out)), "lbm_warm_phase")
    return out


def warm_density(phi, rho_g: float, rho_l: float):
    """rho_g exp(phi ln(rho_l / rho_g)) as float64 (lbm_warm_density)."""
    phi = np.ascontiguousarray(phi, dtype=np.float32)
    out = np.empty(phi.shape)
    _check(load_library().lbm_warm_density(phi.size, _p(phi), float(rho_g), float(rho_l), _p(out)),
           "lbm_warm_density")
    return out


def warm_smooth(pred, lo: float = -0.5, hi: float = 1.5):
    """One D2Q9-weighted smoothing pass of pred clipped to [lo, hi] (lbm_warm_smooth), float32."""
    pred = np.ascontiguousarray(pred, dtype=np.float32)
    ny, nx = pred.shape
    out = np.empty_like(pred)
    _check(load_library().lbm_warm_smooth(nx, ny, _p(pred), float(lo), float(hi), _p(out)), "lbm_warm_smooth")
    return out


def warm_bulk_phases(phi):
    """(liquid, vapour) phase levels of a phase field (lbm_warm_bulk_phases)."""
    phi = np.ascontiguousarray(phi, dtype=np.float32)
    ny, nx = phi.shape
    hl, hg = C.c_double(), C.c_double()
    _check(load_library().lbm_warm_bulk_phases(nx, ny, _p(phi), C.byref(hl), C.byref(hg)), "lbm_warm_bulk_phases")
    return hl.value, hg.value


def lbm_copy_bandwidth(nbytes: int, iters: int = 20) -> float:
    """GB/s of a plain device copy (read + write bytes over time)."""
    g = C.c_double()
    _check(load_library().lbm_copy_bandwidth(int(nbytes), int(iters), C.byref(g)), "lbm_copy_bandwidth")
    return g.value


def lbm_workspace_bytes(p: LbmParams) -> int:
    return int(load_library().lbm_workspace_bytes(C.byref(p)))


# ---------------------------------------------------------------- lattice
def _torch_workspace(nbytes: int):
    """Device workspace and current stream from PyTorch (plumbing only)."""
    if not _torch_runtime:
        raise RuntimeError("workspace='torch' needs `import torch` before liblbm.so is loaded, so that "
                           "the library binds to PyTorch's HIP runtime")
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible to PyTorch")
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    return ws, int(ws.data_ptr()), int(torch.cuda.current_stream().cuda_stream)


def lbm_init(p: LbmParams, rho0, ux0=None, uy0=None, workspace=None):
    """Returns a Lattice owning the context; workspace None lets the library
    allocate, 'torch' takes device memory and the current stream from PyTorch."""
    return Lattice(p, rho0, ux0, uy0, workspace)


class Lattice:
    """One lattice on the GPU: a thin owner of an ``lbm_ctx``."""

    def __init__(self, p: LbmParams, rho0, ux0=None, uy0=None, workspace=None):
        self.lib = load_library()
        self.p = p
        self.nx, self.ny = p.nx, p.ny
        rho0, ux0, uy0 = _f64(rho0), _f64(ux0), _f64(uy0)
        shape = (p.ny, p.nx)
        for a in (rho0, ux0, uy0):
            if a is not None and a.shape != shape:
                raise ValueError("field shape %s, expected %s" % (a.shape, shape))
        self._ws = None
        ws_ptr, ws_bytes, stream = None, 0, None
        if workspace == "torch":
            nbytes = lbm_workspace_bytes(p)
            if nbytes == 0:
                _check(LBM_EINVAL, "lbm_workspace_bytes")
            self._ws, ws_ptr, stream = _torch_workspace(nbytes)
            ws_bytes = nbytes
        ctx = C.c_void_p()
        _check(self.lib.lbm_init(C.byref(p), _p(rho0), _p(ux0), _p(uy0), ws_ptr, ws_bytes, stream,
                                 C.byref(ctx)), "lbm_init")
        self.ctx = ctx

    def step(self, n: int = 1):
        _check(self.lib.lbm_step(self.ctx, int(n)), "lbm_step")

    def step_timed(self, n: int) -> float:
        """Milliseconds of device time for n steps (HIP events on the lattice's stream)."""
        ms = C.c_double()
        _check(self.lib.lbm_step_timed(self.ctx, int(n), C.byref(ms)), "lbm_step_timed")
        return ms.value

    def tune(self, trial_steps: int = 50):
        """Picks the fastest tile height for this lattice; returns (tile_y, ms per step)."""
        ty, ms = C.c_int32(), C.c_double()
        _check(self.lib.lbm_tune(self.ctx, int(trial_steps), C.byref(ty), C.byref(ms)), "lbm_tune")
        return ty.value, ms.value

    def set_tile(self, tile_y: int):
        _check(self.lib.lbm_set_tile(self.ctx, int(tile_y)), "lbm_set_tile")

    def monitor_step(self):
        _check(self.lib.lbm_monitor_step(self.ctx), "lbm_monitor_step")
        return self.monitors()

    def fields(self, noalloc: bool = False, which=("rho", "vx", "vy", "mu")):
        """Output fields (lbm_get_fields; noalloc=True: lbm_get_fields_noalloc, which
        stages them in the library's static device array instead of a per-call
        allocation).  Fields not in `which` are passed as NULL and not returned."""
        shape = (self.ny, self.nx)
        out = {k: np.empty(shape) for k in which}
        fn = self.lib.lbm_get_fields_noalloc if noalloc else self.lib.lbm_get_fields
        _check(fn(self.ctx, *[_p(out.get(k)) for k in ("rho", "vx", "vy", "mu")]),
               "lbm_get_fields_noalloc" if noalloc else "lbm_get_fields")
        return out

    def set_wall_mu(self, wall: int, mu_w):
        mu = np.atleast_1d(_f64(mu_w))
        _check(self.lib.lbm_set_wall_mu(self.ctx, int(wall), _p(mu), int(mu.size)), "lbm_set_wall_mu")

    def monitors(self):
        m, r, s, f = C.c_double(), C.c_double(), C.c_int64(), C.c_int32()
        _check(self.lib.lbm_get_monitors(self.ctx, C.byref(m), C.byref(r), C.byref(s), C.byref(f)),
               "lbm_get_monitors")
        return {"mass": m.value, "residual": r.value, "step": s.value, "flags": f.value}

    def get_state(self):
        f = np.empty((9, self.ny, self.nx))
        s = C.c_int64()
        _check(self.lib.lbm_get_state(self.ctx, _p(f), C.byref(s)), "lbm_get_state")
        return f, s.value

    def set_state(self, f, step: int = 0):
        f = _f64(f)
        if f.shape != (9, self.ny, self.nx):
            raise ValueError("state shape %s" % (f.shape,))
        _check(self.lib.lbm_set_state(self.ctx, _p(f), int(step)), "lbm_set_state")

    def temperature(self):
        T, al = C.c_double(), C.c_double()
        _check(self.lib.lbm_get_temperature(self.ctx, C.byref(T), C.byref(al)), "lbm_get_temperature")
        return T.value, al.value

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.lbm_destroy(self.ctx)
            self.ctx = C.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- batches
def lbm_batch_workspace_bytes(cases) -> int:
    arr = (LbmParams * len(cases))(*cases)
    return int(load_library().lbm_batch_workspace_bytes(arr, len(cases)))


class Batch:
    """Many lattices advanced by one persistent launch per step (``lbm_batch``)."""

    ACTIVE, CONVERGED, DIVERGED = 0, 1, 2

    def __init__(self, cases, rho0s, mu_w_bottom=None):
        self.lib = load_library()
        self.n = len(cases)
        self.cases = list(cases)
        self._arr = (LbmParams * self.n)(*cases)
        self._rho = [_f64(r) for r in rho0s]
        for p, r in zip(self.cases, self._rho):
            if r.shape != (p.ny, p.nx):
                raise ValueError("rho0 shape %s, expected %s" % (r.shape, (p.ny, p.nx)))
        ptrs = (C.c_void_p * self.n)(*[r.ctypes.data for r in self._rho])
        mw = None if mu_w_bottom is None else _f64(np.asarray(mu_w_bottom, dtype=np.float64).ravel())
        ctx = C.c_void_p()
        _check(self.lib.lbm_batch_init(self._arr, self.n, ptrs, _p(mw), None, 0, None, C.byref(ctx)),
               "lbm_batch_init")
        self.ctx = ctx

    def step(self, n: int):
        _check(self.lib.lbm_batch_step(self.ctx, int(n)), "lbm_batch_step")

    def step_timed(self, n: int) -> float:
        ms = C.c_double()
        _check(self.lib.lbm_batch_step_timed(self.ctx, int(n), C.byref(ms)), "lbm_batch_step_timed")
        return ms.value

    def run(self, max_steps: int, check_every: int = 100, window: int = 1, tol: float = 1e-9) -> int:
        s = C.c_int64()
        _check(self.lib.lbm_batch_run(self.ctx, int(max_steps), int(check_every), int(window), float(tol),
                                      C.byref(s)), "lbm_batch_run")
        return s.value

    def stop(self, cases):
        """Masks the given cases out of every later step (lbm_batch_stop)."""
        idx = np.ascontiguousarray(np.atleast_1d(np.asarray(cases, dtype=np.int32)))
        _check(self.lib.lbm_batch_stop(self.ctx, _p(idx), int(idx.size)), "lbm_batch_stop")

    def status(self):
        st = np.zeros(self.n, np.int32)
        steps = np.zeros(self.n, np.int64)
        res, mass = np.zeros(self.n), np.zeros(self.n)
        fl = np.zeros(self.n, np.int32)
        _check(self.lib.lbm_batch_status(self.ctx, _p(st), _p(steps), _p(res), _p(mass), _p(fl)),
               "lbm_batch_status")
        return {"state": st, "steps": steps, "residual": res, "mass": mass, "flags": fl}

    def fields(self, i: int):
        p = self.cases[i]
        out = {k: np.empty((p.ny, p.nx)) for k in ("rho", "vx", "vy", "mu")}
        _check(self.lib.lbm_batch_get_fields(self.ctx, int(i), *[_p(out[k]) for k in ("rho", "vx", "vy", "mu")]),
               "lbm_batch_get_fields")
        return out

    def rho(self, i: int):
        """Density of case i (the other output fields are not computed into host memory)."""
        p = self.cases[i]
        r = np.empty((p.ny, p.nx))
        _check(self.lib.lbm_batch_get_fields(self.ctx, int(i), _p(r), None, None, None), "lbm_batch_get_fields")
        return r

    def get_state(self, i: int):
        p = self.cases[i]
        f = np.empty((9, p.ny, p.nx))
        _check(self.lib.lbm_batch_get_state(self.ctx, int(i), _p(f)), "lbm_batch_get_state")
        return f

    def tune(self, trial_steps: int = 20):
        ty, bpc, ms = C.c_int32(), C.c_int32(), C.c_double()
        _check(self.lib.lbm_batch_tune(self.ctx, int(trial_steps), C.byref(ty), C.byref(bpc), C.byref(ms)),
               "lbm_batch_tune")
        return ty.value, bpc.value, ms.value

    def set_schedule(self, tile_y: int, blocks_per_cu: int):
        _check(self.lib.lbm_batch_set_schedule(self.ctx, int(tile_y), int(blocks_per_cu)), "lbm_batch_set_schedule")

    def fluid_nodes(self, active_only: bool = False) -> int:
        return int(self.lib.lbm_batch_fluid_nodes(self.ctx, 1 if active_only else 0))

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.lbm_batch_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- D3Q19
class Lattice3:
    """A periodic D3Q19 box (``lbm3d_*``); fields [nz][ny][nx], distributions
    [19][nz][ny][nx] in the direction order of lbm.h."""

    def __init__(self, p: LbmParams, nz: int, rho0):
        self.lib = load_library()
        self.p, self.nz = p, int(nz)
        self.shape = (self.nz, p.ny, p.nx)
        rho0 = _f64(rho0)
        if rho0.shape != self.shape:
            raise ValueError("rho0 shape %s, expected %s" % (rho0.shape, self.shape))
        ctx = C.c_void_p()
        _check(self.lib.lbm3d_init(C.byref(p), self.nz, _p(rho0), C.byref(ctx)), "lbm3d_init")
        self.ctx = ctx

    def step(self, n: int):
        _check(self.lib.lbm3d_step(self.ctx, int(n)), "lbm3d_step")

    def step_timed(self, n: int) -> float:
        ms = C.c_double()
        _check(self.lib.lbm3d_step_timed(self.ctx, int(n), C.byref(ms)), "lbm3d_step_timed")
        return ms.value

    def fields(self):
        out = {k: np.empty(self.shape) for k in ("rho", "vx", "vy", "vz", "mu")}
        _check(self.lib.lbm3d_get_fields(self.ctx, *[_p(out[k]) for k in ("rho", "vx", "vy", "vz", "mu")]),
               "lbm3d_get_fields")
        return out

    def get_state(self):
        f = np.empty((19,) + self.shape)
        s = C.c_int64()
        _check(self.lib.lbm3d_get_state(self.ctx, _p(f), C.byref(s)), "lbm3d_get_state")
        return f, s.value

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.lbm3d_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- surrogate
class Surrogate:
    """The convolutional warm-start network (``sur_*``): BF16 MFMA kernels on the GPU.

    Parameters use the exchange layout of ``lbm.h`` (per layer w[co][ci][3][3], b[co])."""

    LAYERS = [("e0a", 16, 32), ("e0b", 32, 32), ("e1a", 32, 64), ("e1b", 64, 64), ("e2a", 64, 96),
              ("e2b", 96, 96), ("e3a", 96, 128), ("e3b", 128, 128), ("d2a", 224, 96), ("d2b", 96, 96),
              ("d1a", 160, 64), ("d1b", 64, 64), ("d0a", 96, 32), ("d0b", 32, 32), ("out", 32, 1)]

    def __init__(self, size: int, max_batch: int):
        self.lib = load_library()
        self.size, self.max_batch = int(size), int(max_batch)
        ctx = C.c_void_p()
        _check(self.lib.sur_create(self.size, self.max_batch, C.byref(ctx)), "sur_create")
        self.ctx = ctx
        self.n_params = int(self.lib.sur_param_count(self.ctx))

    @classmethod
    def unflatten(cls, flat):
        """Exchange-layout vector -> {name: (w [co,ci,3,3], b [co])}."""
        out, o = {}, 0
        for name, ci, co in cls.LAYERS:
            w = flat[o:o + co * ci * 9].reshape(co, ci, 3, 3)
            o += co * ci * 9
            out[name] = (w, flat[o:o + co])
            o += co
        return out

    @classmethod
    def flatten(cls, params):
        return np.concatenate([np.concatenate([np.asarray(params[n][0], np.float64).ravel(),
                                               np.asarray(params[n][1], np.float64).ravel()])
                               for n, _, _ in cls.LAYERS]).astype(np.float32)

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == self.n_params
        _check(self.lib.sur_set_params(self.ctx, _p(flat)), "sur_set_params")

    def get_params(self):
        flat = np.empty(self.n_params, np.float32)
        _check(self.lib.sur_get_params(self.ctx, _p(flat)), "sur_get_params")
        return flat

    def forward(self, inputs):
        x = np.ascontiguousarray(inputs, dtype=np.float32)
        n = x.shape[0]
        out = np.empty((n, self.size, self.size), np.float32)
        _check(self.lib.sur_forward(self.ctx, _p(x), n, _p(out)), "sur_forward")
        return out

    def gradients(self, inputs, targets):
        x = np.ascontiguousarray(inputs, dtype=np.float32)
        t = np.ascontiguousarray(targets, dtype=np.float32)
        g = np.empty(self.n_params, np.float32)
        loss = C.c_double()
        _check(self.lib.sur_gradients(self.ctx, _p(x), _p(t), x.shape[0], _p(g), C.byref(loss)), "sur_gradients")
        return g, loss.value

    def set_dataset(self, inputs, targets):
        self._ds = (np.ascontiguousarray(inputs, dtype=np.float32), np.ascontiguousarray(targets, dtype=np.float32))
        _check(self.lib.sur_set_dataset(self.ctx, _p(self._ds[0]), _p(self._ds[1]), self._ds[0].shape[0]),
               "sur_set_dataset")

    def train(self, steps: int, batch: int, lr: float, seed: int = 0):
        losses = np.empty(int(steps), np.float32)
        _check(self.lib.sur_train(self.ctx, int(steps), int(batch), float(lr), int(seed), _p(losses)), "sur_train")
        return losses

    def trace(self, on: bool = True):
        _check(self.lib.sur_trace(self.ctx, int(bool(on))), "sur_trace")

    def read(self, name: str):
        """Internal tensor of the last pass as float32 NHWC [N][H][W][C] (sur_read)."""
        shape = (C.c_int64 * 4)()
        _check(self.lib.sur_read(self.ctx, name.encode(), None, 0, shape), "sur_read(%s)" % name)
        out = np.empty(tuple(shape), np.float32)
        _check(self.lib.sur_read(self.ctx, name.encode(), _p(out), out.size, shape), "sur_read(%s)" % name)
        return out

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.sur_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
