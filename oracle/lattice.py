"""ctypes binding of the plain C time step (TEST INFRASTRUCTURE ONLY).

The C file ``cplbm_oracle.c`` holds the method (Eqs 8, 12, 13, 14, 28); this
module only marshals numpy arrays and keeps the ping-pong buffers.  It builds
the shared library with gcc on first use if it is missing or stale.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time
from dataclasses import dataclass

import numpy as np

from . import thermo

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cplbm_oracle.c")
_LIB = os.path.join(_HERE, "libcplbm_oracle.so")

PERIODIC, CPWALL, NEUTRAL = 0, 1, 2

# IEEE double without contraction so the oracle's rounding is that of the
# plain formulas; OpenMP only splits rows between threads.
GCC_CMD = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", _SRC, "-o", _LIB, "-lm"]


def build_library(force: bool = False) -> str:
    stale = (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = [tmp if c == _LIB else c for c in GCC_CMD]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


# nonideal force (Eq 12, or Eq 5 with the pressure tensor of Eq 9) and collision
FORCE_CP, FORCE_PTENSOR = 0, 1
COLLIDE_BGK, COLLIDE_TRT, COLLIDE_MRT = 0, 16, 32


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("bottom", C.c_int32), ("top", C.c_int32),
                ("eos", C.c_int32), ("scheme", C.c_int32), ("a", C.c_double), ("b", C.c_double),
                ("R", C.c_double), ("T", C.c_double), ("alpha", C.c_double), ("tau", C.c_double),
                ("kappa", C.c_double), ("trt_lambda", C.c_double), ("s_e", C.c_double),
                ("s_eps", C.c_double), ("s_q", C.c_double)]


_lib = None


def load_library():
    global _lib
    if _lib is None:
        build_library()
        lib = C.CDLL(_LIB)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        P = C.POINTER(_Params)
        lib.ora_eos.argtypes = [P, C.c_int64, dp, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.ora_feq.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        lib.ora_init.argtypes = [P, dp, C.c_void_p, C.c_void_p, dp]
        lib.ora_step.argtypes = [P, dp, dp, dp, dp, dp]
        lib.ora_run.argtypes = [P, dp, dp, dp, dp, dp, C.c_int64]
        lib.ora_fields.argtypes = [P, dp, dp, dp] + [C.c_void_p] * 6 + [dp]
        lib.ora_mass.argtypes = [P, dp]
        lib.ora_mass.restype = C.c_double
        lib.ora_stencils.argtypes = [P, dp, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.ora_mrt_matrix.argtypes = [dp]
        lib.ora_max_threads.restype = C.c_int
        lib.ora_set_threads.argtypes = [C.c_int]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


@dataclass
class OracleParams:
    """Problem statement of the paper: lattice size, boundaries, EOS, tau, kappa.

    ``T`` is absolute; ``alpha`` is alpha(T).  Use ``from_reduced`` to set the
    temperature as Tr = T / Tc (Sec. III)."""

    nx: int
    ny: int
    eos: int
    a: float
    b: float
    R: float
    T: float
    alpha: float
    tau: float
    kappa: float
    bottom: int = PERIODIC
    top: int = PERIODIC
    scheme: int = FORCE_CP | COLLIDE_BGK
    trt_lambda: float = 0.25      # TRT: (tau - 1/2)(tau_minus - 1/2)
    s_e: float = 1.0              # MRT rates of the energy moments e and epsilon
    s_eps: float = 1.0
    s_q: float = -1.0             # MRT rate of the heat-flux moments; < 0: 8 (2 - s) / (8 - s), s = 1/tau

    @staticmethod
    def from_reduced(nx, ny, eos, a, b, Tr, tau, kappa, R=1.0, omega=0.0, bottom=PERIODIC,
                     top=PERIODIC, **scheme) -> "OracleParams":
        fl = thermo.fluid_at(eos, a, b, R, Tr, omega)
        return OracleParams(nx, ny, eos, a, b, R, fl.T, fl.alpha, tau, kappa, bottom, top, **scheme)

    def fluid(self) -> thermo.Fluid:
        return thermo.Fluid(self.eos, self.a, self.b, self.R, self.T, self.alpha)

    def c(self) -> _Params:
        if (self.bottom == PERIODIC) != (self.top == PERIODIC):
            raise ValueError("y is periodic only when both bottom and top are periodic")
        if (self.scheme & 15) == FORCE_PTENSOR and self.bottom != PERIODIC:
            raise ValueError("the pressure-tensor force is defined on periodic lattices only")
        sn = 1.0 / self.tau
        s_q = self.s_q if self.s_q > 0 else 8.0 * (2.0 - sn) / (8.0 - sn)
        return _Params(self.nx, self.ny, self.bottom, self.top, self.eos, self.scheme, self.a, self.b,
                       self.R, self.T, self.alpha, self.tau, self.kappa, self.trt_lambda, self.s_e,
                       self.s_eps, s_q)

    def solid_rows(self):
        rows = []
        if self.bottom != PERIODIC:
            rows.append(0)
        if self.top != PERIODIC:
            rows.append(self.ny - 1)
        return rows

    def fluid_mask(self):
        m = np.ones((self.ny, self.nx), dtype=bool)
        for r in self.solid_rows():
            m[r, :] = False
        return m


def eos_c(p: OracleParams, rho):
    """psi, p0, mu_b of the C oracle at the densities rho (1-D)."""
    lib = load_library()
    rho = np.ascontiguousarray(rho, dtype=np.float64).ravel()
    out = [np.empty_like(rho) for _ in range(3)]
    lib.ora_eos(C.byref(p.c()), rho.size, rho, *[_ptr(o) for o in out])
    return out


def feq_c(rho, ux, uy):
    lib = load_library()
    out = np.empty(9)
    lib.ora_feq(float(rho), float(ux), float(uy), out)
    return out


def stencils_c(p: OracleParams, phi):
    """Isotropic Laplacian and gradient of phi with periodic wrap (test probe)."""
    lib = load_library()
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    lap, gx, gy = (np.empty_like(phi) for _ in range(3))
    q = OracleParams(**{**p.__dict__, "bottom": PERIODIC, "top": PERIODIC})
    lib.ora_stencils(C.byref(q.c()), phi, _ptr(lap), _ptr(gx), _ptr(gy))
    return lap, gx, gy


def mrt_matrix():
    """The D2Q9 moment matrix the oracle's MRT collision uses (rows: rho, e, eps,
    j_x, q_x, j_y, q_y, p_xx, p_xy)."""
    out = np.empty(81)
    load_library().ora_mrt_matrix(out)
    return out.reshape(9, 9)


def set_threads(n: int):
    load_library().ora_set_threads(int(n))


def max_threads() -> int:
    return int(load_library().ora_max_threads())


class OracleLattice:
    """Driver of the C oracle: state f is [9][ny][nx] (post-streaming, time t)."""

    def __init__(self, p: OracleParams, rho0, ux0=None, uy0=None, mu_w_bottom=0.0,
                 mu_w_top=0.0):
        self.p = p
        self._cp = p.c()
        self.lib = load_library()
        shape = (p.ny, p.nx)
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        assert rho0.shape == shape
        self.f = np.zeros((9, p.ny, p.nx))
        self.fbuf = np.zeros_like(self.f)
        self.work = np.zeros((7, p.ny, p.nx))
        self.mu_w_bottom = np.zeros(p.nx)
        self.mu_w_top = np.zeros(p.nx)
        self.set_wall_mu(0, mu_w_bottom)
        self.set_wall_mu(1, mu_w_top)
        ux0 = None if ux0 is None else np.ascontiguousarray(ux0, dtype=np.float64)
        uy0 = None if uy0 is None else np.ascontiguousarray(uy0, dtype=np.float64)
        self.lib.ora_init(C.byref(self._cp), rho0, _ptr(ux0), _ptr(uy0), self.f)
        self.steps = 0

    def set_wall_mu(self, wall: int, mu_w):
        target = self.mu_w_bottom if wall == 0 else self.mu_w_top
        target[:] = np.broadcast_to(np.asarray(mu_w, dtype=np.float64), target.shape)

    def step(self, n: int = 1):
        if n <= 0:
            return
        self.lib.ora_run(C.byref(self._cp), self.mu_w_bottom, self.mu_w_top, self.f, self.fbuf,
                         self.work, int(n))
        self.steps += n

    def fields(self):
        """dict of rho, vx, vy, mu, Fx, Fy ([ny][nx]) of the current state."""
        shape = (self.p.ny, self.p.nx)
        out = {k: np.empty(shape) for k in ("rho", "vx", "vy", "mu", "Fx", "Fy")}
        self.lib.ora_fields(C.byref(self._cp), self.mu_w_bottom, self.mu_w_top, self.f,
                            *[_ptr(out[k]) for k in ("rho", "vx", "vy", "mu", "Fx", "Fy")],
                            self.work)
        return out

    def mass(self) -> float:
        return float(self.lib.ora_mass(C.byref(self._cp), self.f))

    def timed_steps(self, n: int) -> float:
        t0 = time.perf_counter()
        self.step(n)
        return time.perf_counter() - t0
