"""ctypes binding of the plain C D3Q19 step (TEST INFRASTRUCTURE ONLY).

``cplbm3d_oracle.c`` holds the method; this module marshals numpy arrays, keeps
the ping-pong buffers, and builds the shared library with gcc when it is
missing or stale.  Arrays are [nz][ny][nx] (x fastest); distributions
[19][nz][ny][nx].
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
_SRC = os.path.join(_HERE, "cplbm3d_oracle.c")
_LIB = os.path.join(_HERE, "libcplbm3d_oracle.so")
GCC_CMD = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", _SRC, "-o", _LIB, "-lm"]


def build_library(force: bool = False) -> str:
    stale = (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run([tmp if c == _LIB else c for c in GCC_CMD], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("eos", C.c_int32),
                ("a", C.c_double), ("b", C.c_double), ("R", C.c_double), ("T", C.c_double),
                ("alpha", C.c_double), ("tau", C.c_double), ("kappa", C.c_double)]


_lib = None


def load_library():
    global _lib
    if _lib is None:
        build_library()
        lib = C.CDLL(_LIB)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        P = C.POINTER(_Params)
        lib.o3_velocities.argtypes = [ip, ip, ip, dp]
        lib.o3_feq.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
        lib.o3_stencils.argtypes = [P, dp, dp, dp, dp, dp]
        lib.o3_init.argtypes = [P, dp, dp]
        lib.o3_run.argtypes = [P, dp, dp, dp, C.c_int64]
        lib.o3_fields.argtypes = [P, dp, dp] + [dp] * 8
        lib.o3_mass.argtypes = [P, dp]
        lib.o3_mass.restype = C.c_double
        _lib = lib
    return _lib


def velocities():
    """(ex, ey, ez, w) of the oracle's D3Q19 set."""
    ex, ey, ez = (np.empty(19, np.int32) for _ in range(3))
    w = np.empty(19)
    load_library().o3_velocities(ex, ey, ez, w)
    return ex, ey, ez, w


def feq(rho, ux, uy, uz):
    out = np.empty(19)
    load_library().o3_feq(float(rho), float(ux), float(uy), float(uz), out)
    return out


@dataclass
class Params3:
    nx: int
    ny: int
    nz: int
    eos: int
    a: float
    b: float
    R: float
    T: float
    alpha: float
    tau: float
    kappa: float

    @staticmethod
    def from_reduced(nx, ny, nz, eos, a, b, Tr, tau, kappa, R=1.0, omega=0.0) -> "Params3":
        fl = thermo.fluid_at(eos, a, b, R, Tr, omega)
        return Params3(nx, ny, nz, eos, a, b, R, fl.T, fl.alpha, tau, kappa)

    def c(self) -> _Params:
        return _Params(self.nx, self.ny, self.nz, self.eos, self.a, self.b, self.R, self.T, self.alpha,
                       self.tau, self.kappa)


def stencils(p: Params3, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    out = [np.empty_like(phi) for _ in range(4)]
    load_library().o3_stencils(C.byref(p.c()), phi, *out)
    return out


class Oracle3:
    """Driver of the D3Q19 oracle; f is [19][nz][ny][nx] (post-streaming, time t)."""

    def __init__(self, p: Params3, rho0):
        self.p, self._cp, self.lib = p, p.c(), load_library()
        shape = (p.nz, p.ny, p.nx)
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        assert rho0.shape == shape
        self.f = np.zeros((19,) + shape)
        self.fbuf = np.zeros_like(self.f)
        self.work = np.zeros((9,) + shape)
        self.lib.o3_init(C.byref(self._cp), rho0, self.f)
        self.steps = 0

    def step(self, n: int = 1):
        if n > 0:
            self.lib.o3_run(C.byref(self._cp), self.f, self.fbuf, self.work, int(n))
            self.steps += n

    def fields(self):
        shape = (self.p.nz, self.p.ny, self.p.nx)
        keys = ("rho", "vx", "vy", "vz", "mu", "Fx", "Fy", "Fz")
        out = {k: np.empty(shape) for k in keys}
        self.lib.o3_fields(C.byref(self._cp), self.f, self.work, *[out[k] for k in keys])
        return out

    def mass(self) -> float:
        return float(self.lib.o3_mass(C.byref(self._cp), self.f))

    def timed_steps(self, n: int) -> float:
        t0 = time.perf_counter()
        self.step(n)
        return time.perf_counter() - t0
