"""Seeded synthetic inputs (initial density fields and per-case draws).

This module holds no arithmetic of the lattice Boltzmann method: it only draws
random numbers and lays out initial density fields.  The coexistence densities
it places inside and outside a drop are arguments, computed by whoever calls.
Both the GPU library's callers and the CPU oracle's tests take their inputs
from here, so that both sides start from bit-identical fields.

Random numbers come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15,
then two xor-shift-multiply rounds; a double in [0, 1) is (z >> 11) * 2^-53.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """n consecutive SplitMix64 outputs (uint64) starting from ``seed``."""
    with np.errstate(over="ignore"):
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, n: int) -> np.ndarray:
    """n doubles uniform on [0, 1)."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm(seed: int, shape) -> np.ndarray:
    """Uniform on [-1, 1) in row-major order of ``shape``."""
    n = int(np.prod(shape))
    return (2.0 * uniform(seed, n) - 1.0).reshape(shape)


def tanh_drop(nx: int, ny: int, rho_in: float, rho_out: float, radius: float, cx: float,
              cy: float, width: float = 4.0) -> np.ndarray:
    """Circular drop: rho_in inside radius, rho_out outside, tanh interface of
    the given width (distance between the 12 % and 88 % points)."""
    y = np.arange(ny, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * np.tanh(2.0 * (r - radius) / width)


def planar_slab(nx: int, ny: int, rho_in: float, rho_out: float, half_width: float,
                width: float = 4.0) -> np.ndarray:
    """Slab of rho_in, |y - ny/2| < half_width, in rho_out (periodic in x and y)."""
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    d = np.abs(y - ny / 2.0)
    return 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * np.tanh(2.0 * (d - half_width) / width)


def sessile_drop(nx: int, ny: int, rho_in: float, rho_out: float, radius: float,
                 base_row: int = 1, width: float = 4.0) -> np.ndarray:
    """Semicircular drop centred on (nx/2, base_row) sitting on a wall below base_row."""
    return tanh_drop(nx, ny, rho_in, rho_out, radius, nx / 2.0, float(base_row), width)


def with_additive_noise(field: np.ndarray, amplitude: float, seed: int) -> np.ndarray:
    """field + amplitude * U(-1, 1), one draw per node in row-major order."""
    return field + amplitude * uniform_pm(seed, field.shape)


def with_relative_noise(field: np.ndarray, rel: float, seed: int) -> np.ndarray:
    """field * (1 + rel * U(-1, 1)), one draw per node in row-major order."""
    return field * (1.0 + rel * uniform_pm(seed, field.shape))


def draw_uniform(seed: int, lo: float, hi: float, n: int) -> np.ndarray:
    """n values uniform on [lo, hi) (per-case parameters of batched runs)."""
    return lo + (hi - lo) * uniform(seed, n)
