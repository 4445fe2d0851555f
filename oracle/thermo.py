"""Thermodynamics of Sec. III, in numpy FP64 (TEST INFRASTRUCTURE ONLY).

Equations of state, free-energy densities and bulk chemical potentials exactly
as the paper prints them (C = 0 in Eq 15), the temperature functions alpha(T),
the critical point, the Maxwell equal-area coexistence densities used as the
benchmark of Fig. 1, and the planar surface tension of the gradient-squared
functional (Eq 1).

All formulas accept complex arguments so that derivatives can be taken by the
complex-step method (f'(x) = Im f(x + ih) / h, exact to rounding).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import integrate, optimize

VDW, CS, PR, RKS, RK = 0, 1, 2, 3, 4
EOS_NAMES = {"vdw": VDW, "cs": CS, "pr": PR, "rks": RKS, "rk": RK}

_S2 = math.sqrt(2.0)


@dataclass(frozen=True)
class Fluid:
    """EOS id and constants; T is the absolute temperature, alpha = alpha(T)."""

    eos: int
    a: float
    b: float
    R: float
    T: float
    alpha: float = 1.0


def p0(fl: Fluid, rho):
    """Equation of state p0(rho): Eq 16 (VdW), Eq 19 (RK/RKS), Eq 22 (PR), Eq 25 (CS)."""
    a, b, RT, aa = fl.a, fl.b, fl.R * fl.T, fl.a * fl.alpha
    if fl.eos == VDW:
        return rho * RT / (1 - b * rho) - a * rho**2
    if fl.eos in (RK, RKS):
        return rho * RT / (1 - b * rho) - aa * rho**2 / (1 + b * rho)
    if fl.eos == PR:
        return rho * RT / (1 - b * rho) - aa * rho**2 / (1 + 2 * b * rho - b**2 * rho**2)
    if fl.eos == CS:
        q = b * rho / 4
        return rho * RT * (1 + q + q**2 - q**3) / (1 - q) ** 3 - a * rho**2
    raise ValueError(fl.eos)


def psi(fl: Fluid, rho):
    """Free-energy density: Eq 17 (VdW), Eq 20 (RK/RKS), Eq 23 (PR), Eq 26 (CS)."""
    a, b, RT, aa = fl.a, fl.b, fl.R * fl.T, fl.a * fl.alpha
    if fl.eos == VDW:
        return rho * RT * np.log(rho / (1 - b * rho)) - a * rho**2
    if fl.eos in (RK, RKS):
        return RT * rho * np.log(rho / (1 - b * rho)) - aa / b * rho * np.log(1 + b * rho)
    if fl.eos == PR:
        return RT * rho * np.log(rho / (1 - b * rho)) - aa * rho / (2 * _S2 * b) * np.log(
            (_S2 - 1 + b * rho) / (_S2 + 1 - b * rho))
    if fl.eos == CS:
        q = b * rho / 4
        return RT * rho * ((3 - b * rho / 2) / (1 - q) ** 2 + np.log(rho)) - a * rho**2
    raise ValueError(fl.eos)


def mu_b(fl: Fluid, rho):
    """Bulk chemical potential psi'(rho): Eqs 18, 21, 24, 27 without -kappa lap(rho)."""
    a, b, RT, aa = fl.a, fl.b, fl.R * fl.T, fl.a * fl.alpha
    if fl.eos == VDW:
        return RT * (np.log(rho / (1 - b * rho)) + 1 / (1 - b * rho)) - 2 * a * rho
    if fl.eos in (RK, RKS):
        return (RT * np.log(rho / (1 - b * rho)) + RT / (1 - b * rho)
                - aa / b * np.log(1 + b * rho) - aa * rho / (1 + b * rho))
    if fl.eos == PR:
        return (RT * np.log(rho / (1 - b * rho))
                - aa / (2 * _S2 * b) * np.log((_S2 - 1 + b * rho) / (_S2 + 1 - b * rho))
                + RT / (1 - b * rho) - aa * rho / (1 + 2 * b * rho - b**2 * rho**2))
    if fl.eos == CS:
        q = b * rho / 4
        return RT * ((3 - q) / (1 - q) ** 3 + np.log(rho) + 1) - 2 * a * rho
    raise ValueError(fl.eos)


def dcs(fun, x, h=1e-30):
    """Complex-step derivative of a real-analytic function (exact to rounding)."""
    return np.imag(fun(np.asarray(x, dtype=complex) + 1j * h)) / h


def rho_max(eos: int, b: float) -> float:
    """Upper end of the EOS domain: 1/b for the cubic EOSs, 4/b for CS (b rho / 4 < 1)."""
    return 4.0 / b if eos == CS else 1.0 / b


def alpha_of(eos: int, T: float, Tc: float, omega: float) -> float:
    """alpha(T): 1 for VdW/CS; 1/sqrt(T) for RK and the Soave form for RKS (Eq 19 text);
    the PR temperature function after Eq 22."""
    if eos in (VDW, CS):
        return 1.0
    if eos == RK:
        return 1.0 / math.sqrt(T)
    if eos == RKS:
        m = 0.480 + 1.574 * omega - 0.176 * omega**2
        return (1.0 + m * (1.0 - math.sqrt(T / Tc))) ** 2
    if eos == PR:
        m = 0.37464 + 1.54226 * omega - 0.26992 * omega**2
        return (1.0 + m * (1.0 - math.sqrt(T / Tc))) ** 2
    raise ValueError(eos)


def critical_point(eos: int, a: float, b: float, R: float = 1.0):
    """(Tc, rho_c, p_c): the point where dp0/drho = d2p0/drho2 = 0.

    The Soave-type alpha equals 1 at Tc, so for VdW, CS, PR and RKS the EOS is
    p0 = T g(rho) - h(rho); for RK, alpha = T^-1/2 gives p0 = T g - T^-1/2 h.
    On the spinodal dp0/drho = 0 the temperature is T_s(rho) = h'/g' (RK:
    (h'/g')^(2/3)); the critical point is the maximum of T_s.  g' and h' come
    from complex-step derivatives of p0 itself, so no derivative is retyped.
    """
    g = lambda r: p0(Fluid(eos, 0.0, b, R, 1.0, 1.0), r)          # noqa: E731
    h = lambda r: -p0(Fluid(eos, a, b, R, 0.0, 1.0), r)           # noqa: E731

    def t_spin(r):
        ratio = dcs(h, r) / dcs(g, r)
        return ratio ** (2.0 / 3.0) if eos == RK else ratio

    hi = rho_max(eos, b)
    res = optimize.minimize_scalar(lambda r: -t_spin(r), bounds=(1e-6 * hi, 0.999 * hi),
                                   method="bounded", options={"xatol": 1e-14 * hi, "maxiter": 500})
    rc = float(res.x)
    Tc = float(t_spin(rc))
    alpha_c = 1.0 / math.sqrt(Tc) if eos == RK else 1.0
    pc = float(p0(Fluid(eos, a, b, R, Tc, alpha_c), rc))
    return Tc, rc, pc


def fluid_at(eos: int, a: float, b: float, R: float, Tr: float, omega: float = 0.0) -> Fluid:
    """Fluid at reduced temperature Tr = T / Tc (Sec. III, reduced variables)."""
    Tc, _, _ = critical_point(eos, a, b, R)
    T = Tr * Tc
    return Fluid(eos, a, b, R, T, alpha_of(eos, T, Tc, omega))


def spinodal(fl: Fluid):
    """The two roots of dp0/drho = 0 below Tc (gas-side maximum, liquid-side minimum)."""
    dp = lambda r: dcs(lambda z: p0(fl, z), r)                    # noqa: E731
    hi = rho_max(fl.eos, fl.b)
    grid = np.linspace(1e-6 * hi, 0.9999 * hi, 20001)
    vals = dp(grid)
    sgn = np.nonzero(np.diff(np.sign(vals)))[0]
    if len(sgn) < 2:
        raise ValueError("no spinodal: temperature at or above critical")
    s1 = optimize.brentq(dp, grid[sgn[0]], grid[sgn[0] + 1], xtol=1e-16, rtol=1e-15)
    s2 = optimize.brentq(dp, grid[sgn[-1]], grid[sgn[-1] + 1], xtol=1e-16, rtol=1e-15)
    return s1, s2


def maxwell(fl: Fluid):
    """Coexistence (rho_g, rho_l, p*, mu*) from mu_b(rho_g) = mu_b(rho_l) and
    p0(rho_g) = p0(rho_l), the equal-area construction of Sec. III (Fig. 1).

    The pressure p* is bracketed between the spinodal extrema; for each trial
    pressure the gas and liquid branches are inverted by bisection, and p* is
    the root of mu_l(p) - mu_g(p), which falls monotonically (Gibbs-Duhem).  A
    final Newton pass on the 2x2 system polishes both densities.
    """
    s1, s2 = spinodal(fl)
    hi = rho_max(fl.eos, fl.b)
    pmax, pmin = float(p0(fl, s1)), float(p0(fl, s2))
    lo_p = max(pmin, 0.0)

    def branch(p, liquid):
        f = lambda r: float(p0(fl, r)) - p                         # noqa: E731
        if liquid:
            return optimize.brentq(f, s2, hi * (1 - 1e-15), xtol=1e-16, rtol=1e-15)
        return optimize.brentq(f, 1e-300, s1, xtol=1e-300, rtol=1e-15)

    def dmu(p):
        return float(mu_b(fl, branch(p, True)) - mu_b(fl, branch(p, False)))

    span = pmax - lo_p
    pstar = optimize.brentq(dmu, lo_p + 1e-13 * span + 1e-300, pmax - 1e-13 * span,
                            xtol=1e-300, rtol=1e-15)
    rg, rl = branch(pstar, False), branch(pstar, True)
    for _ in range(3):
        F = np.array([float(mu_b(fl, rl) - mu_b(fl, rg)), float(p0(fl, rl) - p0(fl, rg))])
        J = np.array([[-dcs(lambda z: mu_b(fl, z), rg), dcs(lambda z: mu_b(fl, z), rl)],
                      [-dcs(lambda z: p0(fl, z), rg), dcs(lambda z: p0(fl, z), rl)]])
        d = np.linalg.solve(J, -F)
        rg, rl = rg + d[0], rl + d[1]
    return float(rg), float(rl), float(p0(fl, rg)), float(mu_b(fl, rg))


def surface_tension(fl: Fluid, kappa: float, rho_g: float, rho_l: float, mu_star: float,
                    p_star: float) -> float:
    """Planar surface tension of the functional of Eq 1:
    sigma = int_{rho_g}^{rho_l} sqrt(2 kappa W(rho)) d rho with the excess grand
    potential density W = psi - mu* rho + p*  (zero at both bulk phases)."""
    def integrand(r):
        w = float(psi(fl, r)) - mu_star * r + p_star
        return math.sqrt(max(2.0 * kappa * w, 0.0))

    val, _ = integrate.quad(integrand, rho_g, rho_l, epsabs=1e-15, epsrel=1e-12, limit=400)
    return val
