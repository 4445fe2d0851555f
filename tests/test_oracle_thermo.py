"""Pins of the oracle's thermodynamics (Sec. III) against closed forms and identities.

None of these tests retypes a formula of the oracle: each checks a relation the
paper or the mathematics fixes (Eq 3, Eq 15, mu = psi', Gibbs-Duhem, the
second virial coefficient, textbook critical constants, the equal-area rule).
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import thermo
from oracle.lattice import OracleParams, eos_c

# (eos, a, b, omega, Tr) of the paper's parameter set (Sec. III, last paragraph)
CASES = [
    (thermo.VDW, 9 / 49, 2 / 21, 0.0, 0.85),
    (thermo.CS, 1.0, 4.0, 0.0, 0.7),
    (thermo.PR, 2 / 49, 2 / 21, 0.344, 0.8),
    (thermo.PR, 2 / 49, 2 / 21, 0.011, 0.8),
    (thermo.RKS, 2 / 49, 2 / 21, 0.344, 0.8),
    (thermo.RK, 2 / 49, 2 / 21, 0.0, 0.8),
]


def _fluid(case):
    eos, a, b, om, Tr = case
    return thermo.fluid_at(eos, a, b, 1.0, Tr, om)


def _densities(fl, n=64):
    hi = thermo.rho_max(fl.eos, fl.b)
    return np.linspace(0.002 * hi, 0.95 * hi, n)


@pytest.mark.parametrize("case", CASES)
def test_eq3_pressure_from_free_energy(case):
    """Eq 3: p0 = rho psi' - psi, with psi' the printed chemical potential."""
    fl = _fluid(case)
    r = _densities(fl)
    lhs = thermo.p0(fl, r)
    rhs = r * thermo.mu_b(fl, r) - thermo.psi(fl, r)
    scale = np.abs(r * thermo.mu_b(fl, r)) + np.abs(thermo.psi(fl, r))
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-13


@pytest.mark.parametrize("case", CASES)
def test_mu_is_derivative_of_psi(case):
    """Eq 8 bulk term: mu_b = d psi / d rho (complex-step derivative of Eqs 17/20/23/26)."""
    fl = _fluid(case)
    r = _densities(fl)
    d = thermo.dcs(lambda z: thermo.psi(fl, z), r)
    assert np.max(np.abs(d - thermo.mu_b(fl, r)) / (1 + np.abs(d))) < 1e-13


@pytest.mark.parametrize("case", CASES)
def test_gibbs_duhem(case):
    """rho dmu_b/drho = dp0/drho (follows from Eq 3; ties the printed p0 to the printed mu)."""
    fl = _fluid(case)
    r = _densities(fl)
    lhs = r * thermo.dcs(lambda z: thermo.mu_b(fl, z), r)
    rhs = thermo.dcs(lambda z: thermo.p0(fl, z), r)
    assert np.max(np.abs(lhs - rhs) / (1 + np.abs(rhs))) < 1e-12


@pytest.mark.parametrize("case", CASES)
def test_eq15_free_energy_integral(case):
    """Eq 15: psi/rho changes by the integral of p0/rho^2 between two densities."""
    fl = _fluid(case)
    hi = thermo.rho_max(fl.eos, fl.b)
    r1, r2 = 0.05 * hi, 0.8 * hi
    val, _ = integrate.quad(lambda z: float(thermo.p0(fl, z)) / z**2, r1, r2,
                            epsabs=0, epsrel=1e-13, limit=200)
    d = float(thermo.psi(fl, r2)) / r2 - float(thermo.psi(fl, r1)) / r1
    assert abs(val - d) < 1e-10 * (1 + abs(d))


@pytest.mark.parametrize("case", CASES)
def test_second_virial_coefficient(case):
    """Dilute limit of every EOS: p0/(rho R T) = 1 + B2 rho + O(rho^2), with
    B2 = b - a alpha/(RT) for VdW, RK, PR and CS (CS: 4 * (b/4) from 1 + 4 eta)."""
    fl = _fluid(case)
    B2 = fl.b - fl.a * fl.alpha / (fl.R * fl.T)
    hs = [1e-5 / fl.b, 2e-5 / fl.b]
    est = [(float(thermo.p0(fl, h)) / (h * fl.R * fl.T) - 1.0) / h for h in hs]
    rich = 2 * est[0] - est[1]  # Richardson: removes the O(rho) term
    assert abs(rich - B2) < 1e-6 * abs(B2)


@pytest.mark.parametrize("case", CASES)
def test_c_oracle_eos_matches_python(case):
    """The C step's EOS is the same function as the Python one (both oracle copies)."""
    fl = _fluid(case)
    p = OracleParams(8, 8, fl.eos, fl.a, fl.b, fl.R, fl.T, fl.alpha, 1.0, 0.01)
    r = _densities(fl, 200)
    psi_c, p0_c, mu_c = eos_c(p, r)
    for c, py in ((psi_c, thermo.psi(fl, r)), (p0_c, thermo.p0(fl, r)), (mu_c, thermo.mu_b(fl, r))):
        assert np.max(np.abs(c - py) / (1 + np.abs(py))) < 1e-13


def test_vdw_critical_point_closed_form():
    a, b = 9 / 49, 2 / 21
    Tc, rc, pc = thermo.critical_point(thermo.VDW, a, b, 1.0)
    assert abs(Tc - 8 * a / (27 * b)) < 1e-13
    assert abs(rc - 1 / (3 * b)) < 1e-6 * rc      # flat maximum: rho_c to ~sqrt(eps)
    assert abs(pc - a / (27 * b * b)) < 1e-12
    assert abs(Tc - 4 / 7) < 1e-13


def test_rk_family_critical_constants():
    """RKS at Tc has alpha = 1, i.e. plain RK with alpha = 1: Omega_b/Omega_a = 3(2^(1/3)-1)^2
    and Z_c = 1/3 (textbook closed forms of the Redlich-Kwong cubic)."""
    a, b = 2 / 49, 2 / 21
    Tc, rc, pc = thermo.critical_point(thermo.RKS, a, b, 1.0)
    c = 2 ** (1 / 3) - 1
    assert abs(Tc * b / a - 3 * c * c) < 1e-12
    assert abs(pc / (rc * Tc) - 1 / 3) < 1e-7


def test_pr_and_cs_textbook_critical_constants():
    """PR: Tc b R/a = Omega_b/Omega_a = 0.0777960739/0.457235529, Z_c = 0.3074013;
    CS: Tc b R/a = 0.37731, Z_c = 0.35896 (textbook critical constants)."""
    Tc, rc, pc = thermo.critical_point(thermo.PR, 2 / 49, 2 / 21, 1.0)
    assert abs(Tc * (2 / 21) / (2 / 49) - 0.0777960739 / 0.457235529) < 2e-9
    assert abs(pc / (rc * Tc) - 0.3074013) < 1e-6
    Tc, rc, pc = thermo.critical_point(thermo.CS, 1.0, 4.0, 1.0)
    assert abs(Tc * 4.0 - 0.37731) < 1e-5
    assert abs(pc / (rc * Tc) - 0.35896) < 1e-5


@pytest.mark.parametrize("eos,a,b", [(thermo.VDW, 9 / 49, 2 / 21), (thermo.CS, 1.0, 4.0),
                                     (thermo.PR, 2 / 49, 2 / 21), (thermo.RKS, 2 / 49, 2 / 21),
                                     (thermo.RK, 2 / 49, 2 / 21)])
def test_critical_point_is_inflection(eos, a, b):
    """At (Tc, rho_c): dp0/drho = 0 and d2p0/drho2 = 0 (finite differences of the C EOS)."""
    Tc, rc, pc = thermo.critical_point(eos, a, b, 1.0)
    alpha = 1 / math.sqrt(Tc) if eos == thermo.RK else 1.0
    p = OracleParams(8, 8, eos, a, b, 1.0, Tc, alpha, 1.0, 0.01)
    h = 1e-3 * rc
    r = np.array([rc - 2 * h, rc - h, rc, rc + h, rc + 2 * h])
    _, pp, _ = eos_c(p, r)
    d1 = (pp[0] - 8 * pp[1] + 8 * pp[3] - pp[4]) / (12 * h)
    d2 = (-pp[0] + 16 * pp[1] - 30 * pp[2] + 16 * pp[3] - pp[4]) / (12 * h * h)
    scale = pc / rc
    assert abs(d1) < 1e-6 * scale
    assert abs(d2) < 1e-4 * scale / rc


@pytest.mark.parametrize("case", CASES)
def test_maxwell_equal_area(case):
    """Sec. III benchmark: equal pressure, equal mu_b, and the equal-area rule
    int_{v_l}^{v_g} p0 dv = p* (v_g - v_l) (checked with p0 only, by quadrature)."""
    fl = _fluid(case)
    rg, rl, ps, ms = thermo.maxwell(fl)
    assert rg < rl
    assert abs(float(thermo.p0(fl, rl)) - ps) < 1e-13 * (1 + abs(ps))
    assert abs(float(thermo.mu_b(fl, rl)) - ms) < 1e-12 * (1 + abs(ms))
    vg, vl = 1 / rg, 1 / rl
    area, _ = integrate.quad(lambda v: float(thermo.p0(fl, 1 / v)), vl, vg, epsabs=0,
                             epsrel=1e-13, limit=500, points=[1 / s for s in thermo.spinodal(fl)])
    assert abs(area - ps * (vg - vl)) < 1e-9 * abs(ps * (vg - vl))


def test_maxwell_corresponding_states():
    """VdW: reduced coexistence densities depend on Tr only, not on (a, b)."""
    out = []
    for a, b in ((9 / 49, 2 / 21), (1.0, 1.0 / 3.0), (0.5, 0.25)):
        Tc, rc, _ = thermo.critical_point(thermo.VDW, a, b, 1.0)
        rg, rl, _, _ = thermo.maxwell(thermo.fluid_at(thermo.VDW, a, b, 1.0, 0.85))
        out.append((rg * 3 * b, rl * 3 * b))   # rho_c = 1/(3b) exactly
    for o in out[1:]:
        assert abs(o[0] - out[0][0]) < 1e-11 and abs(o[1] - out[0][1]) < 1e-11


def test_pr_density_ratio_above_100():
    """Sec. III: PR coexistence reaches liquid/gas ratios above 100 for water and
    methane (the figure's temperature range is not printed; Tr = 0.6 is inside it)."""
    for om in (0.344, 0.011):
        rg, rl, _, _ = thermo.maxwell(thermo.fluid_at(thermo.PR, 2 / 49, 2 / 21, 1.0, 0.6, om))
        assert rl / rg > 100


def test_eq11_divergence_identity():
    """Eq 11: d/dx P_xx (Eq 9, 1-D) equals rho d mu/dx (Eq 8) on a smooth profile,
    with 6th-order central differences of the oracle's own psi, p0 and mu_b."""
    fl = _fluid(CASES[2])
    kappa = 0.01
    rg, rl, _, _ = thermo.maxwell(fl)
    h = 1e-3
    x = np.arange(-6, 6, h)
    rho = 0.5 * (rl + rg) + 0.5 * (rl - rg) * np.tanh(x / 1.5)

    def d(u):  # 6th-order first derivative on the interior
        return (-u[:-6] + 9 * u[1:-5] - 45 * u[2:-4] + 45 * u[4:-2] - 9 * u[5:-1] + u[6:]) / (60 * h)

    r1 = d(rho)
    r2 = d(r1)
    core = rho[6:-6]
    r1c = r1[3:-3]
    mu = thermo.mu_b(fl, core) - kappa * r2
    pxx = thermo.p0(fl, core) - kappa * core * r2 - kappa / 2 * r1c**2 + kappa * r1c**2
    lhs = d(pxx)
    rhs = core[3:-3] * d(mu)
    inner = slice(20, -20)
    assert np.max(np.abs(lhs[inner] - rhs[inner])) < 1e-6 * np.max(np.abs(rhs[inner]))


# --------------------------------------------------------------------------- surface tension
@pytest.mark.parametrize("case", [CASES[0], CASES[1], CASES[2], CASES[4]])
def test_surface_tension_from_the_relaxed_planar_profile(case):
    """sigma of Eq 1's functional, checked without its first integral: the planar
    profile is solved as the boundary-value problem that Eq 8 with a uniform chemical
    potential states, kappa rho'' = mu_b(rho) - mu* with rho -> rho_g, rho_l at the two
    ends, and sigma is then computed two ways on that profile: as the gradient energy
    int kappa rho'^2 dx and as the excess grand potential
    int (psi - mu* rho + p* + kappa rho'^2 / 2) dx.  The oracle's quadrature
    int sqrt(2 kappa W) d rho must equal both (a dropped 2, a dropped p* or a wrong
    mu* would not)."""
    kappa = 0.01
    fl = _fluid(case)
    rg, rl, ps, ms = thermo.maxwell(fl)
    sigma = thermo.surface_tension(fl, kappa, rg, rl, ms, ps)
    dmu = lambda r: float(thermo.dcs(lambda z: thermo.mu_b(fl, z), r))   # noqa: E731
    ell = math.sqrt(kappa / min(dmu(rl), dmu(rg)))   # the longer decay length of the two phases
    L = 40.0 * ell
    x = np.linspace(-L, L, 801)
    guess = np.vstack([0.5 * (rl + rg) + 0.5 * (rl - rg) * np.tanh(x / (4.0 * ell)), np.zeros_like(x)])
    guess[1] = np.gradient(guess[0], x)
    with np.errstate(invalid="ignore", divide="ignore"):
        sol = integrate.solve_bvp(lambda t, y: np.vstack([y[1], (thermo.mu_b(fl, y[0]) - ms) / kappa]),
                                  lambda ya, yb: np.array([ya[0] - rg, yb[0] - rl]), x, guess, tol=1e-6,
                                  max_nodes=50000)
    xs = np.linspace(-L, L, 200001)
    rho, drho = sol.sol(xs)
    assert np.all(np.diff(rho) > -1e-9 * rl)          # one monotone interface
    gradient_energy = np.trapezoid(kappa * drho**2, xs)
    grand_potential = np.trapezoid(thermo.psi(fl, rho) - ms * rho + ps + 0.5 * kappa * drho**2, xs)
    assert gradient_energy == pytest.approx(sigma, rel=2e-6)
    assert grand_potential == pytest.approx(sigma, rel=2e-6)


def test_surface_tension_scales_as_sqrt_kappa():
    """W does not depend on kappa, so sigma = int sqrt(2 kappa W) d rho is exactly
    proportional to sqrt(kappa)."""
    fl = _fluid(CASES[2])
    rg, rl, ps, ms = thermo.maxwell(fl)
    s1 = thermo.surface_tension(fl, 0.01, rg, rl, ms, ps)
    s4 = thermo.surface_tension(fl, 0.04, rg, rl, ms, ps)
    assert s4 / s1 == pytest.approx(2.0, rel=1e-9)
