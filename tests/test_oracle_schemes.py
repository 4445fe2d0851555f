"""Pins of the oracle's variants of the method that Sec. II names: the force as the
divergence of the full pressure tensor (Eq 5 with P from Eq 9), and the TRT and
MRT collision operators in place of BGK.

Each variant is pinned against what the mathematics fixes: its limits (TRT with
equal even and odd relaxation times, MRT with every rate 1/tau, are BGK), exact
conservation (mass; the momentum change of a collision is the force; the
divergence form of Eq 5 sums to zero over a periodic lattice), the moment basis
of the MRT transform from its defining polynomials, and Eq 11 (the pressure-tensor
force and the chemical-potential force agree up to the stencils' second-order
truncation, which shrinks as the square of the interface width).
"""
import numpy as np
import pytest

from oracle import thermo
from oracle.lattice import (COLLIDE_BGK, COLLIDE_MRT, COLLIDE_TRT, FORCE_CP, FORCE_PTENSOR, OracleLattice,
                            OracleParams, mrt_matrix)
from paper_1611_00907_amd import inputs

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def _params(n=48, tau=1.3, **kw):
    return OracleParams.from_reduced(n, n, thermo.PR, 2 / 49, 2 / 21, 0.8, tau, 0.01, omega=0.344, **kw)


def _drop(n=48, seed=11):
    rg, rl, _, _ = thermo.maxwell(thermo.fluid_at(thermo.PR, 2 / 49, 2 / 21, 1.0, 0.8, 0.344))
    return inputs.with_additive_noise(inputs.tanh_drop(n, n, rl, rg, 12.0, n / 2 + 0.3, n / 2 - 0.2), 1e-3, seed)


def test_mrt_moments_from_their_polynomials():
    """Lallemand and Luo's D2Q9 moments, built from their defining polynomials in
    e_i: 1, e = 3|e|^2 - 4, eps = (9|e|^4 - 21|e|^2 + 8)/2, j = e, q = (3|e|^2 - 5) e,
    p_xx = e_x^2 - e_y^2, p_xy = e_x e_y; the rows are orthogonal."""
    e2 = EX**2 + EY**2
    rows = [np.ones(9), 3 * e2 - 4, (9 * e2**2 - 21 * e2 + 8) / 2, EX, (3 * e2 - 5) * EX, EY, (3 * e2 - 5) * EY,
            EX**2 - EY**2, EX * EY]
    M = mrt_matrix()
    assert np.array_equal(M, np.array(rows, dtype=float))
    G = M @ M.T
    assert np.array_equal(G, np.diag(np.diag(G)))


@pytest.mark.parametrize("force", [FORCE_CP, FORCE_PTENSOR])
def test_trt_with_equal_times_is_bgk(force):
    tau = 1.3
    a = OracleLattice(_params(tau=tau, scheme=force | COLLIDE_BGK), _drop())
    b = OracleLattice(_params(tau=tau, scheme=force | COLLIDE_TRT, trt_lambda=(tau - 0.5) ** 2), _drop())
    a.step(60)
    b.step(60)
    assert np.max(np.abs(a.f - b.f)) < 1e-12 * np.max(a.f)


def test_mrt_with_one_rate_is_bgk():
    tau = 1.3
    a = OracleLattice(_params(tau=tau), _drop())
    b = OracleLattice(_params(tau=tau, scheme=COLLIDE_MRT, s_e=1 / tau, s_eps=1 / tau, s_q=1 / tau), _drop())
    a.step(60)
    b.step(60)
    assert np.max(np.abs(a.f - b.f)) < 1e-12 * np.max(a.f)


@pytest.mark.parametrize("scheme", [COLLIDE_TRT, COLLIDE_MRT, FORCE_PTENSOR, FORCE_PTENSOR | COLLIDE_MRT])
def test_collision_conserves_mass_and_adds_the_force(scheme):
    """Every variant keeps mass exactly and changes the total momentum per step by
    exactly the total force (streaming and the periodic wrap only move momentum)."""
    lat = OracleLattice(_params(scheme=scheme), _drop())
    lat.step(5)
    fl = lat.fields()
    j0 = np.array([(lat.f * EX[:, None, None]).sum(), (lat.f * EY[:, None, None]).sum()])
    m0 = lat.mass()
    lat.step(1)
    j1 = np.array([(lat.f * EX[:, None, None]).sum(), (lat.f * EY[:, None, None]).sum()])
    assert abs(lat.mass() - m0) < 1e-13 * m0
    assert np.max(np.abs((j1 - j0) - np.array([fl["Fx"].sum(), fl["Fy"].sum()]))) < 1e-12


def test_pressure_tensor_force_conserves_total_momentum():
    """Eq 5 is a divergence: on a periodic lattice the discrete divergence of every
    component sums to zero, so the total force vanishes and the total momentum
    stays at its initial value (the chemical-potential force sum_x rho grad(mu)
    does not vanish exactly on the lattice)."""
    lat = OracleLattice(_params(scheme=FORCE_PTENSOR), _drop())
    assert abs(lat.fields()["Fx"].sum()) < 1e-12 and abs(lat.fields()["Fy"].sum()) < 1e-12
    lat.step(200)
    j = np.array([(lat.f * EX[:, None, None]).sum(), (lat.f * EY[:, None, None]).sum()])
    assert np.max(np.abs(j)) < 1e-11
    cp = OracleLattice(_params(), _drop())
    f = cp.fields()
    assert abs(f["Fx"].sum()) + abs(f["Fy"].sum()) > 1e-10


def test_pressure_tensor_force_converges_to_the_chemical_potential_force():
    """Eq 11: div P = rho grad(mu) in the continuum, so the two discrete forces
    differ only by the stencils' truncation, O(h^2 / W^2) relative for an interface
    of width W: doubling the width divides the difference by about four."""
    fl = thermo.fluid_at(thermo.VDW, 9 / 49, 2 / 21, 1.0, 0.85)
    rg, rl, _, _ = thermo.maxwell(fl)
    n = 192
    errs = []
    for width in (6.0, 12.0, 24.0):
        rho = inputs.planar_slab(4, n, rl, rg, n / 4, width)
        f = {}
        for force in (FORCE_CP, FORCE_PTENSOR):
            p = OracleParams.from_reduced(4, n, thermo.VDW, 9 / 49, 2 / 21, 0.85, 1.0, 0.01, scheme=force)
            f[force] = OracleLattice(p, rho).fields()["Fy"][:, 0]
        errs.append(np.linalg.norm(f[FORCE_PTENSOR] - f[FORCE_CP]) / np.linalg.norm(f[FORCE_CP]))
    print("relative difference of the two forces at widths 6, 12, 24:", errs)
    assert errs[0] < 0.2
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


@pytest.mark.parametrize("scheme", [COLLIDE_TRT, COLLIDE_MRT, FORCE_PTENSOR])
def test_uniform_state_is_fixed_point(scheme):
    lat = OracleLattice(_params(12, scheme=scheme), np.full((12, 12), 3.3))
    f0 = lat.f.copy()
    lat.step(3)
    assert np.max(np.abs(lat.f - f0)) < 4e-15 * 3.3


@pytest.mark.parametrize("scheme", [COLLIDE_TRT, COLLIDE_MRT, FORCE_PTENSOR])
def test_translation_invariance(scheme):
    a = OracleLattice(_params(scheme=scheme), _drop())
    b = OracleLattice(_params(scheme=scheme), np.roll(_drop(), (3, -5), axis=(0, 1)))
    a.step(40)
    b.step(40)
    assert np.array_equal(np.roll(a.f, (3, -5), axis=(1, 2)), b.f)


def test_pressure_tensor_needs_a_periodic_lattice():
    from oracle.lattice import CPWALL, NEUTRAL
    p = _params(scheme=FORCE_PTENSOR, bottom=CPWALL, top=NEUTRAL)
    with pytest.raises(ValueError):
        p.c()
