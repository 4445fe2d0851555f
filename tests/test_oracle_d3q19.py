"""Pins of the D3Q19 oracle: the velocity set's defining moments, Eq 14's moments,
exact stencils on quadratics, exact conservation, symmetry, and -- the strongest
tie -- the projection of a z-invariant run onto the xy plane: summing the D3Q19
populations that share (e_x, e_y) gives the D2Q9 weights, equilibrium, stencils
and collision exactly, so it must reproduce the (independently pinned) 2-D
oracle to rounding."""
import numpy as np
import pytest

from oracle import thermo
from oracle.lattice import OracleLattice, OracleParams
from oracle.lattice3d import Oracle3, Params3, feq, stencils, velocities
from paper_1611_00907_amd import inputs

EX, EY, EZ, W = velocities()
E = np.stack([EX, EY, EZ], axis=1).astype(float)
D2 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def test_velocity_set_moments():
    """19 distinct velocities, closed under reversal; sum w = 1, sum w e = 0,
    sum w e_a e_b = delta / 3, and the fourth moments are isotropic:
    sum w e_a e_b e_c e_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc) / 9."""
    assert len({tuple(e) for e in E.astype(int)}) == 19
    for i in range(1, 19):
        assert np.array_equal(E[i + (1 if i % 2 else -1)], -E[i])
    assert abs(W.sum() - 1) < 1e-15
    assert np.max(np.abs(W @ E)) < 1e-15
    assert np.max(np.abs(np.einsum("i,ia,ib->ab", W, E, E) - np.eye(3) / 3)) < 1e-15
    d = np.eye(3)
    want = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.max(np.abs(np.einsum("i,ia,ib,ic,id->abcd", W, E, E, E, E) - want)) < 1e-15


@pytest.mark.parametrize("rho,u", [(1.0, (0, 0, 0)), (7.2, (0.05, -0.02, 0.03))])
def test_feq_moments(rho, u):
    f = feq(rho, *u)
    u = np.array(u, float)
    assert abs(f.sum() - rho) < 1e-14 * rho
    assert np.max(np.abs(f @ E - rho * u)) < 1e-14 * rho
    assert np.max(np.abs(np.einsum("i,ia,ib->ab", f, E, E) - rho * (np.eye(3) / 3 + np.outer(u, u)))) < 1e-14 * rho


def test_stencils_exact_on_quadratics():
    n = 12
    p = Params3(n, n, n, thermo.VDW, 0.1, 0.1, 1.0, 1.0, 1.0, 1.0, 0.01)
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)
    phi = 0.3 * x * x - 0.2 * x * y + 0.7 * y * y + 0.4 * z * z + 0.1 * y * z + 1.1 * x - 0.4 * z + 2.0
    lap, gx, gy, gz = stencils(p, phi)
    inner = (slice(1, -1),) * 3
    assert np.max(np.abs(lap[inner] - 2 * (0.3 + 0.7 + 0.4))) < 1e-11
    assert np.max(np.abs(gx[inner] - (0.6 * x - 0.2 * y + 1.1)[inner])) < 1e-11
    assert np.max(np.abs(gy[inner] - (-0.2 * x + 1.4 * y + 0.1 * z)[inner])) < 1e-11
    assert np.max(np.abs(gz[inner] - (0.8 * z + 0.1 * y - 0.4)[inner])) < 1e-11


def _pr3(nx, ny, nz, tau=1.3):
    return Params3.from_reduced(nx, ny, nz, thermo.PR, 2 / 49, 2 / 21, 0.8, tau, 0.01, omega=0.344)


def _pr_coex():
    return thermo.maxwell(thermo.fluid_at(thermo.PR, 2 / 49, 2 / 21, 1.0, 0.8, 0.344))


def test_z_invariant_run_projects_onto_the_2d_oracle():
    rg, rl, _, _ = _pr_coex()
    nx, ny, nz = 40, 32, 3
    rho2 = inputs.with_additive_noise(inputs.tanh_drop(nx, ny, rl, rg, 9.0, nx / 2 + 0.3, ny / 2 - 0.2), 1e-3, 5)
    o3 = Oracle3(_pr3(nx, ny, nz), np.broadcast_to(rho2, (nz, ny, nx)).copy())
    o2 = OracleLattice(OracleParams.from_reduced(nx, ny, thermo.PR, 2 / 49, 2 / 21, 0.8, 1.3, 0.01, omega=0.344),
                       rho2)
    o3.step(60)
    o2.step(60)
    proj = np.zeros((9, ny, nx))
    for i in range(19):
        proj[D2.index((int(EX[i]), int(EY[i])))] += o3.f[i, 0]
    assert np.max(np.abs(o3.f - o3.f[:, :1])) == 0.0          # stays z-invariant
    assert np.max(np.abs(proj - o2.f)) < 1e-12 * np.max(o2.f)


def _drop3(n=24):
    rg, rl, _, _ = _pr_coex()
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)
    r = np.sqrt((x - n / 2 - 0.3) ** 2 + (y - n / 2 + 0.2) ** 2 + (z - n / 2 - 0.1) ** 2)
    rho = 0.5 * (rl + rg) - 0.5 * (rl - rg) * np.tanh(2.0 * (r - 6.0) / 4.0)
    return inputs.with_additive_noise(rho, 1e-3, 9)


def test_mass_and_momentum():
    """Mass is exact; a step changes the total momentum by exactly the total force."""
    n = 24
    o = Oracle3(_pr3(n, n, n), _drop3(n))
    o.step(3)
    m0 = o.mass()
    fl = o.fields()
    j0 = o.f.sum(axis=(1, 2, 3)) @ E
    o.step(1)
    j1 = o.f.sum(axis=(1, 2, 3)) @ E
    assert abs(o.mass() - m0) < 1e-13 * m0
    F = np.array([fl["Fx"].sum(), fl["Fy"].sum(), fl["Fz"].sum()])
    assert np.max(np.abs((j1 - j0) - F)) < 1e-11


def test_translation_and_uniform_state():
    n = 24
    a = Oracle3(_pr3(n, n, n), _drop3(n))
    b = Oracle3(_pr3(n, n, n), np.roll(_drop3(n), (2, -3, 5), axis=(0, 1, 2)))
    a.step(20)
    b.step(20)
    assert np.array_equal(np.roll(a.f, (2, -3, 5), axis=(1, 2, 3)), b.f)
    u = Oracle3(_pr3(6, 6, 6), np.full((6, 6, 6), 3.3))
    f0 = u.f.copy()
    u.step(3)
    assert np.max(np.abs(u.f - f0)) < 4e-15 * 3.3


def test_mirror_symmetry_x():
    n = 24
    mirror = [int(np.flatnonzero((EX == -EX[i]) & (EY == EY[i]) & (EZ == EZ[i]))[0]) for i in range(19)]
    rho = _drop3(n)
    a = Oracle3(_pr3(n, n, n), rho)
    b = Oracle3(_pr3(n, n, n), rho[:, :, ::-1].copy())
    a.step(30)
    b.step(30)
    assert np.max(np.abs(a.f - b.f[mirror][..., ::-1])) < 1e-12 * np.max(a.f)
