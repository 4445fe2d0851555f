"""GPU: the D3Q19 step against the D3Q19 oracle, element by element (FP64 within
1e-10 of the largest distribution, FP32 within 2e-5), on boxes that are ragged
against the 64 x 8 columns and the runs of planes of the marching step, for every
EOS, on tiny boxes, and at the benchmark's 256^3 in the launch it times."""
import numpy as np
import pytest

from cases import EOS_AB, rel_err
from oracle import thermo
from oracle.lattice3d import Oracle3, Params3, velocities
from paper_1611_00907_amd import inputs

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_1611_00907_amd.lbm")

# the direction order of lbm.h
ABI = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1), (1, 1, 0), (-1, -1, 0),
       (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1),
       (0, -1, 1)]
LBM_EOS = {thermo.VDW: 0, thermo.CS: 1, thermo.PR: 2, thermo.RKS: 3, thermo.RK: 4}
TR = {thermo.VDW: 0.85, thermo.CS: 0.7, thermo.PR: 0.8, thermo.RKS: 0.8, thermo.RK: 0.8}


def _order():
    ex, ey, ez, _ = velocities()
    ora = [(int(a), int(b), int(c)) for a, b, c in zip(ex, ey, ez)]
    return [ora.index(v) for v in ABI]   # oracle index of each ABI direction


def _drop(nx, ny, nz, eos, seed=3):
    a, b = EOS_AB[eos]
    rg, rl, _, _ = thermo.maxwell(thermo.fluid_at(eos, a, b, 1.0, TR[eos], 0.344))
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    r = np.sqrt((x - nx / 2 - 0.3) ** 2 + (y - ny / 2 + 0.2) ** 2 + (z - nz / 2 - 0.1) ** 2)
    R = 0.3 * min(nx, ny, nz)
    rho = 0.5 * (rl + rg) - 0.5 * (rl - rg) * np.tanh(2.0 * (r - R) / 4.0)
    return inputs.with_additive_noise(rho, 1e-3, seed)


def _pair(nx, ny, nz, eos, prec, tau=1.3):
    a, b = EOS_AB[eos]
    om = 0.344 if eos in (thermo.PR, thermo.RKS) else 0.0
    rho0 = _drop(nx, ny, nz, eos)
    ora = Oracle3(Params3.from_reduced(nx, ny, nz, eos, a, b, TR[eos], tau, 0.01, omega=om), rho0)
    p = lbm.make_params(nx, ny, LBM_EOS[eos], a, b, TR[eos], tau, 0.01, omega=om, prec=prec)
    return lbm.Lattice3(p, nz, rho0), ora


def _err(lat, ora):
    f, _ = lat.get_state()
    return rel_err(f, ora.f[_order()])


@pytest.mark.parametrize("prec,tol", [(lbm.LBM_F64, 1e-10), (lbm.LBM_F32, 2e-5)], ids=["f64", "f32"])
def test_d3q19_pr_drop(prec, tol):
    lat, ora = _pair(70, 22, 19, thermo.PR, prec)       # ragged in x, y and z
    for chunk in (1, 9, 40):
        lat.step(chunk)
        ora.step(chunk)
        err = _err(lat, ora)
        assert err < tol, (chunk, err)
    fg, fo = lat.fields(), ora.fields()
    for k in ("rho", "vx", "vy", "vz", "mu"):
        scale = max(np.max(np.abs(fo[k])), 1e-3 if k.startswith("v") else 1e-300)
        assert np.max(np.abs(fg[k] - fo[k])) / scale < 50 * tol, k
    lat.close()


@pytest.mark.parametrize("eos", [thermo.VDW, thermo.CS, thermo.RKS, thermo.RK])
def test_d3q19_every_eos_f64(eos):
    lat, ora = _pair(40, 12, 12, eos, lbm.LBM_F64)
    lat.step(5)
    ora.step(5)
    assert _err(lat, ora) < 1e-10
    lat.close()


@pytest.mark.parametrize("shape", [(3, 2, 1), (1, 5, 7), (65, 5, 5)])
def test_d3q19_tiny_and_ragged_boxes(shape):
    nx, ny, nz = shape
    rho0 = 3.0 + 0.5 * inputs.uniform_pm(17, (nz, ny, nx))
    p3 = Params3.from_reduced(nx, ny, nz, thermo.VDW, 9 / 49, 2 / 21, 0.85, 1.0, 0.01)
    ora = Oracle3(p3, rho0)
    lat = lbm.Lattice3(lbm.make_params(nx, ny, 0, 9 / 49, 2 / 21, 0.85, 1.0, 0.01, prec=lbm.LBM_F64), nz, rho0)
    lat.step(4)
    ora.step(4)
    assert _err(lat, ora) < 1e-10
    lat.close()


def test_d3q19_rejects_walls_and_16bit():
    p = lbm.make_params(16, 8, 0, 9 / 49, 2 / 21, 0.85, 1.0, 0.01, prec=lbm.LBM_F16DEV)
    with pytest.raises(lbm.LbmError):
        lbm.Lattice3(p, 4, np.full((4, 8, 16), 3.0))
    p = lbm.make_params(16, 8, 0, 9 / 49, 2 / 21, 0.85, 1.0, 0.01, bc_bottom=1, bc_top=2)
    with pytest.raises(lbm.LbmError):
        lbm.Lattice3(p, 4, np.full((4, 8, 16), 3.0))


@pytest.mark.parametrize("n,steps", [(128, 3), (256, 2)])
def test_d3q19_spinodal_f32_full_size(n, steps):
    """The benchmark's spinodal box (VdW, Tr 0.85, rho = 2.6 (1 + 0.01 U)) in FP32:
    at 128^3 (non-temporal stores, 16 runs of 8 planes) and at 256^3 (4 runs of 64
    planes, the launch the benchmark times), every distribution against the oracle."""
    rho0 = inputs.with_relative_noise(np.full((n, n, n), 2.6), 0.01, 3)
    p3 = Params3.from_reduced(n, n, n, thermo.VDW, 9 / 49, 2 / 21, 0.85, 1.0, 0.01)
    ora = Oracle3(p3, rho0)
    lat = lbm.Lattice3(lbm.make_params(n, n, 0, 9 / 49, 2 / 21, 0.85, 1.0, 0.01, prec=lbm.LBM_F32), n, rho0)
    lat.step(steps)
    ora.step(steps)
    assert _err(lat, ora) < 2e-5
    lat.close()
