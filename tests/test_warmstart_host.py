"""Host-side pieces of the warm start (CPU): phase maps, the sessile cap, mass
matching, the read-out of a predicted field and the calibration interpolation.
They call only the library's host FP64 tools (coexistence, contact angle)."""
import numpy as np
import pytest

lbm = pytest.importorskip("paper_1611_00907_amd.lbm")
from paper_1611_00907_amd import warmstart as W  # noqa: E402


def _spec(eos=lbm.LBM_EOS_PR, Tr=0.8, side=128, theta0=90.0):
    return W.CaseSpec(eos, Tr, 0.5, 0.0, side, theta0)


def _fluid_mass(rho):
    return float(rho[1:-1].sum())


@pytest.mark.parametrize("eos,Tr", [(lbm.LBM_EOS_PR, 0.8), (lbm.LBM_EOS_CS, 0.65)])
def test_phase_density_inverse(eos, Tr):
    s = _spec(eos, Tr)
    rg, rl, _, _ = s.coexistence()
    rho = np.linspace(0.5 * rg, 1.1 * rl, 50)
    assert np.allclose(W.density(s, W.phase(s, rho)), rho, rtol=1e-12)
    assert abs(W.phase(s, rg)) < 1e-12 and abs(W.phase(s, rl) - 1) < 1e-12


@pytest.mark.parametrize("theta", [45.0, 70.0, 90.0, 110.0, 150.0])
def test_cap_holds_the_cold_mass_and_its_angle(theta):
    """The cap has the cold start's fluid-row mass (the method conserves mass) and
    the requested contact angle by the Sec. V measure."""
    s = _spec()
    rg, rl, _, _ = s.coexistence()
    for levels in ((None, None), (1.01 * rl, 1.5 * rg)):
        cap = W.cap_field(s, theta, *levels)
        assert abs(_fluid_mass(cap) / _fluid_mass(W.initial_density(s)) - 1) < 1e-12
        assert abs(W.measure_angle(cap) - theta) < 0.3


def test_bulk_phases_and_read_prediction():
    s = _spec()
    rg, rl, _, _ = s.coexistence()
    cap = W.cap_field(s, 120.0, 1.01 * rl, 1.3 * rg)
    th, pl, pg = W.read_prediction(s, W.phase(s, cap))
    assert abs(th - 120.0) < 0.5
    assert abs(pg / (1.3 * rg) - 1) < 1e-6
    assert abs(pl / rl - 1) < 0.02          # mass matching moves the liquid level slightly


def test_warm_field_keeps_mass_and_angle():
    s = _spec()
    rg, rl, _, _ = s.coexistence()
    pred = W.phase(s, W.cap_field(s, 75.0, 1.005 * rl, 1.1 * rg))
    warm = W.warm_field(s, pred)
    assert abs(_fluid_mass(warm) / _fluid_mass(W.initial_density(s)) - 1) < 1e-12
    assert abs(W.measure_angle(warm) - 75.0) < 0.5
    # a prediction with no drop falls back to the cold start
    assert np.array_equal(W.warm_field(s, np.zeros((128, 128))), W.initial_density(s))


def test_theta_guess_interpolates_the_sweeps():
    t = W.Calibration()
    t.sweeps[(1, 0.7)] = (np.array([-0.1, 0.0, 0.1]), np.array([30.0, 90.0, 150.0]))
    t.sweeps[(1, 0.8)] = (np.array([-0.2, 0.0, 0.2]), np.array([30.0, 90.0, 150.0]))
    assert W.theta_guess(t, 1, 0.7, 0.05) == pytest.approx(120.0)
    assert W.theta_guess(t, 1, 0.75, 0.1) == pytest.approx(0.5 * (150.0 + 120.0))
    assert W.theta_guess(t, 2, 0.75, 0.1) == 90.0      # no sweeps for that EOS
