"""GPU: the learned warm start end to end at a reduced scale (64 x 64 lattices):
calibration of the wetting range, equilibria from the batched solver, training
with the surrogate kernels, and fewer steps to the plain equilibrium contact
angle from the prediction than from the cold start."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_1611_00907_amd.lbm")
from paper_1611_00907_amd import warmstart as W  # noqa: E402


@pytest.fixture(scope="module")
def table():
    return W.calibrate(Tr_grid=(0.7, 0.8, 0.9), side=64, steps=8000)


def test_calibration_orders_wetting_range(table):
    assert len(table) >= 4
    for (eos, Tr), (lo, hi) in table.items():
        assert lo < hi, (eos, Tr, lo, hi)


def test_warm_start_beats_cold_start(table):
    specs = W.draw_cases(72, seed=5, table=table, side=64, Tr_range=(0.7, 0.9))
    rho_eq, state, steps, _ = W.generate(specs, max_steps=20000, check_every=1000, window=500, tol=1e-7)
    ok = [i for i in range(len(specs)) if state[i] != 2 and np.isfinite(rho_eq[i]).all()]
    theta = np.array([W.measure_angle(rho_eq[i]) for i in ok])
    ok = [i for i, t in zip(ok, theta) if 35 < t < 160]
    assert len(ok) >= 40
    train, test = ok[:-8], ok[-8:]
    net = lbm.Surrogate(64, max_batch=16)
    net.set_params(W.he_init(1))
    x = np.stack([W.features(specs[i]) for i in train])
    t = np.stack([W.target(specs[i], rho_eq[i]) for i in train])
    net.set_dataset(x, t)
    losses = net.train(400, 16, 1e-3, seed=2)
    assert losses[-20:].mean() < 0.5 * losses[:10].mean()
    tspecs = [specs[i] for i in test]
    theta_eq = np.array([W.measure_angle(rho_eq[i]) for i in test])
    res = W.evaluate(net, tspecs, theta_eq, tol_deg=0.5, check_every=100, max_steps=20000)
    cold, warm = res["steps_cold"], res["steps_warm"]
    assert (cold >= 0).all() and (warm >= 0).all(), (cold, warm)
    assert np.median(warm) < np.median(cold), (cold, warm)
