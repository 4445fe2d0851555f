"""GPU: batched persistent launches, graph replay and the tile tuner.

A case inside a batch runs the same per-tile code as a single lattice, so its
state must equal the single-lattice run bit for bit (same tile height); FP64
batches must also match the oracle within 1e-10."""
import numpy as np
import pytest

from cases import C1, Case, rel_err
from oracle import thermo
from oracle.lattice import CPWALL, NEUTRAL, PERIODIC

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_1611_00907_amd.lbm")


def _cases(n=6, prec=None):
    """Uneven sizes, both EOS of the batching configuration, walls and wall mu."""
    out = []
    for k in range(n):
        side = [96, 130, 64, 200, 77, 150][k % 6]
        eos = thermo.CS if k % 2 else thermo.PR
        Tr = [0.8, 0.85, 0.75, 0.9, 0.8, 0.7][k % 6]
        c = Case(side, side - 8 * (k % 3), eos, Tr, 1.3, omega=0.344 if eos == thermo.PR else 0.0,
                 bottom=CPWALL, top=NEUTRAL, drop="sessile", radius=0.25 * side, noise=1e-4, seed=40 + k)
        mu_sat = c.coexistence()[3]
        c.mu_w_bottom = mu_sat + (0.02 if eos == thermo.PR else 0.005) * (k - 2)
        out.append(c)
    return out


def _single(case, prec, tile_y=16):
    lat = lbm.Lattice(case.lbm_params(prec), case.rho0())
    lat.set_tile(tile_y)
    if case.bottom == CPWALL:
        lat.set_wall_mu(0, case.mu_w_bottom)
    return lat


def _batch(cases, prec):
    return lbm.Batch([c.lbm_params(prec) for c in cases], [c.rho0() for c in cases],
                     mu_w_bottom=[float(c.mu_w_bottom) for c in cases])


def test_batch_equals_single_runs_fp32():
    cases = _cases()
    b = _batch(cases, lbm.LBM_F32)
    b.step(150)
    for i, c in enumerate(cases):
        lat = _single(c, lbm.LBM_F32)
        lat.step(150)
        f, _ = lat.get_state()
        assert np.array_equal(b.get_state(i), f), "case %d" % i


def test_batch_beyond_the_caches_equals_single_runs():
    """A batch whose distributions exceed the 256 MB Infinity Cache stores them with
    the non-temporal hint (one 2048^2 case brings it to 0.3 GB); every case must still
    equal its single run bit for bit (the 2048^2 single lattice takes the hint as well,
    the small ones do not)."""
    big = Case(2048, 2048, thermo.PR, 0.8, 1.3, omega=0.344, bottom=CPWALL, top=NEUTRAL, drop="sessile",
               radius=400.0, noise=1e-4, seed=77)
    big.mu_w_bottom = big.coexistence()[3] + 0.01
    cases = _cases(3) + [big]
    b = _batch(cases, lbm.LBM_F32)
    b.step(24)
    for i, c in enumerate(cases):
        lat = _single(c, lbm.LBM_F32)
        lat.step(24)
        f, _ = lat.get_state()
        lat.close()
        assert np.array_equal(b.get_state(i), f), "case %d" % i
    b.close()


@pytest.mark.parametrize("bpc", [-1, 0, 1, 2])
def test_batch_schedules_agree(bpc):
    """Every grid of the batched launch (k workgroups per CU, as many as fit, one
    workgroup per (case, tile) entry) gives the single runs' FP32 result bit for bit."""
    cases = _cases(4)
    b = _batch(cases, lbm.LBM_F32)
    b.set_schedule(16, bpc)
    b.step(40)
    for i, c in enumerate(cases):
        lat = _single(c, lbm.LBM_F32)
        lat.step(40)
        f, _ = lat.get_state()
        assert np.array_equal(b.get_state(i), f), "case %d" % i


@pytest.mark.parametrize("code", [12816, 25608])
@pytest.mark.parametrize("bpc", [-1, 0])
def test_batch_wide_tiles_agree(code, bpc):
    """The wide tiles (128 x 16, 256 x 8) in a batch give the single runs' FP32
    result with the same shape bit for bit, and their monitors sum the same mass."""
    cases = _cases(4)
    b = _batch(cases, lbm.LBM_F32)
    b.set_schedule(code, bpc)
    b.run(40, check_every=20, window=1, tol=0.0)
    st = b.status()
    for i, c in enumerate(cases):
        lat = _single(c, lbm.LBM_F32, tile_y=code)
        lat.step(40)
        f, _ = lat.get_state()
        assert np.array_equal(b.get_state(i), f), "case %d" % i
        rho = lat.fields()["rho"][1:-1]
        assert abs(st["mass"][i] - rho.sum()) < 1e-9 * rho.sum(), i


@pytest.mark.parametrize("bpc", [-1, 0])
def test_batch_mixed_shapes_agree(bpc):
    """The schedule with a tile shape per size class (code 1: 64 x 32 tiles below 256
    columns, 256 x 8 from there) gives each case the single run's FP32 result with its
    class's shape bit for bit, and the monitors (which decode each case's shape) the
    same mass."""
    wide = Case(300, 260, thermo.PR, 0.8, 1.3, omega=0.344, bottom=CPWALL, top=NEUTRAL, drop="sessile",
                radius=70.0, noise=1e-4, seed=61)
    wide.mu_w_bottom = wide.coexistence()[3] - 0.03
    cases = _cases(3) + [wide]
    b = _batch(cases, lbm.LBM_F32)
    b.set_schedule(1, bpc)
    b.run(40, check_every=20, window=1, tol=0.0)
    st = b.status()
    for i, c in enumerate(cases):
        lat = _single(c, lbm.LBM_F32, tile_y=32 if c.nx < 256 else 25608)
        lat.step(40)
        f, _ = lat.get_state()
        assert np.array_equal(b.get_state(i), f), "case %d" % i
        rho = lat.fields()["rho"][1:-1]
        assert abs(st["mass"][i] - rho.sum()) < 1e-9 * rho.sum(), i
        lat.close()
    b.close()


def test_batch_stop_masks_the_listed_cases():
    """lbm_batch_stop: the listed cases keep their state and step count while the
    others advance (and still equal their single runs); a stopped case stays stopped;
    indices outside the batch are rejected."""
    cases = _cases(4)
    b = _batch(cases, lbm.LBM_F32)
    b.step(20)
    held = {i: b.get_state(i) for i in (1, 3)}
    b.stop([1, 3])
    b.stop([3])
    b.step(30)
    st = b.status()
    assert list(st["state"]) == [0, 3, 0, 3]
    assert list(st["steps"]) == [50, 20, 50, 20]
    for i, c in enumerate(cases):
        if i in held:
            assert np.array_equal(b.get_state(i), held[i]), i
        else:
            lat = _single(c, lbm.LBM_F32)
            lat.step(50)
            f, _ = lat.get_state()
            lat.close()
            assert np.array_equal(b.get_state(i), f), i
    for bad in ([4], [-1]):
        with pytest.raises(Exception):
            b.stop(bad)
    b.close()


def test_batch_schedule_rejects_bad_values():
    b = _batch(_cases(1), lbm.LBM_F32)
    for ty, bpc in ((12, 0), (16, -2), (16, 65)):
        with pytest.raises(Exception):
            b.set_schedule(ty, bpc)


@pytest.mark.parametrize("prec,u", [(lbm.LBM_F16DEV, 2.0 ** -11), (lbm.LBM_BF16DEV, 2.0 ** -8)])
def test_batch_matches_single_runs_16bit(prec, u):
    """16-bit deviation storage in a batch against single runs of the same cases.
    The batched kernel inlines the tile step once per EOS, and the compiler contracts
    multiply-adds there differently from the single-lattice kernel: FP16's fine
    rounding then moves a stored value by one rounding now and then (built with
    contraction off, both agree bit for bit; BF16 agrees bit for bit as built).  The
    states agree within a few stored roundings (up to 3.8 u seen after 60 steps)."""
    cases = _cases(3)
    b = _batch(cases, prec)
    b.step(20)
    for i, c in enumerate(cases):
        lat = _single(c, prec)
        lat.step(20)
        f, _ = lat.get_state()
        fb = b.get_state(i)
        err = rel_err(fb, f)
        print("case %d: bit-identical %s, max rel diff %.2e (u = %.1e)" % (i, np.array_equal(fb, f), err, u))
        assert err < 6 * u, (i, err)


def test_batch_fp64_matches_oracle():
    cases = _cases(3)
    b = _batch(cases, lbm.LBM_F64)
    b.step(120)
    for i, c in enumerate(cases):
        ora = c.oracle()
        ora.step(120)
        assert rel_err(b.get_state(i), ora.f) < 1e-10, "case %d" % i


def test_batch_fields_match_single():
    cases = _cases(2)
    b = _batch(cases, lbm.LBM_F64)
    b.step(30)
    for i, c in enumerate(cases):
        lat = _single(c, lbm.LBM_F64)
        lat.step(30)
        fb, fs = b.fields(i), lat.fields()
        for k in ("rho", "vx", "vy", "mu"):
            assert np.array_equal(fb[k], fs[k]), (i, k)


def test_batch_run_masks_converged_and_diverged():
    """A diverging case (the tau = 1 CS drop) is stopped and reported while the
    others go on; converged cases stop advancing; the rest keep running."""
    cases = _cases(4)
    unstable = Case(C1.nx, C1.ny, C1.eos, C1.Tr, C1.tau, drop="circle", radius=25, noise=1e-4, seed=1)
    params = [c.lbm_params(lbm.LBM_F64) for c in cases] + [unstable.lbm_params(lbm.LBM_F64)]
    rhos = [c.rho0() for c in cases] + [unstable.rho0()]
    b = lbm.Batch(params, rhos, mu_w_bottom=[float(c.mu_w_bottom) for c in cases] + [0.0])
    b.run(400, check_every=50, window=1, tol=1e-3)
    st = b.status()
    assert st["state"][4] == lbm.Batch.DIVERGED and st["steps"][4] == 50
    assert st["flags"][4] != 0
    for i in range(4):
        assert st["state"][i] in (lbm.Batch.ACTIVE, lbm.Batch.CONVERGED)
        assert np.isfinite(b.get_state(i)).all()
        if st["state"][i] == lbm.Batch.CONVERGED:
            assert st["residual"][i] < 1e-3
        else:
            assert st["steps"][i] == 400
    # a frozen case keeps its state when the batch advances further
    frozen = b.get_state(4).copy()
    b.step(10)
    assert np.array_equal(np.nan_to_num(b.get_state(4)), np.nan_to_num(frozen))


def test_per_entry_grid_follows_the_masked_list():
    """With one workgroup per (case, tile) entry the grid is resized when a case is
    masked; the run matches the default grid's bit for bit (states, steps, status)."""
    cases = _cases(4)
    unstable = Case(C1.nx, C1.ny, C1.eos, C1.Tr, C1.tau, drop="circle", radius=25, noise=1e-4, seed=1)
    params = [c.lbm_params(lbm.LBM_F64) for c in cases] + [unstable.lbm_params(lbm.LBM_F64)]
    rhos = [c.rho0() for c in cases] + [unstable.rho0()]
    mu_w = [float(c.mu_w_bottom) for c in cases] + [0.0]
    runs = []
    for bpc in (0, -1):
        b = lbm.Batch(params, rhos, mu_w_bottom=mu_w)
        b.set_schedule(16, bpc)
        b.run(300, check_every=50, window=1, tol=1e-3)
        runs.append(b)
    sa, sb = runs[0].status(), runs[1].status()
    assert sb["state"][4] == lbm.Batch.DIVERGED
    assert np.array_equal(sa["state"], sb["state"]) and np.array_equal(sa["steps"], sb["steps"])
    for i in range(4):
        assert np.array_equal(runs[0].get_state(i), runs[1].get_state(i)), "case %d" % i


def test_batch_residual_matches_oracle():
    cases = _cases(2)
    b = _batch(cases, lbm.LBM_F64)
    b.run(100, check_every=100, window=1, tol=0.0)
    st = b.status()
    for i, c in enumerate(cases):
        ora = c.oracle()
        ora.step(99)
        r0 = ora.fields()["rho"]
        ora.step(1)
        r1 = ora.fields()["rho"]
        fluid = ora.p.fluid_mask()
        res = np.max(np.abs(r1 - r0)[fluid])
        assert abs(st["residual"][i] - res) < 1e-10 * res + 1e-15
        assert abs(st["mass"][i] - ora.mass()) < 1e-12 * ora.mass()


def test_batch_tune_keeps_state_and_results():
    cases = _cases(3)
    b = _batch(cases, lbm.LBM_F32)
    b.step(20)
    before = [b.get_state(i) for i in range(3)]
    ty, bpc, ms = b.tune(trial_steps=5)
    assert ty in (1, 8, 16, 32, 12816, 25608) and ms > 0
    for i in range(3):
        assert np.array_equal(b.get_state(i), before[i])
    b.step(30)
    for i, c in enumerate(cases):
        # the mixed schedule (1) runs 64 x 32 tiles below 256 columns, 256 x 8 from there
        lat = _single(c, lbm.LBM_F32, tile_y=ty if ty != 1 else (32 if c.nx < 256 else 25608))
        lat.step(50)
        f, _ = lat.get_state()
        assert np.array_equal(b.get_state(i), f)


@pytest.mark.parametrize("tile_y", [8, 16, 32, 12816, 12832, 25608, 25616, 1000016, 1000032])
def test_tile_heights_agree(tile_y):
    """Every tile height gives the same FP64 result as the oracle (and FP32 results
    identical across heights: the per-node arithmetic does not depend on tiling)."""
    c = _cases(1)[0]
    lat = _single(c, lbm.LBM_F64, tile_y)
    lat.step(60)
    ora = c.oracle()
    ora.step(60)
    f, _ = lat.get_state()
    assert rel_err(f, ora.f) < 1e-10
    a = _single(c, lbm.LBM_F32, tile_y)
    b = _single(c, lbm.LBM_F32, 16)
    a.step(60)
    b.step(60)
    assert np.array_equal(a.get_state()[0], b.get_state()[0])


def test_tuner_keeps_state():
    c = _cases(1)[0]
    lat = _single(c, lbm.LBM_F32)
    lat.step(10)
    f0, s0 = lat.get_state()
    ty, ms = lat.tune(trial_steps=5)
    f1, s1 = lat.get_state()
    assert ty in (8, 16, 32, 12816, 12832, 25608, 25616, 1000016, 1000032) or -8 <= ty <= -1
    assert ms > 0 and s0 == s1
    assert np.array_equal(f0, f1)


@pytest.mark.parametrize("shape", [-1, -3, -4, -8])
def test_marching_matches_tiles_fp32(shape):
    """Column marching computes the same FP32 step as the tiles: the per-node
    arithmetic is the same code, so the states agree to FP32 rounding (the compiler
    may contract the two instances differently) over 200 steps."""
    c = _cases(1)[0]
    a = _single(c, lbm.LBM_F32, 16)
    b = _single(c, lbm.LBM_F32, 16)
    b.set_tile(shape)
    a.step(200)
    b.step(200)
    fa, fb = a.get_state()[0], b.get_state()[0]
    print("marching %d vs tiles: bit-identical %s, max rel diff %.2e" % (shape, np.array_equal(fa, fb),
                                                                      rel_err(fb, fa)))
    assert rel_err(fb, fa) < 2e-5


def test_graph_replay_equals_single_launches():
    """lbm_step(n >= 32) replays captured graphs; one step at a time does not."""
    c = _cases(1)[0]
    a = _single(c, lbm.LBM_F32)
    b = _single(c, lbm.LBM_F32)
    a.step(96)
    for _ in range(96):
        b.step(1)
    assert np.array_equal(a.get_state()[0], b.get_state()[0])
