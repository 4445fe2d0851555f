"""GPU parity: the HIP library against the FP64 oracle, element by element.

FP64 storage must match within 1e-10 of the largest distribution; FP32 within
2e-5 (about 300 FP32 ulps of rounding in the chemical potential and force,
carried by a contracting map).  FP16/BF16 deviation storage rounds every stored
value once per step, by at most u |f - w rho_ref| <= u max|f| with the unit
roundoff u = 2^-11 (half) or 2^-8 (bfloat16): the initial state and one step
give two roundings (bound 3u), ten steps at most 12u once the rounding noise
is carried by the contracting map.
"""
import numpy as np
import pytest

from cases import C1, C1_TAU13, C2, C3, C3_512, WALLED_PR, Case, rel_err
from oracle import thermo
from oracle.lattice import CPWALL, NEUTRAL, PERIODIC, OracleLattice, eos_c, stencils_c

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_1611_00907_amd.lbm")


def _gpu(case: Case, prec, monitor_every=0):
    lat = lbm.Lattice(case.lbm_params(prec, monitor_every), case.rho0())
    if case.bottom == CPWALL:
        lat.set_wall_mu(0, case.mu_w_bottom)
    if case.top == CPWALL:
        lat.set_wall_mu(1, case.mu_w_top)
    return lat


def _compare_state(lat, ora, tol):
    f, _ = lat.get_state()
    err = rel_err(f, ora.f)
    assert np.isfinite(f).all()
    assert err < tol, "max |f_gpu - f_oracle| / max |f| = %.3e" % err
    return err


@pytest.mark.parametrize("steps", [1, 5, 11])
def test_fp64_config1_as_written(steps):
    """100^2 CS drop, tau = 1, up to the step before the oracle itself turns
    non-finite (step 12)."""
    lat, ora = _gpu(C1, lbm.LBM_F64), C1.oracle()
    lat.step(steps)
    ora.step(steps)
    _compare_state(lat, ora, 1e-10)


def test_fp64_config1_tau13_5000_steps():
    lat, ora = _gpu(C1_TAU13, lbm.LBM_F64), C1_TAU13.oracle()
    for chunk in (1, 9, 90, 900, 4000):
        lat.step(chunk)
        ora.step(chunk)
        _compare_state(lat, ora, 1e-10)


def test_fp64_walled_pr_2000_steps():
    lat, ora = _gpu(WALLED_PR, lbm.LBM_F64), WALLED_PR.oracle()
    for chunk in (1, 99, 1900):
        lat.step(chunk)
        ora.step(chunk)
        _compare_state(lat, ora, 1e-10)


RAGGED = [(70, 37, False), (130, 45, True), (5, 7, False), (1, 9, False), (3, 4, True), (65, 17, True),
          (200, 3, True), (64, 16, False), (129, 18, False)]


def _ragged_case(nx, ny, walls):
    kw = dict(bottom=CPWALL, top=NEUTRAL, drop="sessile") if walls else dict(drop="circle")
    return Case(nx, ny, thermo.PR, 0.8, 1.3, omega=0.344, radius=max(min(nx, ny) / 3, 0.8), noise=1e-3,
                seed=nx * 1000 + ny, mu_w_bottom=0.25, **kw)


@pytest.mark.parametrize("nx,ny,walls", RAGGED)
def test_fp64_ragged_and_tiny(nx, ny, walls):
    """Sizes that are not multiples of the 64 x 16 tile, smaller than one tile,
    one column wide, or a single fluid row between walls."""
    c = _ragged_case(nx, ny, walls)
    lat, ora = _gpu(c, lbm.LBM_F64), c.oracle()
    lat.step(25)
    ora.step(25)
    _compare_state(lat, ora, 1e-10)


WIDE_CASES = RAGGED + [(300, 70, False), (257, 37, True), (520, 130, True), (129, 33, True)]


@pytest.mark.parametrize("code", [12816, 12832, 25608, 25616, 1000016, 1000032])
@pytest.mark.parametrize("nx,ny,walls", WIDE_CASES)
def test_fp64_wide_tiles(nx, ny, walls, code):
    """Tiles of 128 and 256 columns (shape code 100 * width + height) and the
    64-wide tiles with the ring pulls issued up front (1000000 + height) on ragged,
    tiny and walled lattices."""
    c = _ragged_case(nx, ny, walls)
    lat, ora = _gpu(c, lbm.LBM_F64), c.oracle()
    lat.set_tile(code)
    lat.step(25)
    ora.step(25)
    _compare_state(lat, ora, 1e-10)


# Column marching: strips of at most 252 columns (256 lanes with two halo lanes per
# side), rows split into segments of at least 4 rows that fill k workgroups per CU.
# Cases span several strips and segments with ragged ends, strips one column past
# 252, segments that hold the bottom wall's ghost rows and the top wall, segments
# of 4 rows, and lattices narrower than one strip.
MARCH_CASES = RAGGED + [(300, 70, False), (252, 64, True), (253, 37, True), (520, 130, True),
                        (505, 97, False), (700, 300, False)]


@pytest.mark.parametrize("shape", [-1, -2, -4, -8])
@pytest.mark.parametrize("nx,ny,walls", MARCH_CASES)
def test_fp64_marching_shapes(nx, ny, walls, shape):
    c = _ragged_case(nx, ny, walls)
    lat, ora = _gpu(c, lbm.LBM_F64), c.oracle()
    lat.set_tile(shape)
    lat.step(25)
    ora.step(25)
    _compare_state(lat, ora, 1e-10)


def test_fp64_marching_cp_top_and_every_eos():
    """Per-column surface chemical potentials on both walls, and each EOS, marching."""
    c = Case(300, 40, thermo.PR, 0.8, 1.3, omega=0.344, bottom=CPWALL, top=CPWALL, drop="sessile",
             radius=14, noise=1e-3, seed=9)
    x = np.arange(300)
    c.mu_w_bottom = 0.2 + 0.05 * np.sin(2 * np.pi * x / 300)
    c.mu_w_top = 0.27 + 0.01 * np.cos(2 * np.pi * x / 60)
    lat, ora = _gpu(c, lbm.LBM_F64), c.oracle()
    lat.set_tile(-4)
    lat.step(300)
    ora.step(300)
    _compare_state(lat, ora, 1e-10)
    for eos in (thermo.VDW, thermo.CS, thermo.PR, thermo.RKS, thermo.RK):
        Tr = {thermo.CS: 0.8}.get(eos, 0.85)
        c = Case(260, 48, eos, Tr, 1.3, omega=0.344 if eos in (thermo.PR, thermo.RKS) else 0.0,
                 drop="circle", radius=12, noise=1e-3, seed=eos + 20)
        lat, ora = _gpu(c, lbm.LBM_F64), c.oracle()
        lat.set_tile(-2)
        lat.step(100)
        ora.step(100)
        _compare_state(lat, ora, 1e-10)


def test_fp64_per_node_wall_mu_and_cp_top():
    """Per-column surface chemical potentials on both walls (CP wall on top too)."""
    c = Case(96, 40, thermo.PR, 0.8, 1.3, omega=0.344, bottom=CPWALL, top=CPWALL, drop="sessile",
             radius=14, noise=1e-3, seed=9)
    x = np.arange(96)
    c.mu_w_bottom = 0.2 + 0.05 * np.sin(2 * np.pi * x / 96)
    c.mu_w_top = 0.27 + 0.01 * np.cos(2 * np.pi * x / 48)
    lat, ora = _gpu(c, lbm.LBM_F64), c.oracle()
    lat.step(300)
    ora.step(300)
    _compare_state(lat, ora, 1e-10)


@pytest.mark.parametrize("code", [8, 16, 32, 12816, 12832, 25608, 25616, 1000016, 1000032])
@pytest.mark.parametrize("nx,ny", [(150, 33), (300, 65), (70, 17)])
def test_fp64_cp_walls_every_tile_shape(nx, ny, code):
    """CP walls on both sides with per-column surface chemical potentials, on every
    tile shape.  ny - 1 is a multiple of every tile height, so the top wall is the
    first row of the last tile row and sits in the chemical-potential ring of the
    tiles below it."""
    c = Case(nx, ny, thermo.PR, 0.8, 1.3, omega=0.344, bottom=CPWALL, top=CPWALL, drop="sessile",
             radius=min(nx, ny) / 3, noise=1e-3, seed=nx + ny)
    x = np.arange(nx)
    c.mu_w_bottom = 0.2 + 0.05 * np.sin(2 * np.pi * x / nx)
    c.mu_w_top = 0.27 + 0.01 * np.cos(2 * np.pi * x / 30)
    lat, ora = _gpu(c, lbm.LBM_F64), c.oracle()
    lat.set_tile(code)
    lat.step(40)
    ora.step(40)
    _compare_state(lat, ora, 1e-10)


@pytest.mark.parametrize("eos", [thermo.VDW, thermo.CS, thermo.PR, thermo.RKS, thermo.RK])
def test_fp64_every_eos(eos):
    Tr = {thermo.CS: 0.8}.get(eos, 0.85)
    c = Case(80, 48, eos, Tr, 1.3, omega=0.344 if eos in (thermo.PR, thermo.RKS) else 0.0,
             drop="circle", radius=12, noise=1e-3, seed=eos + 20)
    lat, ora = _gpu(c, lbm.LBM_F64), c.oracle()
    lat.step(200)
    ora.step(200)
    _compare_state(lat, ora, 1e-10)


def test_fp64_fields_and_monitors():
    """Output fields (rho with Eq 28 rows, v = u + F/2rho, mu with wall values) and
    the monitors (mass, max |rho(t) - rho(t-1)|) against the oracle."""
    lat, ora = _gpu(WALLED_PR, lbm.LBM_F64), WALLED_PR.oracle()
    lat.step(49)
    ora.step(49)
    rho_prev = ora.fields()["rho"]
    mon = lat.monitor_step()
    ora.step(1)
    fo = ora.fields()
    fg = lat.fields()
    for k in ("rho", "vx", "vy", "mu"):
        scale = max(np.max(np.abs(fo[k])), 1e-12)
        assert np.max(np.abs(fg[k] - fo[k])) < 1e-10 * scale, k
    fluid = ora.p.fluid_mask()
    assert abs(mon["mass"] - ora.mass()) < 1e-12 * ora.mass()
    res_o = np.max(np.abs(fo["rho"] - rho_prev)[fluid])
    assert abs(mon["residual"] - res_o) < 1e-10 * res_o + 1e-14
    assert mon["step"] == 50 and mon["flags"] == 0


def test_checkpoint_resume_bit_exact():
    for prec in (lbm.LBM_F64, lbm.LBM_F32):
        a = _gpu(WALLED_PR, prec)
        a.step(40)
        f, s = a.get_state()
        a.step(40)
        fa, _ = a.get_state()
        b = _gpu(WALLED_PR, prec)
        b.set_state(f, s)
        b.step(40)
        fb, sb = b.get_state()
        assert sb == 80
        assert np.array_equal(fa, fb)


def test_state_roundtrip_fp64():
    lat = _gpu(C1_TAU13, lbm.LBM_F64)
    f0, _ = lat.get_state()
    lat.set_state(f0, 0)
    f1, _ = lat.get_state()
    assert np.array_equal(f0, f1)


def test_divergence_is_reported():
    """Config 1 as written (tau = 1) blows up; the oracle does too in the same window,
    and the library stops with LBM_EDIVERGED at a monitor point."""
    lat = _gpu(C1, lbm.LBM_F64, monitor_every=10)
    with pytest.raises(lbm.LbmDiverged):
        lat.step(400)
    m = lat.monitors()
    assert m["step"] == 20 and m["flags"] != 0
    ora = C1.oracle()
    ora.step(12)
    assert not np.isfinite(ora.f).all()


def test_zero_steps_is_noop():
    lat = _gpu(WALLED_PR, lbm.LBM_F64)
    f0, _ = lat.get_state()
    lat.step(0)
    f1, s = lat.get_state()
    assert s == 0 and np.array_equal(f0, f1)


@pytest.mark.parametrize("steps", [10, 200])
def test_fp32_walled_pr(steps):
    lat, ora = _gpu(WALLED_PR, lbm.LBM_F32), WALLED_PR.oracle()
    lat.step(steps)
    ora.step(steps)
    _compare_state(lat, ora, 2e-5)


@pytest.mark.parametrize("prec,u", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_reduced_storage_one_and_ten_steps(prec, u):
    """Deviation storage: one stored rounding per value per step."""
    p = {"f16": lbm.LBM_F16DEV, "bf16": lbm.LBM_BF16DEV}[prec]
    lat, ora = _gpu(WALLED_PR, p), WALLED_PR.oracle()
    lat.step(1)
    ora.step(1)
    _compare_state(lat, ora, 3 * u)
    lat.step(9)
    ora.step(9)
    _compare_state(lat, ora, 12 * u)


@pytest.fixture(scope="module")
def spinodal_separated():
    """The 512^2 VdW spinodal lattice (rho = 2.6 (1 + 0.01 U)) after 1500 oracle
    steps: phase-separated, densities from about 1.1 to 6.4, so that deviations from
    w_i 2.6 are as large as on the benchmarked 4096^2 lattice."""
    ora = C3_512.oracle()
    ora.step(1500)
    return ora


@pytest.mark.parametrize("prec,u", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
@pytest.mark.parametrize("start", ["initial", "separated"])
def test_reduced_storage_rho_ref_26(prec, u, start, spinodal_separated):
    """The 16-bit storage the benchmark runs: deviations from w_i 2.6 (rho_ref =
    2.6) on the spinodal lattice, one and ten steps against the oracle, from the
    initial field and from a phase-separated state (set as the checkpoint, one
    rounding), with the bounds of the literal base (3u, 12u of max |f|)."""
    p = {"f16": lbm.LBM_F16DEV, "bf16": lbm.LBM_BF16DEV}[prec]
    lat = lbm.Lattice(C3_512.lbm_params(p, rho_ref=2.6), C3_512.rho0())
    if start == "initial":
        ora = C3_512.oracle()
    else:
        ora = OracleLattice(spinodal_separated.p, C3_512.rho0())
        ora.f[:] = spinodal_separated.f
        lat.set_state(ora.f, 0)
    lat.step(1)
    ora.step(1)
    e1 = _compare_state(lat, ora, 3 * u)
    lat.step(9)
    ora.step(9)
    e10 = _compare_state(lat, ora, 12 * u)
    print("%s rho_ref 2.6 from the %s state: %.2f u after 1 step, %.2f u after 10" % (prec, start, e1 / u,
                                                                                     e10 / u))


@pytest.mark.parametrize("prec,u", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_reduced_storage_every_tile_shape(prec, u):
    """16-bit deviation storage through every tile shape: the per-node arithmetic and
    its roundings do not depend on the tiling, so the stored states agree bit for
    bit; column marching (the same arithmetic, possibly contracted differently by
    the compiler) agrees within a few stored roundings."""
    p = {"f16": lbm.LBM_F16DEV, "bf16": lbm.LBM_BF16DEV}[prec]
    ref = _gpu(WALLED_PR, p)
    ref.set_tile(16)
    ref.step(20)
    f0, _ = ref.get_state()
    for code in (8, 32, 12816, 12832, 25608, 25616, 1000016, 1000032):
        lat = _gpu(WALLED_PR, p)
        lat.set_tile(code)
        lat.step(20)
        f, _ = lat.get_state()
        assert np.array_equal(f, f0), code
    for k in (-2, -4):
        lat = _gpu(WALLED_PR, p)
        lat.set_tile(k)
        lat.step(20)
        f, _ = lat.get_state()
        assert rel_err(f, f0) < 4 * u, (k, rel_err(f, f0))


@pytest.mark.parametrize("shape", [16, 32, 25608, 25616, 1000032, -4])
def test_fp32_full_size_config2(shape):
    """1024 x 1024 wetting case in both launch shapes: every node against the
    oracle after 20 steps."""
    lat, ora = _gpu(C2, lbm.LBM_F32), C2.oracle()
    lat.set_tile(shape)
    lat.step(20)
    ora.step(20)
    _compare_state(lat, ora, 2e-5)


@pytest.mark.parametrize("shape", [16, 25608, 25616, 1000032, -2])
def test_fp32_full_size_4096_sampled(shape):
    """4096^2 spinodal case: after k steps a node depends on the initial field within
    3k nodes, so periodic oracle windows with a 3k margin give exact samples."""
    k = 8
    lat = _gpu(C3, lbm.LBM_F32)
    lat.set_tile(shape)
    rho0 = C3.rho0()
    lat.step(k)
    f, _ = lat.get_state()
    m, w = 3 * k + 2, 32
    for (y0, x0) in ((0, 0), (2000, 3000), (4096 - 32, 4096 - 32), (1234, 77)):
        ys = (np.arange(y0 - m, y0 + w + m)) % 4096
        xs = (np.arange(x0 - m, x0 + w + m)) % 4096
        sub = Case(len(xs), len(ys), C3.eos, C3.Tr, C3.tau, drop="uniform")
        ora = OracleLattice(sub.oracle_params(), rho0[np.ix_(ys, xs)])
        ora.step(k)
        got = f[:, (ys[m:m + w])[:, None], xs[m:m + w][None, :]]
        want = ora.f[:, m:m + w, m:m + w]
        assert rel_err(got, want) < 2e-5


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_band_chemical_potential_of_16bit_storage(prec):
    """Inside the spinodal band the 16-bit formats evaluate psi' in FP64 with a
    Newton-refined reciprocal and a series logarithm, rounded to FP32.  On the
    512^2 spinodal start (every node in the band) the output mu must equal
    psi'(rho) - kappa lap(rho), evaluated by the oracle in FP64 from the same output
    rho, within FP32 rounding of the terms: 8 u32 (|psi'| + kappa 20 rho)."""
    p = {"f16": lbm.LBM_F16DEV, "bf16": lbm.LBM_BF16DEV}[prec]
    lat = lbm.Lattice(C3_512.lbm_params(p, rho_ref=2.6), C3_512.rho0())
    fd = lat.fields()
    lat.close()
    rho, mu = fd["rho"], fd["mu"]
    op = C3_512.oracle_params()
    lo, hi = thermo.spinodal(thermo.fluid_at(C3_512.eos, *C3_512.ab, 1.0, C3_512.Tr))
    assert lo < rho.min() and rho.max() < hi
    mu_b = eos_c(op, rho)[2].reshape(rho.shape)
    want = mu_b - op.kappa * stencils_c(op, rho)[0]
    bound = 8 * 2.0 ** -24 * (np.abs(mu_b) + op.kappa * 20 * rho)
    excess = np.abs(mu - want) / bound
    print("%s band mu: max |error| / bound %.3f" % (prec, excess.max()))
    assert excess.max() <= 1.0
