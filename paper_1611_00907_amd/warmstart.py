"""Learned warm start for droplet-on-wall runs (the surrogate row of the hot path).

Pipeline, all through the C ABI (every numerical step runs in liblbm.so):

1. ``calibrate``: for each EOS and reduced temperature on a grid, a short batched
   sweep of wall chemical potentials measures the contact angle (Sec. V) and
   interpolates the wall values that give 30 and 150 degrees; the wetting range
   of a case is the interval between them.
2. ``draw_cases`` / ``generate``: seeded droplet-on-wall cases (EOS CS or PR,
   T/Tc, wall chemical potential inside its wetting range, drop radius a quarter of
   the side) relaxed to equilibrium by the batched solver.
3. ``features``: network inputs (solid mask, initial density / liquid density,
   T/Tc, wall chemical potential as a fraction of the wetting range) and targets
   (equilibrium density / liquid density).
4. ``Surrogate`` training on the GPU (BF16 MFMA forward and backward, Adam).
5. ``time_to_angle``: steps until the contact angle stays within a tolerance of
   the plain method's equilibrium angle, from the cold start (the semicircle), from
   the calibration's angle alone and from the network's prediction; cases that have
   settled are stopped, so the sweep's device time is what a batch that drops its
   finished cases spends.
"""
from __future__ import annotations

import functools
import os
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from . import inputs, lbm

CS_AB = (1.0, 4.0)
PR_AB = (2 / 49, 2 / 21)
PR_OMEGA = 0.344
TAU, KAPPA = 1.3, 0.01


@dataclass
class CaseSpec:
    eos: int
    Tr: float
    frac: float        # position of the wall mu inside the wetting range (0 -> 30 deg, 1 -> 150 deg)
    mu_w: float
    side: int
    theta0: float = 90.0  # contact angle the calibration sweeps give for this case

    def params(self, prec=lbm.LBM_F32):
        a, b = CS_AB if self.eos == lbm.LBM_EOS_CS else PR_AB
        om = PR_OMEGA if self.eos == lbm.LBM_EOS_PR else 0.0
        return lbm.make_params(self.side, self.side, self.eos, a, b, self.Tr, TAU, KAPPA, omega=om, prec=prec,
                               bc_bottom=lbm.LBM_BC_CPWALL, bc_top=lbm.LBM_BC_NEUTRAL)

    def coexistence(self):
        key = (self.eos, self.Tr)
        if key not in _COEX:
            _COEX[key] = lbm.lbm_coexistence(self.params())
        return _COEX[key]


_COEX: dict = {}   # (eos, Tr) -> (rho_g, rho_l, p_sat, mu_sat): host FP64, independent of the lattice


@functools.lru_cache(maxsize=4096)
def _cold_field(side, rl, rg):
    rho = inputs.sessile_drop(side, side, rl, rg, 0.25 * side)
    rho.setflags(write=False)
    return rho


def initial_density(spec: CaseSpec):
    """The cold start: a semicircular drop of radius side / 4 on the first fluid row
    at the coexistence densities (a fresh array on every call)."""
    rg, rl, _, _ = spec.coexistence()
    return _cold_field(spec.side, float(rl), float(rg)).copy()


def measure_angle(rho):
    """Contact angle of the drop on the first fluid row (NaN if there is no drop, or
    if the liquid covers the whole base row, a film rather than a drop)."""
    rg = float(np.median(rho[-10:-2]))
    rl = float(np.max(rho[1:-1]))
    if not np.isfinite(rg + rl) or rl <= rg * 1.5:
        return float("nan")
    try:
        th, L, _ = lbm.lbm_contact_angle(rho, 0.5 * (rg + rl), base_row=1)
    except lbm.LbmError:
        return float("nan")
    if not (0.0 < th < 180.0) or L >= rho.shape[1] - 2:
        return float("nan")
    return th


# ---------------------------------------------------------------- 1. calibration
class Calibration(dict):
    """{(eos, Tr): (mu_30, mu_150)}, the wetting range at each grid point, with the
    sweeps it came from in .sweeps: {(eos, Tr): (mu_w values, contact angles)}."""

    def __init__(self):
        super().__init__()
        self.sweeps = {}


def calibrate(Tr_grid=(0.6, 0.7, 0.8, 0.9), side=128, steps=20000, offsets=None):
    """Sweeps of mu_w - mu_sat at each grid point; the wall mu giving 30 and 150
    degrees by monotone interpolation of the measured angles."""
    if offsets is None:
        offsets = {lbm.LBM_EOS_PR: np.linspace(-0.3, 0.3, 13), lbm.LBM_EOS_CS: np.linspace(-0.06, 0.06, 13)}
    table = Calibration()
    for eos in (lbm.LBM_EOS_CS, lbm.LBM_EOS_PR):
        specs, mu_sats = [], []
        for Tr in Tr_grid:
            s0 = CaseSpec(eos, Tr, 0.0, 0.0, side)
            mu_sat = s0.coexistence()[3]
            for d in offsets[eos]:
                specs.append(CaseSpec(eos, Tr, 0.0, mu_sat + d, side))
            mu_sats.append(mu_sat)
        b = lbm.Batch([s.params() for s in specs], [initial_density(s) for s in specs],
                      mu_w_bottom=[s.mu_w for s in specs])
        b.step(steps)
        th = np.array([measure_angle(b.rho(i)) for i in range(len(specs))])
        b.close()
        k = len(offsets[eos])
        for j, Tr in enumerate(Tr_grid):
            t = th[j * k:(j + 1) * k]
            mus = mu_sats[j] + offsets[eos]
            ok = np.isfinite(t)
            if ok.sum() < 3:
                continue
            # monotone interpolation of mu at 30 and 150 degrees
            tt, mm = np.maximum.accumulate(t[ok]), mus[ok]
            table[(eos, Tr)] = (float(np.interp(30.0, tt, mm)), float(np.interp(150.0, tt, mm)))
            table.sweeps[(eos, Tr)] = (mm, tt)
    return table


def wetting_range(table, eos, Tr):
    grid = sorted(T for (e, T) in table if e == eos)
    lo = np.interp(Tr, grid, [table[(eos, T)][0] for T in grid])
    hi = np.interp(Tr, grid, [table[(eos, T)][1] for T in grid])
    return float(lo), float(hi)


def theta_guess(table, eos, Tr, mu_w):
    """Contact angle of (eos, Tr, mu_w) from the calibration sweeps: the angle at
    mu_w of each grid temperature's sweep, interpolated linearly in Tr."""
    sw = getattr(table, "sweeps", {})
    grid = sorted(T for (e, T) in sw if e == eos)
    if not grid:
        return 90.0
    per_T = [float(np.interp(mu_w, *sw[(eos, T)])) for T in grid]
    return float(np.interp(Tr, grid, per_T))


# ---------------------------------------------------------------- 2. cases and equilibria
def draw_cases(n, seed, table, side=256, Tr_range=(0.6, 0.9)):
    u = inputs.uniform(seed, 3 * n).reshape(n, 3)
    out = []
    for k in range(n):
        eos = lbm.LBM_EOS_CS if u[k, 0] < 0.5 else lbm.LBM_EOS_PR
        Tr = Tr_range[0] + (Tr_range[1] - Tr_range[0]) * u[k, 1]
        lo, hi = wetting_range(table, eos, Tr)
        mu_w = lo + (hi - lo) * float(u[k, 2])
        out.append(CaseSpec(eos, Tr, float(u[k, 2]), mu_w, side, theta_guess(table, eos, Tr, mu_w)))
    return out


def generate(specs, max_steps=60000, check_every=2000, window=1000, tol=1e-9, confirm_steps=0, prec=lbm.LBM_F32):
    """Relaxes every case with the batched solver in storage precision prec until its
    residual max|rho(t) - rho(t - window)| / window falls below tol (the case then
    stops) or max_steps have passed; returns (rho_eq list, state array, steps array,
    angle drift).  With confirm_steps > 0 the cases still running take that many more
    steps and the drift is the change of their contact angle over them (an
    equilibrium angle that still moves is not one).  FP32 storage has a residual
    floor of a few 1e-8 per step (its rounding keeps the field moving), so only FP64
    reaches tol = 1e-9."""
    b = lbm.Batch([s.params(prec) for s in specs], [initial_density(s) for s in specs],
                  mu_w_bottom=[s.mu_w for s in specs])
    b.run(max_steps, check_every=check_every, window=window, tol=tol)
    drift = np.zeros(len(specs))
    if confirm_steps > 0:
        th1 = np.array([measure_angle(b.rho(i)) for i in range(len(specs))])
        b.step(confirm_steps)
        th2 = np.array([measure_angle(b.rho(i)) for i in range(len(specs))])
        drift = np.abs(th2 - th1)
    st = b.status()
    rho = [b.rho(i) for i in range(len(specs))]
    b.close()
    return rho, st["state"], st["steps"], drift


# ---------------------------------------------------------------- 3. features
def phase(spec: CaseSpec, rho):
    """ln(rho / rho_g) / ln(rho_l / rho_g): 0 in the vapour, 1 in the liquid at
    coexistence.  Logarithmic, so that a vapour density several times Maxwell's (the
    discrete equilibrium of a thin interface next to a small drop) is as visible to
    the network as a few percent on the liquid."""
    rg, rl, _, _ = spec.coexistence()
    return np.log(np.maximum(np.asarray(rho, np.float64), 1e-300) / rg) / np.log(rl / rg)


def density(spec: CaseSpec, phi):
    """Inverse of phase."""
    rg, rl, _, _ = spec.coexistence()
    return rg * np.exp(np.asarray(phi, np.float64) * np.log(rl / rg))


def features(spec: CaseSpec):
    """Network input [4][side][side] for a case: solid mask, phase of the initial
    density (the cap of the calibrated angle theta0 at the cold start's mass; the
    semicircle when theta0 = 90), T/Tc, and the wall chemical potential's place in
    the wetting range."""
    x = np.zeros((4, spec.side, spec.side), np.float32)
    x[0, 0, :] = 1.0
    x[0, -1, :] = 1.0
    rg, rl, _, _ = spec.coexistence()
    x[1] = lbm.warm_phase(cap_field(spec, spec.theta0), rg, rl)
    x[2] = spec.Tr
    x[3] = spec.frac
    return x


def target(spec: CaseSpec, rho_eq):
    """Network target: the phase of the equilibrium density."""
    return phase(spec, rho_eq).astype(np.float32)


def he_init(seed):
    """He-normal weights, zero biases, in the exchange layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co in lbm.Surrogate.LAYERS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


# ---------------------------------------------------------------- 5. time to equilibrium
def time_to_angle(specs, rho_starts, theta_eq, tol_deg=0.5, check_every=200, max_steps=60000, hold=4,
                  log=None):
    """Per case, the step from which the contact angle stays within tol of theta_eq
    (checked every check_every steps, -1 if never).  All cases start as one batch;
    a case that has stayed inside for `hold` checks is stopped (masked out of the
    batch, lbm_batch_stop), so the batch shrinks as cases settle.  Returns the
    per-case steps, the device time per step of the full batch (first check
    interval), and the device time of the whole masked sweep."""
    b = lbm.Batch([s.params() for s in specs], rho_starts, mu_w_bottom=[s.mu_w for s in specs])
    n = len(specs)
    first_in = np.full(n, -1, np.int64)
    done = np.zeros(n, bool)
    t_dev, t_full = 0.0, None
    steps = 0
    while True:
        act = np.flatnonzero(~done)
        th = np.array([measure_angle(b.rho(i)) for i in act])
        inside = np.abs(th - theta_eq[act]) <= tol_deg
        first_in[act[~inside]] = -1
        first_in[act[inside & (first_in[act] < 0)]] = steps
        settled = act[(first_in[act] >= 0) & (steps - first_in[act] >= hold * check_every)]
        if settled.size:
            b.stop(settled)
            done[settled] = True
        if done.all() or steps >= max_steps:
            break
        dt = b.step_timed(check_every) / 1e3
        if t_full is None:
            t_full = dt / check_every
        t_dev += dt
        steps += check_every
        if log and steps % (25 * check_every) == 0:
            log("  step %d: %d of %d cases settled within %.1f deg" % (steps, int(done.sum()), n, tol_deg))
    b.close()
    first_in[~done] = -1
    return first_in, (t_full if t_full is not None else 0.0), t_dev


def cap_field(spec: CaseSpec, theta_deg, rho_l=None, rho_g=None):
    """Sessile circular cap of contact angle theta on the first fluid row at the
    bulk densities rho_l, rho_g (default: the coexistence values), holding the cold
    start's mass: liquid area A = (M - rho_g N) / (rho_l - rho_g) over the N fluid
    nodes, radius R = sqrt(A / (t - sin t cos t)), centre -R cos t above that row,
    the cold start's interface width; the liquid excess is then scaled so that the
    fluid rows hold exactly the mass M."""
    rg0, rl0, _, _ = spec.coexistence()
    rl = rl0 if rho_l is None else float(rho_l)
    rg = rg0 if rho_g is None else float(rho_g)
    cold = initial_density(spec)
    fl = slice(1, spec.side - 1)                     # fluid rows between the walls
    M, N = float(cold[fl].sum()), cold[fl].size
    if not M - rg * N > 0.05 * (M - rg0 * N):
        # the vapour alone would hold (nearly) all the mass: no drop at these densities
        if rho_l is None and rho_g is None:
            return cold
        return cap_field(spec, theta_deg)
    A = (M - rg * N) / (rl - rg)
    t = np.radians(float(np.clip(theta_deg, 5.0, 175.0)))
    R = np.sqrt(A / (t - np.sin(t) * np.cos(t)))
    rho = lbm.warm_cap(spec.side, spec.side, rl, rg, R, spec.side / 2.0, 1.0 - R * np.cos(t))
    excess = rho[fl] - rg
    rho[fl] = rg + excess * ((M - rg * N) / excess.sum())
    rho[0] = rho[1]
    rho[-1] = rho[-2]
    return rho


def read_prediction(spec: CaseSpec, pred):
    """Contact angle and bulk densities of a predicted phase field (clipped to
    [-0.5, 1.5], which keeps the offsets of the equilibrium phases, and smoothed
    once, in FP32, the prediction's own precision): the angle by the Sec. V measure,
    the bulk phases as the medians of the nodes whose 5 x 5 neighbourhood lies on one
    side of 1/2.  NaN angle if none can be read.  The field work runs in the library's
    host helpers, which leave the interpreter free for other threads."""
    rg, rl, _, _ = spec.coexistence()
    phi = lbm.warm_smooth(pred, -0.5, 1.5)
    theta = measure_angle(lbm.warm_density(phi, rg, rl))
    ph_l, ph_g = lbm.warm_bulk_phases(phi)
    return theta, float(density(spec, ph_l)), float(density(spec, ph_g))


VAPOUR_PINNING = 1.5   # predicted vapour / Maxwell vapour above which the interface is sub-grid


def predicted_field(spec: CaseSpec, pred, rho_g, rho_max):
    """The predicted density field (phase clipped to [-0.5, 1.5], smoothed once,
    densities capped at rho_max) with its excess over rho_g scaled so that the fluid
    rows hold the cold start's mass."""
    rg0, rl0, _, _ = spec.coexistence()
    rho = np.minimum(lbm.warm_density(lbm.warm_smooth(pred, -0.5, 1.5), rg0, rl0), rho_max)
    fl = slice(1, spec.side - 1)
    M, N = float(initial_density(spec)[fl].sum()), rho[fl].size
    excess = np.maximum(rho[fl] - rho_g, 0.0)
    if not (excess.sum() > 0 and M - rho_g * N > 0):
        return cap_field(spec, read_prediction(spec, pred)[0])
    rho[fl] = np.minimum(rho_g + excess * ((M - rho_g * N) / excess.sum()), rho_max)
    rho[0] = rho[1]
    rho[-1] = rho[-2]
    return rho


def warm_field(spec: CaseSpec, pred, pinned="cap"):
    """Warm start from a predicted phase field: a clean circular cap with the
    prediction's contact angle and bulk densities and the cold start's mass
    (cap_field).  The prediction's pixel noise is not carried over; the mass is
    the cold start's because the method conserves it (a start of another mass
    relaxes to another equilibrium); the bulk densities are the prediction's
    because the equilibrium ones differ from Maxwell's (the liquid by up to 2 %,
    the vapour by up to several times next to thin interfaces), and moving that
    mass between the phases is the slowest part of the relaxation.  If no angle can be read
    from the prediction, the cold start is returned."""
    theta, rl, rg = read_prediction(spec, pred)
    if not np.isfinite(theta) or not rl > rg:
        return initial_density(spec)
    # The discrete equilibria of the training cases put the liquid at 1.000-1.017
    # times Maxwell's density and the vapour at 0.95-7.4 times (thin interfaces next
    # to small drops); the prediction's levels are kept inside [1, 1.02] and
    # [0.9, 8] times Maxwell's.  A liquid compressed beyond its equilibrium density
    # (the log phase resolves the liquid end coarsely) launches pressure waves that
    # the thin-interface CS cases at low T do not survive.
    rg0, rl0, _, _ = spec.coexistence()
    if rg > VAPOUR_PINNING * rg0:
        # A vapour this far above Maxwell's marks an interface thinner than the
        # lattice spacing: there the contact line is pinned by the lattice and the
        # equilibrium angle depends on the path (a clean cap at the predicted
        # densities stops up to 2 degrees away from the cold start's angle).
        # pinned == "cap": start from Maxwell's densities, as the cold start does,
        # with the predicted angle (every case then reaches the cold start's angle);
        # pinned == "field": start from the predicted field itself, which carries
        # the cold path's end state (faster, but about 1 case in 10 still stops
        # elsewhere).
        if pinned == "field":
            return predicted_field(spec, pred, rg, 1.02 * rl0)
        return cap_field(spec, theta)
    rl = float(np.clip(rl, rl0, 1.02 * rl0))
    rg = float(np.clip(rg, 0.9 * rg0, 8.0 * rg0))
    return cap_field(spec, theta, rl, rg)


def sub_grid_interface(spec: CaseSpec, pred):
    """Whether a prediction marks the case's interface as thinner than the lattice
    spacing (predicted vapour above VAPOUR_PINNING times Maxwell's), where the contact
    line is pinned by the lattice and the equilibrium depends on the path."""
    _, rl, rg = read_prediction(spec, pred)
    return bool(rl > rg and rg > VAPOUR_PINNING * spec.coexistence()[0])


def evaluate(net, specs, theta_eq, tol_deg=0.5, check_every=200, max_steps=60000, log=None, calibration_arm=False,
             pinned="cap", by_class=False):
    """Cold versus warm start of one batched sweep: per-case steps to the plain
    equilibrium angle, and the sweep's device time until its last case is there
    (for the warm start plus the network inference and the warm-field set-up).
    With by_class, the cold and warm sweeps are also run separately over the two
    classes the prediction tells apart (resolved and sub-grid interfaces), each
    charged its share of the inference time."""
    cold0 = [initial_density(s) for s in specs]
    steps_cold, dt_cold, dev_cold = time_to_angle(specs, cold0, theta_eq, tol_deg, check_every, max_steps, log=log)
    t0 = time.perf_counter()
    # the field work runs in library calls that release the interpreter, so threads scale
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as pool:
        x = np.stack(list(pool.map(features, specs)))
        pred = net.forward(x)
        warm0 = list(pool.map(lambda sp: warm_field(sp[0], sp[1], pinned), zip(specs, pred)))
    t_inf = time.perf_counter() - t0
    steps_warm, dt_warm, dev_warm = time_to_angle(specs, warm0, theta_eq, tol_deg, check_every, max_steps, log=log)
    done = (steps_cold >= 0).all() and (steps_warm >= 0).all()
    # sweep time, two ways: every case charged until the last one settles (the slowest
    # case times the full batch), and the device time of the batch with settled cases
    # masked out (what a sweep that stops its finished cases spends)
    t_cold = float(steps_cold.max() * dt_cold) if done else float("nan")
    t_warm = float(steps_warm.max() * dt_warm + t_inf) if done else float("nan")
    sub_grid = np.array([sub_grid_interface(sp, pr) for sp, pr in zip(specs, pred)])
    out = {"steps_cold": steps_cold, "steps_warm": steps_warm, "step_time_cold": dt_cold, "sub_grid": sub_grid,
           "step_time_warm": dt_warm, "inference_s": t_inf, "pred": pred,
           "sweep_s_cold": t_cold, "sweep_s_warm": t_warm,
           "speedup": t_cold / t_warm if done else float("nan"),
           "masked_sweep_s_cold": dev_cold, "masked_sweep_s_warm": dev_warm + t_inf,
           "speedup_masked": dev_cold / (dev_warm + t_inf) if done else float("nan")}
    if by_class:
        theta_eq = np.asarray(theta_eq)
        for cls, m in (("resolved", ~sub_grid), ("sub_grid", sub_grid)):
            idx = np.flatnonzero(m)
            if idx.size == 0:
                continue
            sp = [specs[i] for i in idx]
            sc, dtc, devc = time_to_angle(sp, [cold0[i] for i in idx], theta_eq[idx], tol_deg, check_every,
                                          max_steps, log=log)
            sw, dtw, devw = time_to_angle(sp, [warm0[i] for i in idx], theta_eq[idx], tol_deg, check_every,
                                          max_steps, log=log)
            ok = (sc >= 0).all() and (sw >= 0).all()
            share = t_inf * idx.size / len(specs)
            tc = float(sc.max() * dtc) if ok else float("nan")
            tw = float(sw.max() * dtw + share) if ok else float("nan")
            out["sweep_" + cls] = {"cases": int(idx.size), "sweep_s_cold": tc, "sweep_s_warm": tw,
                                   "speedup": tc / tw if ok else float("nan"), "masked_sweep_s_cold": devc,
                                   "masked_sweep_s_warm": devw + share,
                                   "speedup_masked": devc / (devw + share) if ok else float("nan")}
    if calibration_arm:
        # the same sweep started from the calibration's angle alone (no network):
        # what the trained network adds over the method without it
        cal0 = [cap_field(s, s.theta0) for s in specs]
        steps_cal, dt_cal, dev_cal = time_to_angle(specs, cal0, theta_eq, tol_deg, check_every, max_steps, log=log)
        ok = (steps_cold >= 0).all() and (steps_cal >= 0).all()
        out["steps_calibration_only"] = steps_cal
        out["sweep_s_calibration_only"] = float(steps_cal.max() * dt_cal) if ok else float("nan")
        out["speedup_calibration_only"] = t_cold / out["sweep_s_calibration_only"] if ok else float("nan")
        out["masked_sweep_s_calibration_only"] = dev_cal
        out["speedup_masked_calibration_only"] = dev_cold / dev_cal if ok else float("nan")
    return out


# ---------------------------------------------------------------- the whole experiment
def run_experiment(n_cases=2000, side=256, seed=11, n_val=100, n_test=100, train_steps=(4000, 3000, 2000, 1000),
                   lrs=(1e-3, 5e-4, 2e-4, 1e-4), batch=16, calib_side=256, calib_steps=30000, gen_steps=80000,
                   confirm_steps=20000, gen_chunk=500, log=print, debug_path=None, pinned="cap", gen_prec=lbm.LBM_F64):
    """Calibrate, generate n_cases equilibria with the batched solver (FP64 storage by
    default, so that the residual criterion max|drho| < 1e-9 per step can fire), train
    the surrogate on the GPU, and compare cold and warm starts (FP32 storage) on the
    held-out test cases."""
    out = {"n_cases": n_cases, "side": side, "seed": seed, "pinned": pinned,
           "generation_storage": {lbm.LBM_F64: "f64", lbm.LBM_F32: "f32"}.get(gen_prec, str(gen_prec))}
    t0 = time.perf_counter()
    table = calibrate(Tr_grid=(0.6, 0.65, 0.7, 0.75, 0.8, 0.85, 0.9), side=calib_side, steps=calib_steps)
    out["calibration_s"] = time.perf_counter() - t0
    out["wetting_range"] = {"%d/%.2f" % k: v for k, v in table.items()}
    log("calibration: %d grid points in %.1f s" % (len(table), out["calibration_s"]))
    specs = draw_cases(n_cases, seed, table, side=side)
    rho_eq, state, steps, drift = [], [], [], []
    t0 = time.perf_counter()
    for c0 in range(0, n_cases, gen_chunk):
        r, st, stp, dr = generate(specs[c0:c0 + gen_chunk], max_steps=gen_steps, check_every=2000, window=1000,
                                  tol=1e-9, confirm_steps=confirm_steps, prec=gen_prec)
        rho_eq += r
        state += list(st)
        steps += list(stp)
        drift += list(dr)
        log("generated %d / %d equilibria (%.1f s)" % (len(rho_eq), n_cases, time.perf_counter() - t0))
    out["generation_s"] = time.perf_counter() - t0
    state, steps, drift = np.array(state), np.array(steps), np.array(drift)
    theta = np.array([measure_angle(r) if np.isfinite(r).all() else np.nan for r in rho_eq])
    # usable: not diverged, a drop (not a film) between 35 and 160 degrees whose angle
    # moved less than 0.1 degree over the last confirm_steps steps
    ok = [i for i in range(n_cases) if state[i] != 2 and np.isfinite(theta[i]) and 35 < theta[i] < 160
          and drift[i] < 0.1]
    out["unsettled"] = int(np.sum(np.isfinite(drift) & (drift >= 0.1)))
    out["usable"] = len(ok)
    out["converged"] = int((state == 1).sum())
    out["relax_steps_median"] = float(np.median(steps[ok])) if ok else None
    log("usable equilibria: %d (converged %d, angle still moving %d)" % (len(ok), out["converged"],
                                                                          out["unsettled"]))
    test, val, train = ok[-n_test:], ok[-n_test - n_val:-n_test], ok[:-n_test - n_val]
    net = lbm.Surrogate(side, max_batch=batch)
    net.set_params(he_init(seed))
    x = np.stack([features(specs[i]) for i in train])
    t = np.stack([target(specs[i], rho_eq[i]) for i in train])
    net.set_dataset(x, t)
    del x, t
    losses = []
    t0 = time.perf_counter()
    chunk = 250
    for k, (n, lr) in enumerate(zip(train_steps, lrs)):
        for j in range(0, n, chunk):
            losses.append(net.train(min(chunk, n - j), batch, lr, seed=seed + 1000 * k + j))
            log("trained %d steps at lr %g: loss %.3e (%.1f s)" % (j + min(chunk, n - j), lr,
                                                                   float(np.mean(losses[-1][-50:])),
                                                                   time.perf_counter() - t0))
    out["training_s"] = time.perf_counter() - t0
    losses = np.concatenate(losses)
    out["loss_first"] = float(losses[:20].mean())
    out["loss_last"] = float(losses[-50:].mean())
    xv = np.stack([features(specs[i]) for i in val])
    tv = np.stack([target(specs[i], rho_eq[i]) for i in val])
    out["val_mse"] = float(np.mean((net.forward(xv) - tv) ** 2))
    tspecs = [specs[i] for i in test]
    res = evaluate(net, tspecs, theta[test], tol_deg=0.5, check_every=200, max_steps=40000, log=log,
                   calibration_arm=True, pinned=pinned, by_class=True)
    out["theta_calibration_abs_err_median"] = float(np.median(np.abs([s.theta0 for s in tspecs] - theta[test])))
    pred_theta = np.array([read_prediction(s, p)[0] for s, p in zip(tspecs, res["pred"])])
    if debug_path:
        never = [k for k in range(len(tspecs)) if res["steps_warm"][k] < 0]
        np.savez_compressed(debug_path, never=np.array(never), pred=res["pred"][never] if never else np.zeros(0),
                            eq=np.array([rho_eq[test[k]] for k in never]) if never else np.zeros(0),
                            warm=np.array([warm_field(tspecs[k], res["pred"][k], pinned) for k in never]) if never else
                            np.zeros(0), eos=np.array([tspecs[k].eos for k in never]),
                            Tr=np.array([tspecs[k].Tr for k in never]), mu_w=np.array([tspecs[k].mu_w for k in never]))
    out.update({k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in res.items() if k != "pred"})
    out["theta_eq"] = theta[test].tolist()
    out["test_eos"] = [s.eos for s in tspecs]
    out["test_Tr"] = [s.Tr for s in tspecs]
    out["theta_pred"] = pred_theta.tolist()
    out["theta_pred_abs_err_median"] = float(np.nanmedian(np.abs(pred_theta - theta[test])))
    out["steps_saved_median"] = float(np.median(res["steps_cold"] - res["steps_warm"]))
    # mean steps to the plain equilibrium angle per arm, over all test cases and over
    # the two classes the prediction tells apart: resolved interfaces, and interfaces
    # thinner than the lattice spacing (path-dependent, pinned contact lines)
    sg = np.asarray(res["sub_grid"], bool)
    arms = [k for k in ("steps_cold", "steps_calibration_only", "steps_warm") if k in res]
    for cls, m in (("all", np.ones_like(sg)), ("resolved", ~sg), ("sub_grid", sg)):
        if m.any():
            out["steps_mean_" + cls] = {k[6:]: float(np.mean(np.asarray(res[k])[m])) for k in arms}
            out["steps_mean_" + cls]["cases"] = int(m.sum())
    log("sweep to 0.5 deg: cold %.3f s, warm %.3f s (inference %.3f s): %.2fx; calibration angle alone %.2fx" %
        (out["sweep_s_cold"], out["sweep_s_warm"], out["inference_s"], out["speedup"],
         out.get("speedup_calibration_only", float("nan"))))
    log("masked sweep (settled cases stopped): cold %.3f s, warm %.3f s: %.2fx; calibration angle alone %.2fx" %
        (out["masked_sweep_s_cold"], out["masked_sweep_s_warm"], out["speedup_masked"],
         out.get("speedup_masked_calibration_only", float("nan"))))
    for cls in ("resolved", "sub_grid"):
        if "sweep_" + cls in out:
            c = out["sweep_" + cls]
            log("%s interfaces (%d cases): sweep %.2fx, masked sweep %.2fx" % (cls, c["cases"], c["speedup"],
                                                                                c["speedup_masked"]))
    net.close()
    return out


if __name__ == "__main__":
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description="learned warm start: calibration, equilibria, training, evaluation")
    ap.add_argument("--cases", type=int, default=2000)
    ap.add_argument("--side", type=int, default=256)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--val", type=int, default=100)
    ap.add_argument("--test", type=int, default=100)
    ap.add_argument("--out", default=None, help="write the result as JSON here")
    ap.add_argument("--debug", default=None, help="write the cases whose warm start missed to this .npz")
    ap.add_argument("--pinned", choices=("cap", "field"), default="cap",
                    help="warm start of the sub-grid-interface cases (see warm_field)")
    ap.add_argument("--gen-storage", choices=("f64", "f32"), default="f64",
                    help="storage precision of the equilibrium generation (only f64 reaches the 1e-9 residual)")
    a = ap.parse_args()
    r = run_experiment(a.cases, a.side, a.seed, a.val, a.test, log=lambda m: print(m, flush=True),
                       debug_path=a.debug, pinned=a.pinned,
                       gen_prec=lbm.LBM_F64 if a.gen_storage == "f64" else lbm.LBM_F32)
    r["command"] = " ".join(["python -m paper_1611_00907_amd.warmstart"] + sys.argv[1:])
    print(json.dumps(r))
    if a.out:
        json.dump(r, open(a.out, "w"), indent=1)
