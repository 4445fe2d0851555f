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
5. ``time_to_angle``: steps and device time until the contact angle stays within
   a tolerance of the plain method's equilibrium angle, from the cold start (the
   semicircle) and from the network's prediction.
"""
from __future__ import annotations

import time
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

    def params(self, prec=lbm.LBM_F32):
        a, b = CS_AB if self.eos == lbm.LBM_EOS_CS else PR_AB
        om = PR_OMEGA if self.eos == lbm.LBM_EOS_PR else 0.0
        return lbm.make_params(self.side, self.side, self.eos, a, b, self.Tr, TAU, KAPPA, omega=om, prec=prec,
                               bc_bottom=lbm.LBM_BC_CPWALL, bc_top=lbm.LBM_BC_NEUTRAL)

    def coexistence(self):
        return lbm.lbm_coexistence(self.params())


def initial_density(spec: CaseSpec):
    rg, rl, _, _ = spec.coexistence()
    return inputs.sessile_drop(spec.side, spec.side, rl, rg, 0.25 * spec.side)


def measure_angle(rho):
    """Contact angle of the drop on the first fluid row (NaN if there is no drop)."""
    rg = float(np.median(rho[-10:-2]))
    rl = float(np.max(rho[1:-1]))
    if not np.isfinite(rg + rl) or rl <= rg * 1.5:
        return float("nan")
    try:
        return lbm.lbm_contact_angle(rho, 0.5 * (rg + rl), base_row=1)[0]
    except lbm.LbmError:
        return float("nan")


# ---------------------------------------------------------------- 1. calibration
def calibrate(Tr_grid=(0.6, 0.7, 0.8, 0.9), side=128, steps=20000, offsets=None):
    """{(eos, Tr): (mu_30, mu_150)} from sweeps of mu_w - mu_sat at each grid point."""
    if offsets is None:
        offsets = {lbm.LBM_EOS_PR: np.linspace(-0.3, 0.3, 13), lbm.LBM_EOS_CS: np.linspace(-0.06, 0.06, 13)}
    table = {}
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
        th = np.array([measure_angle(b.fields(i)["rho"]) for i in range(len(specs))])
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
    return table


def wetting_range(table, eos, Tr):
    grid = sorted(T for (e, T) in table if e == eos)
    lo = np.interp(Tr, grid, [table[(eos, T)][0] for T in grid])
    hi = np.interp(Tr, grid, [table[(eos, T)][1] for T in grid])
    return float(lo), float(hi)


# ---------------------------------------------------------------- 2. cases and equilibria
def draw_cases(n, seed, table, side=256, Tr_range=(0.6, 0.9)):
    u = inputs.uniform(seed, 3 * n).reshape(n, 3)
    out = []
    for k in range(n):
        eos = lbm.LBM_EOS_CS if u[k, 0] < 0.5 else lbm.LBM_EOS_PR
        Tr = Tr_range[0] + (Tr_range[1] - Tr_range[0]) * u[k, 1]
        lo, hi = wetting_range(table, eos, Tr)
        out.append(CaseSpec(eos, Tr, float(u[k, 2]), lo + (hi - lo) * float(u[k, 2]), side))
    return out


def generate(specs, max_steps=60000, check_every=2000, window=1000, tol=1e-9):
    """Relaxes every case with the batched solver; returns (rho_eq list, state array, steps array)."""
    b = lbm.Batch([s.params() for s in specs], [initial_density(s) for s in specs],
                  mu_w_bottom=[s.mu_w for s in specs])
    b.run(max_steps, check_every=check_every, window=window, tol=tol)
    st = b.status()
    rho = [b.fields(i)["rho"] for i in range(len(specs))]
    b.close()
    return rho, st["state"], st["steps"]


# ---------------------------------------------------------------- 3. features
def features(spec: CaseSpec):
    """Network input [4][side][side] for a case."""
    rg, rl, _, _ = spec.coexistence()
    x = np.zeros((4, spec.side, spec.side), np.float32)
    x[0, 0, :] = 1.0
    x[0, -1, :] = 1.0
    x[1] = initial_density(spec) / rl
    x[2] = spec.Tr
    x[3] = spec.frac
    return x


def target(spec: CaseSpec, rho_eq):
    rl = spec.coexistence()[1]
    return (rho_eq / rl).astype(np.float32)


def he_init(seed):
    """He-normal weights, zero biases, in the exchange layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co in lbm.Surrogate.LAYERS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


# ---------------------------------------------------------------- 5. time to equilibrium
def time_to_angle(specs, rho_starts, theta_eq, tol_deg=0.5, check_every=200, max_steps=60000):
    """Steps until each case's angle enters tol of theta_eq and stays there at every
    later check, starting from rho_starts; also the device time per batched step."""
    b = lbm.Batch([s.params() for s in specs], rho_starts, mu_w_bottom=[s.mu_w for s in specs])
    n = len(specs)
    first_in = np.full(n, -1, np.int64)
    t_dev = 0.0
    steps = 0
    while steps < max_steps:
        th = np.array([measure_angle(b.fields(i)["rho"]) for i in range(n)])
        inside = np.abs(th - theta_eq) <= tol_deg
        for i in range(n):
            if inside[i] and first_in[i] < 0:
                first_in[i] = steps
            elif not inside[i]:
                first_in[i] = -1
        if steps > 0 and (first_in >= 0).all() and steps - first_in.min() >= 4 * check_every:
            break
        t_dev += b.step_timed(check_every) / 1e3
        steps += check_every
    b.close()
    step_time = t_dev / max(steps, 1)
    return first_in, step_time


def clamp_prediction(spec: CaseSpec, pred):
    rg, rl, _, _ = spec.coexistence()
    pole = (1.0 if spec.eos == lbm.LBM_EOS_PR else 4.0) / (PR_AB[1] if spec.eos == lbm.LBM_EOS_PR else CS_AB[1])
    return np.clip(pred * rl, 0.5 * rg, 0.95 * pole)


def evaluate(net, specs, theta_eq, tol_deg=0.5, check_every=200, max_steps=60000):
    """Cold versus warm start: per-case steps to the plain equilibrium angle and the
    wall-clock cost (device step time, plus the network inference for the warm start)."""
    cold0 = [initial_density(s) for s in specs]
    steps_cold, dt_cold = time_to_angle(specs, cold0, theta_eq, tol_deg, check_every, max_steps)
    x = np.stack([features(s) for s in specs])
    t0 = time.perf_counter()
    pred = net.forward(x)
    t_inf = time.perf_counter() - t0
    warm0 = [clamp_prediction(s, p) for s, p in zip(specs, pred)]
    steps_warm, dt_warm = time_to_angle(specs, warm0, theta_eq, tol_deg, check_every, max_steps)
    return {"steps_cold": steps_cold, "steps_warm": steps_warm, "step_time_cold": dt_cold,
            "step_time_warm": dt_warm, "inference_s": t_inf, "pred": pred}
