#!/usr/bin/env python3
"""Throughput of the fused chemical-potential LBM step on one MI355X.

Headline workload (the precision configuration with FP32 storage, the HBM-bound
size): 4096 x 4096 periodic D2Q9 lattice, van der Waals EOS (a = 9/49, b = 2/21)
at T = 0.85 Tc, tau = 1, kappa = 0.01, spinodal decomposition from
rho = 2.6 (1 + 0.01 U(-1, 1)).  A step is one fused update (moments, Eq 8
chemical potential, Eq 12 force, Eqs 13-14 collision, streaming) plus the
mass / residual / divergence monitors every min(100, K) steps.  The 1024^2
wetting lattice (whose 75 MB stay in the 256 MB Infinity Cache), the 16-bit
storage types, the 256-case batch and the surrogate's training step are
reported beside it under "aux".

Prints one JSON line: MLUPS (fluid-node updates per second / 1e6) with inputs
resident in HBM, the roofline of the step kernel (72 algorithmic bytes per node
update in FP32: nine loads and nine stores), and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
MONITOR_EVERY = 100
KERNEL_SRC = os.path.join(ROOT, "paper_1611_00907_amd", "csrc", "lbm_kernels.hip")
KERNEL3_SRC = os.path.join(ROOT, "paper_1611_00907_amd", "csrc", "lbm3d_kernels.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-aux", action="store_true")
    ap.add_argument("--surrogate-only", type=int, default=0, metavar="STEPS",
                    help="time STEPS surrogate training steps only, print their JSON and exit (for profiling)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-bytes", type=int, default=1 << 30,
                    help="size of the plain copy whose bandwidth is reported beside the roofline")
    ap.add_argument("--warmstart", action="store_true",
                    help="also run the learned warm-start experiment live (2000 cases at 256^2: "
                         "equilibria, training, cold vs warm sweep; several minutes)")
    ap.add_argument("--workload", choices=("spinodal4096", "wetting1024", "spinodal4096_f16dev",
                                           "spinodal4096_bf16dev", "batch256", "batch256_residual", "d3q19",
                                           "variants"),
                    default="spinodal4096",
                    help="main measurement: the 4096^2 FP32 spinodal lattice (default, HBM-bound); the others "
                         "(the 1024^2 FP32 wetting lattice, the 16-bit storage types, the 256-case batch) "
                         "are reported under aux and can be run alone as the main line for profiling; "
                         "batch256_residual runs the 256-case batch in FP64 storage to the residual "
                         "max|drho| < 1e-9 per step (about two minutes) and reports how many cases get there")
    return ap.parse_args()


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def wetting_workload(lbm, inputs, prec):
    nx = ny = 1024
    p = lbm.make_params(nx, ny, lbm.LBM_EOS_PR, 2 / 49, 2 / 21, 0.8, 1.3, 0.01, omega=0.344, prec=prec,
                        bc_bottom=lbm.LBM_BC_CPWALL, bc_top=lbm.LBM_BC_NEUTRAL)
    rg, rl, _, mu_sat = lbm.lbm_coexistence(p)
    rho0 = inputs.sessile_drop(nx, ny, rl, rg, 200.0)
    # one draw from the wetting range suggested by the paper's Fig. 2 span around mu_sat
    mu_w = float(inputs.draw_uniform(2, mu_sat - 0.18, mu_sat + 0.23, 1)[0])
    return p, rho0, mu_w, nx * (ny - 2)


def spinodal_workload(lbm, inputs, prec, n=4096, rho_mean=2.6):
    """Precision configuration: 4096^2 periodic VdW spinodal decomposition at Tr = 0.85,
    tau = 1, kappa = 0.01, rho = rho_mean (1 + 0.01 U(-1, 1)); the mean density is not
    stated, 2.6 lies inside the spinodal (a quench from the critical density 3.5
    overshoots into the EOS pole at this size).  The 16-bit formats store deviations from
    w_i rho_mean: with the literal base w_i, BF16 loses the field within 1000 steps."""
    rho_ref = rho_mean if prec in (lbm.LBM_F16DEV, lbm.LBM_BF16DEV) else 1.0
    p = lbm.make_params(n, n, lbm.LBM_EOS_VDW, 9 / 49, 2 / 21, 0.85, 1.0, 0.01, prec=prec, rho_ref=rho_ref)
    rho0 = inputs.with_relative_noise(np.full((n, n), rho_mean), 0.01, 3)
    return p, rho0, None, n * n


def batch_workload(lbm, inputs, n_cases=256, seed=4):
    """The batching configuration: n droplet-on-wall cases, side ~ U{128..512},
    CS or PR (50/50), Tr ~ U[0.6, 0.9], drop radius 0.25 side on a CP wall whose
    mu_w is drawn around the case's coexistence chemical potential."""
    u = inputs.uniform(seed, 4 * n_cases).reshape(n_cases, 4)
    params, rhos, muw = [], [], []
    for k in range(n_cases):
        side = 128 + int(u[k, 0] * 385)
        eos = lbm.LBM_EOS_CS if u[k, 1] < 0.5 else lbm.LBM_EOS_PR
        Tr = 0.6 + 0.3 * u[k, 2]
        a, b = (1.0, 4.0) if eos == lbm.LBM_EOS_CS else (2 / 49, 2 / 21)
        om = 0.0 if eos == lbm.LBM_EOS_CS else 0.344
        p = lbm.make_params(side, side, eos, a, b, Tr, 1.3, 0.01, omega=om, prec=lbm.LBM_F32,
                            bc_bottom=lbm.LBM_BC_CPWALL, bc_top=lbm.LBM_BC_NEUTRAL)
        rg, rl, _, mu_sat = lbm.lbm_coexistence(p)
        span = 0.2 if eos == lbm.LBM_EOS_PR else 0.02
        params.append(p)
        rhos.append(inputs.sessile_drop(side, side, rl, rg, 0.25 * side))
        muw.append(mu_sat + span * (2 * u[k, 3] - 1))
    return params, rhos, muw


def measure_batch(lbm, inputs, steps):
    params, rhos, muw = batch_workload(lbm, inputs)
    b = lbm.Batch(params, rhos, mu_w_bottom=muw)
    nodes = b.fluid_nodes()
    ty, bpc, ms_tuned = b.tune(trial_steps=10)
    b.step(20)
    n = max(steps // 16, 1) * 16
    t = b.step_timed(n) / 1e3
    b.close()
    return {"workload": "batch of 256 droplet-on-wall cases, side 128-512, CS/PR, Tr 0.6-0.9, f32 storage",
            "fluid_nodes": nodes, "mlups": round(nodes * n / t / 1e6, 1),
            "ms_per_step": round(t / n * 1e3, 4), "tile_y": ty, "blocks_per_cu": bpc,
            "grid": "one workgroup per (case, tile) entry" if bpc < 0 else "%d workgroups per CU, persistent" % bpc,
            "roofline": {"bound": "hbm", "achieved": round(nodes * 72.0 * n / t / 1e9, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(nodes * 72.0 * n / t / 1e9 / PEAK_HBM_GBS, 4),
                         "traffic": traffic_for("step_f32_batch256", ty)}}


def measure_batch_residual(lbm, inputs, max_steps=200000, check_every=2000, window=1000, tol=1e-9):
    """The batching configuration run to its stopping rule: every case in FP64
    storage until max|rho(t) - rho(t - window)| / window < tol (the case then stops),
    diverges, or max_steps pass.  FP32 storage cannot get there: its rounding keeps
    the field moving at a few 1e-8 per step."""
    params, rhos, muw = batch_workload(lbm, inputs)
    for p in params:
        p.prec = lbm.LBM_F64
    b = lbm.Batch(params, rhos, mu_w_bottom=muw)
    nodes = b.fluid_nodes()
    t0 = time.perf_counter()
    done = 0
    while done < max_steps:
        n = min(20000, max_steps - done)
        b.run(n, check_every=check_every, window=window, tol=tol)
        done += n
        st = b.status()["state"]
        print("batch256 FP64 to %.0e: %d steps, %d converged, %d diverged" % (tol, done, (st == 1).sum(),
                                                                               (st == 2).sum()),
              file=sys.stderr, flush=True)
        if (st != 0).all():
            break
    wall = time.perf_counter() - t0
    st = b.status()
    b.close()
    state, steps = st["state"], st["steps"]
    pr = np.array([p.eos == lbm.LBM_EOS_PR for p in params])
    Tr = np.array([p.Tr for p in params])
    conv = state == 1

    def rng(m):
        return [round(float(Tr[m].min()), 3), round(float(Tr[m].max()), 3)] if m.any() else None

    return {"workload": "batch of 256 droplet-on-wall cases, side 128-512, CS/PR, Tr 0.6-0.9, f64 storage, "
                        "run to max|drho| < %.0e per step (window %d, checked every %d steps)" % (tol, window,
                                                                                                check_every),
            "fluid_nodes": nodes, "max_steps": max_steps, "wall_s": round(wall, 1),
            "converged": int(conv.sum()), "diverged": int((state == 2).sum()), "still_running": int((state == 0).sum()),
            "steps_converged_median": float(np.median(steps[conv])) if conv.any() else None,
            "steps_converged_max": int(steps[conv].max()) if conv.any() else None,
            "converged_cs_pr": [int((conv & ~pr).sum()), int((conv & pr).sum())],
            "cases_cs_pr": [int((~pr).sum()), int(pr.sum())],
            "diverged_pr_Tr": rng((state == 2) & pr), "diverged_cs": int(((state == 2) & ~pr).sum()),
            "running_pr_Tr": rng((state == 0) & pr), "running_cs": int(((state == 0) & ~pr).sum())}


def measure_variants(lbm, inputs, steps=100):
    """The force of Eq 5 (pressure tensor) against Eq 12 (chemical potential), and
    the TRT / MRT collisions against BGK, on the 4096^2 FP32 spinodal lattice with
    the one tile shape every variant runs (64 x 16): kernel time per step."""
    variants = [("eq12_bgk", 0), ("eq5_bgk", lbm.LBM_FORCE_PTENSOR), ("eq12_trt", lbm.LBM_COLLIDE_TRT),
                ("eq12_mrt", lbm.LBM_COLLIDE_MRT), ("eq5_mrt", lbm.LBM_FORCE_PTENSOR | lbm.LBM_COLLIDE_MRT)]
    p0, rho0, _, fluid = spinodal_workload(lbm, inputs, lbm.LBM_F32)
    out = {"workload": "force and collision variants, spinodal 4096x4096 VdW Tr=0.85, f32 storage, 64x16 tiles",
           "kernel_us": {}, "mlups": {}, "achieved_gbs": {}, "hbm_bytes": {}}
    traffic = {}
    path = os.path.join(ROOT, "profiles", "traffic_step_f32_variants4096.json")
    if os.path.exists(path):
        d = json.load(open(path))
        if d.get("kernel_sha") == kernel_sha():
            traffic = {k: round((v["fetch_kib_per_dispatch"] * d["fetch_factor"] +
                                 v["write_kib_per_dispatch"] * d["write_factor"]) * 1024.0, 0)
                       for k, v in d.get("variants", {}).items()}
    for name, scheme in variants:
        p = _with_monitor(p0, 0)
        p.scheme = scheme
        lat = lbm.Lattice(p, rho0)
        lat.set_tile(16)
        lat.step(32)
        t = lat.step_timed(steps) / 1e3 / steps
        lat.close()
        out["kernel_us"][name] = round(t * 1e6, 2)
        out["mlups"][name] = round(fluid / t / 1e6, 1)
        out["achieved_gbs"][name] = round(fluid * 72.0 / t / 1e9, 1)
        out["hbm_bytes"][name] = traffic.get(name)
    return out


def measure_d3q19(lbm, inputs, n=256, steps=50):
    """The D3Q19 step on a periodic n^3 box of the spinodal workload (VdW, Tr =
    0.85, tau = 1, kappa = 0.01, rho = 2.6 (1 + 0.01 U)), FP32 storage: 152
    algorithmic bytes per node update (19 loads and 19 stores)."""
    p = lbm.make_params(n, n, lbm.LBM_EOS_VDW, 9 / 49, 2 / 21, 0.85, 1.0, 0.01, prec=lbm.LBM_F32)
    rho0 = inputs.with_relative_noise(np.full((n, n, n), 2.6), 0.01, 3)
    lat = lbm.Lattice3(p, n, rho0)
    lat.step(5)
    t = lat.step_timed(steps) / 1e3 / steps
    lat.close()
    nodes = n ** 3
    return {"workload": "D3Q19 spinodal %d^3 periodic VdW Tr=0.85, f32 storage (one-pass marching step)" % n,
            "mlups": round(nodes / t / 1e6, 1), "ms_per_step": round(t * 1e3, 4),
            "roofline": {"bound": "hbm", "achieved": round(nodes * 152.0 / t / 1e9, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(nodes * 152.0 / t / 1e9 / PEAK_HBM_GBS, 4),
                         "traffic": traffic3_for("step3_f32_d3q19_256")}}


def traffic3_for(workload: str):
    """HBM bytes per D3Q19 step (one launch of the marching kernel) from committed rocprofv3
    FETCH_SIZE / WRITE_SIZE counts, scaled as for the 2-D step, if they were taken on
    the current 3-D kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_sha") != hashlib.sha256(open(KERNEL3_SRC, "rb").read()).hexdigest()[:16]:
        return None
    return round((d["fetch_kib_per_step"] * d["fetch_factor"] + d["write_kib_per_step"] * d["write_factor"]) * 1024.0,
                 0)


PEAK_BF16_TFLOPS = 2500.0      # MI355X dense BF16 MFMA


def surrogate_step_flops(lbm, size, batch):
    """Algorithmic flops of one training step of the surrogate: every 3x3
    convolution costs 2 * 9 * c_in * c_out per output pixel in the forward pass, the
    same again for its weight gradient and, except the first layer (whose input
    needs no gradient), for its input gradient."""
    level = {"0": 0, "1": 1, "2": 2, "3": 3, "u": 0}
    fwd = first = 0.0
    for name, ci, co in lbm.Surrogate.LAYERS:
        lv = level[name[1]]
        f = 2.0 * 9 * ci * co * (size >> lv) ** 2
        fwd += f
        if name == lbm.Surrogate.LAYERS[0][0]:
            first = f
    return batch * (3.0 * fwd - first)


def surrogate_step_floor(lbm, size, batch):
    """Roofline floor of one training step of the surrogate: every pass costs at
    least max(bytes / 8 TB/s, flops / 2.5 PFLOP/s).  Bytes are the pass's own
    operands, BF16 (2 B per channel and pixel) unless stated: a convolution's forward
    pass reads its input and writes its output (the one-channel output in FP32), its
    input gradient reads the output gradient and the ReLU mask (the input) and writes
    the input gradient, its weight gradient reads the input and the output gradient;
    each pooling reads its input and writes a quarter of it, each upsampling the
    reverse; the pooling gradient with the skip share reads three maps and the
    pooled gradient and writes one, the upsampling gradient reads one map and writes
    a quarter of it twice over; the loss reads the prediction and target (FP32) and
    writes the output gradient.  Returns (seconds, bytes)."""
    lv = {"0": 0, "1": 1, "2": 2, "3": 3, "u": 0}
    bw, pk = PEAK_HBM_GBS * 1e9, PEAK_BF16_TFLOPS * 1e12
    t = nbytes = 0.0

    def add(b, f=0.0):
        nonlocal t, nbytes
        t += max(b / bw, f / pk)
        nbytes += b

    first = lbm.Surrogate.LAYERS[0][0]
    for name, ci, co in lbm.Surrogate.LAYERS:
        px = batch * (size >> lv[name[1]]) ** 2
        f = 2.0 * 9 * ci * co * px
        add(px * (2 * ci + (4 if co == 1 else 2) * co), f)     # forward
        if name != first:
            add(px * (2 * co + 4 * ci), f)                       # input gradient
        add(px * 2 * (ci + co), f)                               # weight gradient
    for level, c in ((0, 32), (1, 64), (2, 96)):                 # pooling, skip gradient
        px = batch * (size >> level) ** 2
        add(px * c * 2 + px // 4 * c * 2)
        add(px * c * 2 * 3 + px // 4 * c * 2)
    for level, c in ((2, 128), (1, 96), (0, 64)):                # upsampling and its gradient
        px = batch * (size >> level) ** 2
        add(px // 4 * c * 2 + px * c * 2)
        add(px * c * 2 + px // 4 * c * 2 * 2)
    add(batch * size * size * (4 + 4 + 2))                       # loss
    return t, nbytes


def measure_surrogate(lbm, size=256, batch=16, steps=40):
    """Training steps of the surrogate (BF16 MFMA convolutions, FP32 accumulation)
    on a device-resident synthetic dataset, timed on the host around sur_train."""
    from paper_1611_00907_amd import warmstart
    rng = np.random.default_rng(7)
    n = 4 * batch
    x = rng.normal(size=(n, 4, size, size)).astype(np.float32)
    t = rng.normal(size=(n, size, size)).astype(np.float32)
    net = lbm.Surrogate(size, max_batch=batch)
    net.set_params(warmstart.he_init(3))
    net.set_dataset(x, t)
    net.train(3, batch, 1e-4, seed=1)
    t0 = time.perf_counter()
    net.train(steps, batch, 1e-4, seed=2)
    dt = (time.perf_counter() - t0) / steps
    flops = surrogate_step_flops(lbm, size, batch)
    floor_s, floor_bytes = surrogate_step_floor(lbm, size, batch)
    tf = flops / dt / 1e12
    return {"workload": "surrogate training step: batch %d at %d^2, 4-level U-Net (32-128 channels), BF16 MFMA "
                        "convolutions with FP32 accumulation, Adam" % (batch, size),
            "ms_per_step": round(dt * 1e3, 3), "gflop_per_step": round(flops / 1e9, 1),
            "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / PEAK_BF16_TFLOPS, 5), "traffic": None},
            # per pass max(bytes at the HBM peak, flops at the BF16 peak), summed
            "step_floor": {"ms": round(floor_s * 1e3, 4), "bytes": round(floor_bytes, 0),
                           "frac": round(floor_s / dt, 4)}}


def traffic_for(workload: str, shape: int):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE / WRITE_SIZE counts of
    this launch shape, each scaled by what the counter reads for a plain copy of known
    size, if they were taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    rec = d.get("shapes", {}).get("march" if shape < 0 else str(shape))  # marching: all k together
    if d.get("kernel_sha") != kernel_sha() or rec is None:
        return None
    return round((rec["fetch_kib_per_dispatch"] * d["fetch_factor"] +
                  rec["write_kib_per_dispatch"] * d["write_factor"]) * 1024.0, 0)


def _with_monitor(p, every):
    q = type(p)()
    for name, _ in p._fields_:
        setattr(q, name, getattr(p, name))
    q.monitor_every = every
    return q


def measure(lbm, p, rho0, mu_w, fluid_nodes, steps, warmup, bytes_per_lu, workload, kernel_steps=None):
    """Times the step with HIP events on the lattice's own stream (lbm_step_timed).

    Whole step: exactly `steps` fused updates with the monitors every
    min(MONITOR_EVERY, steps) steps.  Kernel: `kernel_steps` (default
    max(steps, 1000)) back-to-back fused updates without monitors, on a second
    lattice of the same state, for the roofline.  The library captures the HIP
    graph that the steps replay before its first event, so capture and
    instantiation are never inside a timed interval.  The whole-step lattice does
    its warm-up steps first and is timed right after the kernel measurement, so
    that both intervals see the GPU at its sustained clocks (a short window timed
    after the host-side set-up of a fresh lattice reads about 5 % slower)."""
    def lattice(every, shape=None):
        lat = lbm.Lattice(_with_monitor(p, every), rho0)
        if mu_w is not None:
            lat.set_wall_mu(0, mu_w)
        if shape is not None:
            lat.set_tile(shape)
        lat.step(warmup)
        return lat

    # launch shape from the library's tuner (tiles of several widths, column marching)
    lat = lattice(0)
    shape, _ = lat.tune(trial_steps=60)
    lat.close()
    # whole step (fused update plus the monitors): its lattice and warm-up steps first
    every = min(MONITOR_EVERY, steps)
    lat_w = lattice(every, shape)
    lat_w.step_timed(0)  # waits for the warm-up steps
    # kernel only: back-to-back fused steps, no monitors
    lat = lattice(0, shape)
    k_steps = kernel_steps if kernel_steps is not None else max(steps, 1000)
    t_kernel = lat.step_timed(k_steps) / 1e3 / k_steps
    # then the whole-step window
    t_total = lat_w.step_timed(steps) / 1e3
    mon = lat_w.monitors()
    lat.close()
    lat_w.close()
    achieved = fluid_nodes * bytes_per_lu / t_kernel / 1e9
    traffic = traffic_for(workload, shape)
    return {
        "mlups": fluid_nodes * steps / t_total / 1e6,
        "ms_per_step": t_total / steps * 1e3,
        "steps": steps,
        "monitor_every": every,
        "kernel_steps": k_steps,
        "kernel_us": t_kernel * 1e6,
        "shape": shape,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic},
        "monitor": {"mass": mon["mass"], "residual": mon["residual"], "flags": mon["flags"]},
    }


WARMSTART_RECORD = os.path.join(ROOT, "profiles", "warmstart_c5.json")
WARMSTART_KEYS = ("n_cases", "side", "usable", "loss_first", "loss_last", "val_mse", "sweep_s_cold", "sweep_s_warm",
                  "inference_s", "speedup", "speedup_calibration_only", "masked_sweep_s_cold", "masked_sweep_s_warm",
                  "speedup_masked", "speedup_masked_calibration_only", "steps_saved_median",
                  "theta_pred_abs_err_median", "training_s", "generation_s", "converged", "generation_storage",
                  "steps_mean_all", "steps_mean_resolved", "steps_mean_sub_grid", "sweep_resolved",
                  "sweep_sub_grid")


def warmstart_summary(live: bool):
    """Time to the plain equilibrium contact angle (within 0.5 deg) of a batched sweep of
    100 held-out 256^2 cases, cold start vs the surrogate's warm start.  Run live with
    --warmstart (several minutes); otherwise the record of the last full run, marked as
    such, with the command that made it."""
    if live:
        from paper_1611_00907_amd import warmstart
        r = warmstart.run_experiment(log=lambda m: print(m, file=sys.stderr, flush=True))
        out = {k: r[k] for k in WARMSTART_KEYS if k in r}
        out["measured_in_this_run"] = True
        out["source"] = "measured in this run"
        return out
    if not os.path.exists(WARMSTART_RECORD):
        return None
    r = json.load(open(WARMSTART_RECORD))
    out = {k: r[k] for k in WARMSTART_KEYS if k in r}
    out["measured_in_this_run"] = False
    out["source"] = "not measured in this run; record of profiles/warmstart_c5.json (%s)" % r.get("command", "")
    return out


def cpu_baseline(seconds: float, workload: str):
    """The FP64 oracle on the main workload, timed on the host cores for about
    `seconds` (a bounded sample of steps of the same lattice)."""
    from oracle import thermo
    from oracle.lattice import CPWALL, NEUTRAL, OracleLattice, OracleParams, max_threads
    from paper_1611_00907_amd import inputs

    if workload == "wetting1024":
        nx = ny = 1024
        op = OracleParams.from_reduced(nx, ny, thermo.PR, 2 / 49, 2 / 21, 0.8, 1.3, 0.01, omega=0.344,
                                       bottom=CPWALL, top=NEUTRAL)
        rg, rl, _, mu_sat = thermo.maxwell(op.fluid())
        mu_w = float(inputs.draw_uniform(2, mu_sat - 0.18, mu_sat + 0.23, 1)[0])  # the GPU workload's wall
        ora = OracleLattice(op, inputs.sessile_drop(nx, ny, rl, rg, 200.0), mu_w_bottom=mu_w)
        fluid, name = nx * (ny - 2), "1024x1024 wetting workload"
    else:
        n = 4096
        op = OracleParams.from_reduced(n, n, thermo.VDW, 9 / 49, 2 / 21, 0.85, 1.0, 0.01)
        ora = OracleLattice(op, inputs.with_relative_noise(np.full((n, n), 2.6), 0.01, 3))
        fluid, name = n * n, "4096x4096 spinodal workload"
    t1 = ora.timed_steps(1)
    n_steps = max(2, int(seconds / max(t1, 1e-6)))
    t = ora.timed_steps(n_steps)
    return {"value": round(fluid * n_steps / t / 1e6, 3), "unit": "MLUPS", "cores": max_threads(),
            "kind": "oracle",
            "sample": "%d steps of the %s in FP64 (%.1f s)" % (n_steps, name, t)}


SPINODAL_CONFIG = {"workload": "spinodal 4096x4096 D2Q9, VdW a=9/49 b=2/21, Tr=0.85, tau=1, kappa=0.01, "
                               "periodic, rho = 2.6 (1 + 0.01 U(-1,1)), FP32 storage; HBM-bound (1.2 GB per step)",
                   "nx": 4096, "ny": 4096, "storage": "f32", "parallelism": "single GPU"}
WETTING_CONFIG = {"workload": "wetting 1024x1024 D2Q9, PR omega=0.344 Tr=0.8, tau=1.3, kappa=0.01, "
                              "CP wall + neutral top, drop R=200, FP32 storage; cache-resident (75 MB per step "
                              "inside the 256 MB Infinity Cache)",
                  "nx": 1024, "ny": 1024, "storage": "f32", "parallelism": "single GPU"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (requested --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    from paper_1611_00907_amd import inputs, lbm

    lbm.load_library()
    if args.surrogate_only > 0:
        print(json.dumps(measure_surrogate(lbm, steps=args.surrogate_only)), flush=True)
        return

    copy_gbs = lbm.lbm_copy_bandwidth(args.copy_bytes, 20)
    print("copy: %.1f GB/s over %d bytes" % (copy_gbs, args.copy_bytes), file=sys.stderr, flush=True)
    dtype = "f32"
    if args.workload == "batch256":
        res = measure_batch(lbm, inputs, args.steps)
        print(json.dumps({"workload": "batch256", "aux": [res]}), flush=True)
        return
    if args.workload == "batch256_residual":
        print(json.dumps(measure_batch_residual(lbm, inputs)), flush=True)
        return
    if args.workload == "variants":
        print(json.dumps({"workload": "variants", "aux": [measure_variants(lbm, inputs, steps=args.steps)]}),
              flush=True)
        return
    if args.workload == "d3q19":
        print(json.dumps({"workload": "d3q19", "aux": [measure_d3q19(lbm, inputs, steps=args.steps)]}), flush=True)
        return
    if args.workload == "spinodal4096":
        p, rho0, mu_w, fluid = spinodal_workload(lbm, inputs, lbm.LBM_F32)
        config, bpl, wname = dict(SPINODAL_CONFIG), 72.0, "step_f32_spinodal4096"
    elif args.workload == "wetting1024":
        p, rho0, mu_w, fluid = wetting_workload(lbm, inputs, lbm.LBM_F32)
        config, bpl, wname = dict(WETTING_CONFIG), 72.0, "step_f32_wetting1024"
    else:
        dtype = args.workload.split("_")[1]
        prec = lbm.LBM_F16DEV if dtype == "f16dev" else lbm.LBM_BF16DEV
        p, rho0, mu_w, fluid = spinodal_workload(lbm, inputs, prec)
        config = dict(SPINODAL_CONFIG, storage=dtype,
                      workload=SPINODAL_CONFIG["workload"].replace("FP32 storage", "%s storage" % dtype))
        bpl, wname = 36.0, "step_%s_spinodal4096" % dtype
    main_res = measure(lbm, p, rho0, mu_w, fluid, args.steps, args.warmup, bpl, wname)
    config["monitor_every"] = main_res["monitor_every"]
    print("main: %.1f MLUPS, step %.2f us, kernel %.2f us, %.1f GB/s" % (
        main_res["mlups"], main_res["ms_per_step"] * 1e3, main_res["kernel_us"], main_res["roofline"]["achieved"]),
        file=sys.stderr, flush=True)

    aux = []
    if not args.no_aux:
        if args.workload != "wetting1024":
            pp, r0, mw, fl = wetting_workload(lbm, inputs, lbm.LBM_F32)
            res = measure(lbm, pp, r0, mw, fl, 1000, 100, 72.0, "step_f32_wetting1024")
            aux.append({"workload": WETTING_CONFIG["workload"], "mlups": round(res["mlups"], 1),
                        "ms_per_step": round(res["ms_per_step"], 5), "kernel_us": round(res["kernel_us"], 2),
                        "shape": res["shape"], "roofline": res["roofline"]})
            print("aux f32 wetting1024: %.1f MLUPS %.1f GB/s" % (res["mlups"], res["roofline"]["achieved"]),
                  file=sys.stderr, flush=True)
        for prec, name, b in ((lbm.LBM_F16DEV, "f16dev", 36.0), (lbm.LBM_BF16DEV, "bf16dev", 36.0)):
            if args.workload.endswith(name):
                continue
            pp, r0, _, fl = spinodal_workload(lbm, inputs, prec)
            res = measure(lbm, pp, r0, None, fl, 300, 20, b, "step_%s_spinodal4096" % name)
            aux.append({"workload": "spinodal 4096x4096 VdW Tr=0.85, %s storage (deviations from w_i 2.6)" % name,
                        "mlups": round(res["mlups"], 1), "kernel_us": round(res["kernel_us"], 2),
                        "shape": res["shape"], "roofline": res["roofline"]})
            print("aux %s: %.1f MLUPS %.1f GB/s" % (name, res["mlups"], res["roofline"]["achieved"]),
                  file=sys.stderr, flush=True)
        res = measure_variants(lbm, inputs)
        aux.append(res)
        print("aux variants: %s us" % res["kernel_us"], file=sys.stderr, flush=True)
        res = measure_d3q19(lbm, inputs)
        aux.append(res)
        print("aux d3q19: %.1f MLUPS %.1f GB/s" % (res["mlups"], res["roofline"]["achieved"]), file=sys.stderr,
              flush=True)
        res = measure_batch(lbm, inputs, 320)
        aux.append(res)
        print("aux batch: %.1f MLUPS %.1f GB/s (tile %d, %s)" % (res["mlups"], res["roofline"]["achieved"],
                                                                res["tile_y"], res["grid"]),
              file=sys.stderr, flush=True)
        res = measure_surrogate(lbm)
        aux.append(res)
        print("aux surrogate: %.2f ms/step %.2f TFLOP/s" % (res["ms_per_step"], res["roofline"]["achieved"]),
              file=sys.stderr, flush=True)

    line = {
        "metric": "MLUPS + % HBM roofline; time-to-equilibrium (surrogate vs plain) at 0.5deg",
        "value": round(main_res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": main_res["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
        "roofline": main_res["roofline"],
        "kernel_us": round(main_res["kernel_us"], 3),
        "kernel_steps": main_res["kernel_steps"],
        "shape": main_res["shape"],
        "copy_kernel": {"bytes": args.copy_bytes, "gbs": round(copy_gbs, 1),
                        "step_frac_of_copy": round(main_res["roofline"]["achieved"] / copy_gbs, 4)},
        "aux": aux,
    }
    ws = warmstart_summary(args.warmstart)
    if ws is not None:
        line["warm_start"] = ws
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, "wetting1024" if args.workload == "wetting1024"
                                            else "spinodal4096")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
