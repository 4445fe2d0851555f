"""CPU: the host-side pieces of bench.py (flop count of the surrogate's training
step, the counter-traffic lookup, the one-GPU guard and the CPU-baseline record)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1611_00907_amd import lbm  # noqa: E402


def test_surrogate_step_flops_by_hand():
    """Resolutions written out level by level (encoder 0..3, decoder 2..0, output at
    full size), independent of the layer-name parsing in bench.py."""
    size, batch = 64, 3
    res = {"e0a": 64, "e0b": 64, "e1a": 32, "e1b": 32, "e2a": 16, "e2b": 16, "e3a": 8, "e3b": 8,
           "d2a": 16, "d2b": 16, "d1a": 32, "d1b": 32, "d0a": 64, "d0b": 64, "out": 64}
    fwd = {name: 2 * 9 * ci * co * res[name] ** 2 for name, ci, co in lbm.Surrogate.LAYERS}
    want = batch * (3 * sum(fwd.values()) - fwd["e0a"])
    assert bench.surrogate_step_flops(lbm, size, batch) == pytest.approx(want, rel=1e-12)


def test_surrogate_step_flops_at_the_benchmark_size():
    assert bench.surrogate_step_flops(lbm, 256, 16) / 1e9 == pytest.approx(789.4, abs=0.05)


def test_traffic_lookup_follows_the_kernel_source(monkeypatch):
    assert bench.traffic_for("no_such_workload", 32) is None
    path = os.path.join(ROOT, "profiles", "traffic_step_f32_wetting1024.json")
    d = json.load(open(path))
    shape = next(k for k in d["shapes"] if k != "march")
    monkeypatch.setattr(bench, "kernel_sha", lambda: d["kernel_sha"])
    got = bench.traffic_for("step_f32_wetting1024", int(shape))
    rec = d["shapes"][shape]
    want = (rec["fetch_kib_per_dispatch"] * d["fetch_factor"] + rec["write_kib_per_dispatch"] * d["write_factor"]) * 1024
    assert got == pytest.approx(want, abs=1.0)
    # counters taken on another kernel source are not reported
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0" * 16)
    assert bench.traffic_for("step_f32_wetting1024", int(shape)) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_baseline_record():
    rec = bench.cpu_baseline(0.2, "wetting1024")
    assert rec["kind"] == "oracle" and rec["unit"] == "MLUPS"
    assert rec["cores"] >= 1 and rec["value"] > 0
    assert "1024x1024 wetting workload" in rec["sample"]


def test_cpu_baseline_record_spinodal():
    rec = bench.cpu_baseline(0.5, "spinodal4096")
    assert rec["kind"] == "oracle" and rec["value"] > 0
    assert "4096x4096 spinodal workload" in rec["sample"]


class _FakeLattice:
    """Stands in for lbm.Lattice: records what the bench asks of it."""
    log = []

    def __init__(self, p, rho0):
        self.every = p.monitor_every
        _FakeLattice.log.append(("new", self.every))

    def set_wall_mu(self, wall, mu):
        pass

    def set_tile(self, shape):
        _FakeLattice.log.append(("tile", shape))

    def step(self, n):
        _FakeLattice.log.append(("step", n))

    def tune(self, trial_steps):
        return 25608, 0.25

    def step_timed(self, n):
        _FakeLattice.log.append(("timed", n, self.every))
        return 0.25 * n  # ms

    def monitors(self):
        return {"mass": 1.0, "residual": 0.0, "flags": 0}

    def close(self):
        pass


class _FakeLbm:
    Lattice = _FakeLattice


@pytest.mark.parametrize("steps,warmup", [(20, 5), (1000, 100), (7, 0)])
def test_measure_times_exactly_the_requested_steps(steps, warmup):
    """The whole-step interval covers exactly --steps steps with monitors every
    min(100, steps) steps and comes right after the kernel interval (no monitors,
    max(steps, 1000) steps); warm-up runs on every lattice before its timed interval
    (a zero-step timed call only waits for the warm-up)."""
    _FakeLattice.log = []
    p = lbm.make_params(64, 64, lbm.LBM_EOS_VDW, 9 / 49, 2 / 21, 0.85, 1.0, 0.01)
    res = bench.measure(_FakeLbm, p, None, None, 4096 * 4096, steps, warmup, 72.0, "no_such_workload")
    timed = [e for e in _FakeLattice.log if e[0] == "timed" and e[1] > 0]
    assert len(timed) == 2
    assert timed[-1] == ("timed", steps, min(100, steps))
    assert timed[0][2] == 0 and timed[0][1] == max(steps, 1000)
    i_k, i_w = (i for i, e in enumerate(_FakeLattice.log) if e in timed)
    assert i_w == i_k + 1
    assert res["steps"] == steps and res["monitor_every"] == min(100, steps)
    assert res["ms_per_step"] == pytest.approx(0.25)
    assert res["kernel_us"] == pytest.approx(250.0)
    assert res["roofline"]["frac"] == pytest.approx(4096 * 4096 * 72 / 250e-6 / 1e9 / 8000.0, rel=1e-3)
    # every lattice warms up before it is timed
    for i, e in enumerate(_FakeLattice.log):
        if e[0] == "timed":
            assert ("step", warmup) in _FakeLattice.log[:i]


def test_surrogate_step_floor_by_hand():
    """The step floor at a small size, pass by pass written out: 2-D maps of
    side s >> level, BF16 operands, each pass at max(bytes / 8 TB/s, flops / 2.5
    PFLOP/s); independent of bench.py's layer-name parsing."""
    size, batch = 32, 2
    res = {"e0a": 32, "e0b": 32, "e1a": 16, "e1b": 16, "e2a": 8, "e2b": 8, "e3a": 4, "e3b": 4,
           "d2a": 8, "d2b": 8, "d1a": 16, "d1b": 16, "d0a": 32, "d0b": 32, "out": 32}
    bw, pk = 8e12, 2.5e15
    t = b_all = 0.0
    for name, ci, co in lbm.Surrogate.LAYERS:
        px = batch * res[name] ** 2
        f = 18.0 * ci * co * px
        out_b = 4 * co if name == "out" else 2 * co
        passes = [px * (2 * ci + out_b), px * 2 * (ci + co)] + ([] if name == "e0a" else [px * (2 * co + 4 * ci)])
        for b in passes:
            t += max(b / bw, f / pk)
            b_all += b
    for side, c in ((32, 32), (16, 64), (8, 96)):
        px = batch * side * side
        for b in (px * c * 2 + px // 4 * c * 2, px * c * 6 + px // 4 * c * 2):
            t += b / bw
            b_all += b
    for side, c in ((8, 128), (16, 96), (32, 64)):
        px = batch * side * side
        for b in (px // 4 * c * 2 + px * c * 2, px * c * 2 + px // 4 * c * 4):
            t += b / bw
            b_all += b
    b = batch * 32 * 32 * 10
    t += b / bw
    b_all += b
    got_t, got_b = bench.surrogate_step_floor(lbm, size, batch)
    assert got_t == pytest.approx(t, rel=1e-12) and got_b == pytest.approx(b_all, rel=1e-12)


def test_surrogate_step_floor_at_the_benchmark_size():
    t, b = bench.surrogate_step_floor(lbm, 256, 16)
    assert t * 1e3 == pytest.approx(0.658, abs=0.001) and b / 1e9 == pytest.approx(5.03, abs=0.01)


def test_warm_start_record_names_the_command_that_made_it():
    """The bench line cites the committed warm-start record when the experiment is not
    rerun; the citation carries the record's own command, which reruns it."""
    out = bench.warmstart_summary(False)
    assert out is not None and out["measured_in_this_run"] is False
    cmd = json.load(open(bench.WARMSTART_RECORD))["command"]
    assert cmd.startswith("python -m paper_1611_00907_amd.warmstart ")
    assert out["source"].endswith("(%s)" % cmd)
