"""The benchmark's JSON line: one short run of the default workload, checked
for the fields and relations its readers rely on."""
import json
import os
import subprocess
import sys

import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line():
    say("case: bench.py --steps 20 --warmup 5 (autotuned; no baselines, compare or adjoint)")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "20",
                        "--warmup", "5", "--no-cpu-baseline", "--no-compare", "--no-adjoint"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    b = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "value_without_sampling"):
        assert k in b, k
    assert b["n_gpus"] == 1 and b["steps"] == 20 and b["warmup"] == 5
    assert b["dtype"] == "f32" and b["data"] == "synthetic" and b["higher_is_better"]
    nodes = b["config"]["nodes"]
    assert nodes == 4177920 and b["config"]["workload"] == "batched96"
    # value is the whole batch's node updates per second over the timed steps
    assert b["value"] == pytest.approx(nodes / (b["ms_per_step"] * 1e3), rel=1e-3)
    rf = b["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    spl = rf["steps_per_launch"]
    assert spl in (1, 2) and b["config"]["steps_per_launch"] == spl
    assert rf["algorithmic_bytes_per_launch"] == 144 * nodes * spl
    assert rf["achieved"] == pytest.approx(
        rf["algorithmic_bytes_per_launch"] / (rf["launch_ms"] * 1e-3) / 1e9, rel=1e-3)
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], abs=1e-4)
    # a two-step launch moves about half its algorithmic bytes, so its
    # algorithmic rate may pass the plain copy's up to about twice over
    assert 0 < rf["frac"] < 1 and 0 < rf["frac_of_copy"] < 1.2 * spl
    # steady state even at 20 steps after 5: the graphs the timed steps replay
    # were captured before the timing began, so a step costs the step kernel
    # plus the sampling's share (about 8% at one sample in 10), not a capture
    assert b["ms_per_step"] <= 1.2 * rf["launch_ms"] / spl, (b["ms_per_step"], rf["launch_ms"])
    assert b["value_without_sampling"] >= b["value"]
    say(f"  value {b['value']} MLUPS, launch {rf['launch_ms'] * 1e3:.1f} us ({spl} steps), "
        f"frac {rf['frac']}")
