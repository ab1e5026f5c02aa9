"""bench.py end to end on a small box: the JSON line's keys and their consistency, for the
nearest-neighbour and the octilateral current (Sec. 2.2, 2.3).  GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.gpu


def _bench(*args):
    print("bench.py", *args, flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    return json.loads(lines[0])


def _check_line(d, steps, warmup):
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d
    assert d["n_gpus"] == 1 and d["steps"] == steps and d["warmup"] == warmup
    assert d["higher_is_better"] is True and d["data"] == "synthetic" and d["dtype"] == "f64"
    nodes = 1
    for n in d["config"]["grid"]:
        nodes *= n
    # value is the whole-job rate: nodes x steps over the timed wall time
    assert d["value"] == pytest.approx(nodes / (d["ms_per_step"] * 1e-3), rel=1e-6)
    rf = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"])
    assert 0.0 < rf["frac"] < 1.0
    assert "workload" in d["config"]


def test_bench_line_nearest_neighbour_both_precisions():
    d = _bench("--n", "64", "--steps", "3", "--warmup", "1", "--no-cpu-baseline", "--no-adjoint")
    _check_line(d, 3, 1)
    assert "Sec. 2.2" in d["config"]["current"]
    mm = d["fp32_mixed"]
    assert mm["value"] > 0 and mm["dtype"] == "f64+f32"
    acc = mm["accuracy_vs_fp64_fixed_dt"]
    assert acc["final_E_M_rel"] < 1e-5


def test_bench_line_octilateral():
    d = _bench("--n", "64", "--steps", "3", "--warmup", "1", "--no-cpu-baseline", "--curl", "nnn")
    _check_line(d, 3, 1)
    assert "Sec. 2.3" in d["config"]["current"]
    assert "octilateral" in d["roofline"]["kernel"]
    assert "fp32_mixed" not in d and "adjoint" not in d
