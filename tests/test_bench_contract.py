"""bench.py's output contract: one JSON line on stdout with the fields its readers
rely on (metric, value and unit; the step count and time; the workload; the
roofline object of the timed kernel; the CPU baseline of the oracle).  The refusal
of several GPUs runs on the CPU; the JSON line itself needs a GPU."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused_before_touching_a_gpu():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.gpu
def test_json_line_carries_the_contract_fields():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    print("case bench.py --steps 200 --warmup 20 --no-secondary --no-accuracy", flush=True)
    r = subprocess.run([sys.executable, "-u", BENCH, "--steps", "200", "--warmup", "20", "--no-secondary",
                        "--no-accuracy", "--cpu-seconds", "2"], capture_output=True, text=True, timeout=300,
                       cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 200 and d["warmup"] == 20
    assert d["unit"] == "MLUPS" and d["higher_is_better"] is True and d["dtype"] == "f64"
    assert d["data"] == "synthetic" and d["vs_baseline"] is None
    nodes = 512 * 512
    assert d["config"]["workload"].startswith("D2Q9 512x512") and d["config"]["nodes"] == nodes
    assert d["config"]["stores"] in ("streaming", "device")
    # value: lattice updates per second of the timed steps; achieved: 144 B per update (float64 D2Q9)
    assert d["value"] == pytest.approx(nodes / (d["ms_per_step"] * 1e-3) / 1e6, rel=1e-9)
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["achieved"] == pytest.approx(144 * nodes / (d["ms_per_step"] * 1e-3) / 1e9, rel=1e-9)
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], rel=1e-12)
    assert rf["traffic"] is None or rf["traffic"] > 144 * nodes
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["unit"] == "MLUPS" and cb["cores"] >= 1 and cb["value"] > 0
    assert "512x512" in cb["sample"]
