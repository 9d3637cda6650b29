"""The benchmark's one-line JSON record: required keys, units and the roofline
object, on a small Quantum-Volume run (24 qubits, library defaults); its refusal
of several GPUs; and the committed traffic profile it reads."""

import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_bench_json_line():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "24", "--steps", "1", "--warmup", "1",
           "--autotune", "off", "--skip-cpu"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["warmup"] == 1
    assert d["unit"] == "GB/s" and d["value"] > 0 and d["higher_is_better"] is True
    assert d["dtype"] == "f64" and "24q c128" in d["metric"]
    rf = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    assert rf["bound"] in ("hbm", "alu") and 0 < rf["frac"] < 1
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert d["parity"]["one_minus_F_blocked_vs_pergate"] < 1e-12


def test_bench_refuses_several_gpus():
    """Asking for more than one GPU exits with a message before touching a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_traffic_profile_matches_sources():
    """The committed PMC traffic profile of the headline kernel was taken on the
    current section-kernel sources (the benchmark reports it as roofline.traffic
    only then), and its figures agree with one another."""
    spec = importlib.util.spec_from_file_location("bench_for_test", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    with open(bench.PROFILE_TRAFFIC) as f:
        prof = json.load(f)
    assert prof["kernel_source_hash"] == bench.kernel_source_hash()
    scaled = 1024.0 * (prof["fetch_kib_per_dispatch"] * prof["fetch_scale"]
                       + prof["write_kib_per_dispatch"] * prof["write_scale"])
    assert abs(scaled - prof["bytes_per_launch"]) <= 1e-9 * scaled
    algorithmic = 2 * (1 << prof["n"]) * 16  # one read and one write of the complex128 state
    assert prof["algorithmic_bytes_per_launch"] == algorithmic
    assert abs(prof["ratio_to_algorithmic"] - scaled / algorithmic) < 1e-9
    assert 1.0 <= prof["ratio_to_algorithmic"] < 1.05
