"""Host-side checks of bench.py (CPU): the one-GPU guard and the counter
traffic lookup that feeds the roofline's `traffic` field."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_lookup_matches_the_committed_counter_summary(monkeypatch):
    import re

    sys.path.insert(0, ROOT)
    sys.path.insert(0, os.path.join(ROOT, "paper_2404_17133_amd"))
    import bench
    import profsum

    text = open(os.path.join(ROOT, "profiles", "exch_contractions_c2_mixed_hbm_traffic.md")).read()
    taken = re.search(r"GEMM source hash: (\w+)", text).group(1)
    # with the GEMM source the counters were taken with, the summary's
    # dispatch-weighted bytes per launch are reported
    monkeypatch.setattr(profsum, "gemm_source_hash", lambda: taken)
    t = bench.measured_traffic("exch_w", "f32", "c2")
    assert t is not None and t > 0
    # more than the 0.37 GB of algorithmic bytes per launch, less than 3 GB
    assert 0.37e9 < t < 3e9
    assert bench.measured_traffic("exch_w", "f32", "c1") is None  # only the no=200 workload was counted
    assert bench.measured_traffic("no_such_family", "f32", "c2") is None
    # once the GEMM source changes, the old counters no longer describe it
    monkeypatch.setattr(profsum, "gemm_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("exch_w", "f32", "c2") is None


def test_stored_bench_line_keeps_the_contract():
    """The committed no=200 bench line (written by a GPU run of bench.py) has
    every field of the one-line JSON contract, a roofline of the dominant
    kernel whose fraction is achieved / peak, and a CPU baseline of the
    oracle; the values are consistent with each other."""
    import json

    line = json.load(open(os.path.join(ROOT, "profiles", "exch_contractions_c2_mixed_bench_line.json")))["line"]
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in line, key
    assert line["n_gpus"] == 1 and line["higher_is_better"] is True and line["data"] == "synthetic"
    assert "workload" in line["config"]
    # value = solutions per second over the timed steps
    per_step = line["config"]["roots_per_step"]
    assert abs(line["value"] - per_step / (line["ms_per_step"] / 1000.0)) < 1e-3 * line["value"]
    rf = line["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in rf, key
    assert rf["bound"] in ("hbm", "mfma", "alu") and rf["peak"] == 157.3 and rf["unit"] == "TFLOP/s"
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    # achieved = algorithmic flops per launch over the measured launch time
    assert abs(rf["achieved"] - rf["flops_per_launch"] / (rf["avg_launch_ms"] * 1e-3) / 1e12) < 0.01 * rf["achieved"]
    cb = line["cpu_baseline"]
    for key in ("value", "unit", "cores", "kind", "sample"):
        assert key in cb, key
    assert cb["kind"] == "oracle" and cb["unit"] == line["unit"] and cb["cores"] >= 1
