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


def test_traffic_lookup_matches_the_committed_counter_summary():
    sys.path.insert(0, ROOT)
    import bench

    t = bench.measured_traffic("exch_w", "f32", "c2")
    # the committed summary was taken with the GEMM source as it stands
    assert t is not None and t > 0
    # about 1.7 GB per launch against 0.37 GB of algorithmic bytes
    assert 1e9 < t < 3e9
    assert bench.measured_traffic("exch_w", "f32", "c1") is None  # only the no=200 workload was counted
    assert bench.measured_traffic("no_such_family", "f32", "c2") is None
