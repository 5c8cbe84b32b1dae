"""Host-side checks of bench.py (no GPU): the single-GPU contract and the
committed HBM traffic figure of the bulk sweep."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "single-GPU" in out["error"]


def test_committed_traffic_matches_the_bulk_kernel_source():
    """The rocprofv3 traffic figure is reported only while k_bulk's source is
    the one it was measured on; this fails when the kernel changes without
    the counters being taken again."""
    import bench
    t = bench.measured_traffic("batch", 1024)
    assert t is not None and t > 0
    assert bench.measured_traffic("bubble", 1024) is None
    assert bench.measured_traffic("batch", 512) is None
