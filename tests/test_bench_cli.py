"""bench.py's command-line contract that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_record_only_for_the_measured_source():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.measured_traffic("power_fused", "dense-100^4 bf16") is None
    assert bench.measured_traffic("sketch_fused", "dense-200^4 bf16") is None
