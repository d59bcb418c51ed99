"""bench.py keeps its command-line contract (runs without a GPU up to the device check)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_has_main_and_refuses_several_gpus():
    sys.path.insert(0, ROOT)
    import bench
    assert callable(bench.main)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one MI355X" in r.stderr
