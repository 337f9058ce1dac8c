"""Host-side pieces of bench.py: the one-GPU guard and the all-cores oracle
leg (worker processes started together), run on the CPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_all_cores_oracle_leg():
    sys.path.insert(0, ROOT)
    import bench

    r = bench.cpu_all_cores(2, 0.2)
    assert r["cores"] == 2 and r["unit"] == "Mpix/s"
    # each worker finishes at least one frame after the go line
    assert r["frames_per_s"] > 0 and r["value"] > 0
    assert "2 single-threaded oracle processes" in r["sample"]
