"""bench.py runs on one GPU only: other GPU counts exit with a message
before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_worker_times_oracle_steps():
    """The CPU-baseline worker builds a nested sample of the realistic
    recipe and times oracle steps on it (tiny sample here)."""
    sys.path.insert(0, ROOT)
    import bench
    secs, n, its = bench._oracle_sample_worker((40, 1, 2, 1))
    assert secs > 0 and n > 40 and len(its) == 1 and its[0] >= 1


def test_per_field_errors():
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    ref = np.arange(1, 21, dtype=float).reshape(4, 5)
    u = ref.copy()
    u[2, 1] += 0.5
    e = bench.per_field_errors(u, ref)
    assert e["S"]["linf_rel"] == 0.0 and e["E"]["linf_rel"] == 0.5 / 17.0
    assert abs(e["E"]["l2_rel"] - 0.5 / np.linalg.norm(ref[:, 1])) < 1e-15
