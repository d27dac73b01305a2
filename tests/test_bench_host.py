"""bench.py on the host (no GPU): the one-GPU contract and the timing
summary helper."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_distribution_summary():
    sys.path.insert(0, ROOT)
    import bench
    d = bench.distribution([2.0, 1.0, 3.0, 2.0], np)
    assert d["n"] == 4 and d["median"] == 2.0 and d["mean"] == 2.0
    # Student-t 95% half width: t(0.975, 3) * s / sqrt(n), s = sqrt(2/3)
    assert abs(d["ci95_half_width"] - 3.182446 * np.sqrt(2.0 / 3.0) / 2.0) < 1e-3
    assert d["p5_p25_p75_p95"][0] <= d["p5_p25_p75_p95"][-1]
