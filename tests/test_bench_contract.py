"""Host-side checks of the benchmark script's contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes_per_query():
    """A(Q) = sum_i DF(q_i) * (4 + s) + 16 |Q| + 8 k, positions counted with multiplicity."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    df = np.array([5, 0, 7, 100], np.int64)
    q_ids = np.array([0, 2, 2, 3, 1], np.int32)
    q_off = np.array([0, 3, 3, 5], np.int64)
    k = np.array([10, 1, 100])
    got = bench.algorithmic_bytes(df, q_ids, q_off, k, 2)
    want = [(5 + 7 + 7) * 6 + 16 * 3 + 80, 8, (100 + 0) * 6 + 32 + 800]
    assert list(got) == want
