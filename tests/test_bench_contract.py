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


def test_launch_work_counts():
    """Unique rows, method additions and issued operations of a launch on a hand-counted batch:
    N = 32 documents, so rows with DF >= 2 are dense (padded to 4096 documents, 2-byte values)."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    df = np.array([20, 1, 3, 0], np.int64)
    q_ids = np.array([0, 0, 1, 2], np.int32)       # query 0 = [0, 0, 1], query 1 = [2]
    q_off = np.array([0, 3, 4], np.int64)
    w = bench.launch_work(df, q_ids, q_off, 10, 32, 2)
    assert w["unique_bytes"] == 2 * 4096 * 2 + 1 * 6 + 16 * 4 + 8 * 10 * 2
    assert w["method_adds"] == 20 + 20 + 1 + 3
    assert w["dense_fmas"] == 2 * 32          # (query 0, token 0) and (query 1, token 2)
    assert w["sparse_adds"] == 1              # (query 0, token 1)
    assert w["select_ops"] == 2 * 32
    assert w["issued_ops"] == 64 + 1 + 64


def test_roofline_names_the_binding_bound():
    """The bound with the longest lower-bound time sets bound, achieved and frac; every frac is
    that bound's time over the kernel time."""
    sys.path.insert(0, ROOT)
    import bench
    work = dict(unique_bytes=8e9, method_adds=1e12, select_ops=0.0, issued_ops=3.93e12)
    r = bench.roofline(work, kernel_ms=400.0, traffic=1.6e12, no_reuse_bytes=1e13)
    # traffic: 200 ms at 8 TB/s; issued: 100 ms at 39.3 T/s; unique rows: 1 ms
    assert r["binding"] == "hbm_traffic" and r["bound"] == "hbm"
    assert abs(r["frac"] - 0.5) < 1e-9 and abs(r["achieved"] - 4000.0) < 1e-6
    assert all(b["frac"] <= 1.0 for b in r["bounds"].values())
    r = bench.roofline(work, kernel_ms=400.0, traffic=None, no_reuse_bytes=1e13)
    assert r["binding"] == "valu_issued" and r["bound"] == "alu"
    assert abs(r["frac"] - 0.25) < 1e-3
