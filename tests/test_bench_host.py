"""Host-side contract of bench.py (no GPU): the one-GPU guard and the
recorded search-kernel traffic, which must belong to the kernel source as it
stands (a changed kernel needs its counters taken again)."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_recorded_traffic_matches_kernel_source():
    for (workload, L), rec in bench.SEARCH_TRAFFIC.items():
        assert bench.search_traffic(workload, L) == rec["bytes"], (workload, L)
    assert bench.search_traffic("sift_like_1m", 12345) is None


def test_recall_counts_ties():
    # result 2 ties with the 2nd true neighbour: strict recall misses it, the
    # tie-aware count takes it
    ids = np.array([[0, 2]])
    gt = np.array([[0, 1]])
    res_d = np.array([[0.0, 1.0]])
    gt_dk = np.array([1.0])
    strict, tie = bench.recall(ids, gt, gt_dk, res_d)
    assert strict == 0.5 and tie == 1.0
