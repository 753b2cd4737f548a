"""GPU backward-edge phase (Algorithm 3, phase 3; Section 4.3) against the
oracle, bit for bit: the stage alone on the same pruned graph, and whole builds
with the phase switched on."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2510_05975_amd as cng
import workloads
from gpu_util import dev, dev_ids, host_ids

pytestmark = pytest.mark.gpu

NONE = oracle.NONE
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("case", [(1, 5000, 24, 64, 64), (2, 4000, 32, 128, 128),
                                  (4, 3000, 32, 128, 128), (1, 3000, 12, 48, 8),
                                  (3, 1500, 48, 192, 192)])
def test_backward_stage(case):
    cfg, n, R, C, Cb = case
    print(f"backward cfg{cfg} n={n} R={R} C={C} Cb={Cb}", flush=True)
    x, _ = workloads.generate(cfg, n=n, nq=1)
    cand, D = oracle.knn(x, x, C, exclude_self=True)
    pruned = oracle.prune(x, cand, D, R=R, alpha=1.2, width=R + 1)
    want = oracle.backward(x, pruned, R, Cb, 1.2)
    a = dev_ids(pruned)
    cng.backward(dev(x), a, R, Cb, 1.2)
    torch.cuda.synchronize()
    assert (host_ids(a) == want).all()


def test_backward_hand_worked_line():
    g = json.load(open(os.path.join(GOLD, "backward_line.json")))
    x = np.array(g["points"], np.float32)
    for case in g["cases"]:
        R = case["R"]
        adj = np.full((len(x), R + 1), NONE, np.uint32)
        for u, r in enumerate(g["adj_before"]):
            adj[u, : len(r)] = r
        a = dev_ids(adj)
        cng.backward(dev(x), a, R, case["Cb"], case["alpha"])
        torch.cuda.synchronize()
        got = host_ids(a)
        assert [int(v) for v in got[0] if v != NONE] == case["row0"], case


def test_backward_tau_and_wide_rows():
    x, _ = workloads.generate(1, n=2000, nq=1)
    cand, D = oracle.knn(x, x, 96, exclude_self=True)
    pruned = oracle.prune(x, cand, D, R=70, alpha=1.5, tau=0.3, width=80)  # rows wider than 64
    want = oracle.backward(x, pruned, 70, 96, 1.5, tau=0.3)
    a = dev_ids(pruned)
    cng.backward(dev(x), a, 70, 96, 1.5, 0.3)
    torch.cuda.synchronize()
    assert (host_ids(a) == want).all()


@pytest.mark.parametrize("case", [(1, 10000, 24, 64), (2, 5000, 32, 128), (4, 4000, 32, 128)])
def test_build_with_backward_bit_exact(case):
    cfg, n, R, C = case
    print(f"build+backward cfg{cfg} n={n}", flush=True)
    x, _ = workloads.generate(cfg, n=n, nq=1)
    oadj, oe, oadded = oracle.build(x, R, C, 1.2, backward=True)
    g = cng.build(dev(x), R, C, 1.2, backward=True)
    assert g.entry == oe
    assert (host_ids(g.adj) == oadj).all()
    assert g.stats["connect_added"] == oadded
    assert g.stats["ms_backward"] > 0
