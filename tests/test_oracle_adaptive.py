"""Oracle: Algorithm 4 (adaptive local pruning, Section 4.2).

Pinned by hand-worked cases (the M/2 stopping rule, odd M, alpha_max itself
reached, the never-reached case) and by its definition in terms of the fixed
pruning: the row equals the capped shortcut set of the first alpha_i whose set
holds at least M/2 points (else of the last alpha_i)."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

NONE = oracle.NONE
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _row(a, p=0):
    return [int(v) for v in a[p] if v != NONE]


def test_hand_worked():
    g = json.load(open(os.path.join(GOLD, "adaptive_alpha.json")))
    for case in g["cases"]:
        x = np.array(case["points"], np.float32)
        n, c = len(x), len(case["cand0"])
        cand = np.full((n, c), NONE, np.uint32)
        cD = np.full((n, c), np.inf)
        cand[0] = case["cand0"]
        cD[0] = [oracle.dist_f64(x[0], x[v]) for v in case["cand0"]]
        for run in case["runs"]:
            for mode in (oracle.FP32, oracle.FP64):
                a = oracle.prune(x, cand, cD, run["M"], run.get("alpha0", 0.9), mode=mode,
                                 alpha_max=run["alpha_max"], alpha_step=run.get("alpha_step", 0.05))
                assert _row(a) == run["row0"], (run, mode)


@pytest.mark.parametrize("M", [8, 9, 16])
def test_is_the_first_alpha_reaching_half_M(M):
    x, _ = workloads.uniform_cube(400, 1, 6, seed=21)
    cand, D = oracle.knn(x, x, 48, exclude_self=True, mode=oracle.FP64)
    alphas = [0.9 + i * 0.05 for i in range(15)]  # 0.9 .. 1.6
    fixed = [oracle.prune(x, cand, D, M, a, mode=oracle.FP64) for a in alphas]
    got = oracle.prune(x, cand, D, M, 0.9, mode=oracle.FP64, alpha_max=1.6, alpha_step=0.05)
    chosen = []
    for p in range(len(x)):
        sizes = [len(_row(f, p)) for f in fixed]
        i = next((j for j, s in enumerate(sizes) if 2 * s >= M), len(alphas) - 1)
        chosen.append(i)
        assert _row(got, p) == _row(fixed[i], p), p
    assert len(set(chosen)) > 2  # several alphas are in use


def test_build_and_backward_accept_adaptive():
    x, _ = workloads.generate(1, n=2000, nq=1)
    adj, e, _ = oracle.build(x, 16, 48, 0.9, alpha_max=1.6, alpha_step=0.05, backward=True)
    assert oracle.reachable(adj, e).all()
    assert ((adj != NONE).sum(1) <= 17).all()
    with pytest.raises(RuntimeError):
        oracle.build(x, 16, 48, 1.2, alpha_max=1.0, alpha_step=0.05)  # alpha_max < alpha0
