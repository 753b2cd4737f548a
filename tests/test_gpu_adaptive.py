"""GPU adaptive local pruning (Algorithm 4, Section 4.2) against the oracle, bit
for bit: the pruning stage alone, the hand-worked cases, and whole builds with
adaptive alpha and the backward-edge phase."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2510_05975_amd as cng
import workloads
from gpu_util import dev, dev_ids, f32_of, host_ids

pytestmark = pytest.mark.gpu

NONE = oracle.NONE
GOLD = os.path.join(os.path.dirname(__file__), "golden")
A0, AMAX, STEP = 0.9, 1.6, 0.05


@pytest.mark.parametrize("case", [(1, 4000, 24, 64, 0.0), (2, 3000, 32, 128, 0.0),
                                  (4, 3000, 32, 128, 0.0), (1, 3000, 16, 48, 0.2),
                                  (3, 1000, 48, 192, 0.0), (2, 3000, 48, 160, 0.0)])
def test_prune_adaptive(case):
    """d <= 128 with R <= 32 and C <= 128 runs the register kernel; the last two
    cases (d = 960; R = 48 and C = 160 at d = 128) the kernel with the LDS pair
    table."""
    cfg, n, R, C, tau = case
    print(f"adaptive prune cfg{cfg} n={n} R={R} C={C} tau={tau}", flush=True)
    x, _ = workloads.generate(cfg, n=n, nq=1)
    cand, D = oracle.knn(x, x, C, exclude_self=True)
    want = oracle.prune(x, cand, D, R, A0, tau=tau, width=R + 1, alpha_max=AMAX, alpha_step=STEP)
    got = cng.prune(dev(x), dev_ids(cand), dev(f32_of(D)), R, A0, tau, width=R + 1, alpha_max=AMAX,
                    alpha_step=STEP)
    torch.cuda.synchronize()
    assert (host_ids(got) == want).all()


@pytest.mark.parametrize("d", [1500, 3001])
def test_prune_adaptive_long_rows(d):
    """Rows of 12 and 24 chunks of 128 values (aligned and not) in the kernel
    with the LDS pair table."""
    print(f"adaptive prune d={d}", flush=True)
    x, _ = workloads.uniform_cube(500, 1, d, seed=d)
    cand, D = oracle.knn(x, x, 32, exclude_self=True)
    want = oracle.prune(x, cand, D, 12, A0, width=13, alpha_max=AMAX, alpha_step=STEP)
    got = cng.prune(dev(x), dev_ids(cand), dev(f32_of(D)), 12, A0, 0.0, width=13, alpha_max=AMAX,
                    alpha_step=STEP)
    torch.cuda.synchronize()
    assert (host_ids(got) == want).all()


@pytest.mark.parametrize("step,R", [(0.02, 15), (0.01, 16)])
def test_prune_adaptive_many_passes(step, R):
    """36 passes (all alpha passes in one sweep) and 71 passes (more than the
    sweep holds: one pass after the other), odd and even R."""
    x, _ = workloads.generate(1, n=3000, nq=1)
    cand, D = oracle.knn(x, x, 48, exclude_self=True)
    want = oracle.prune(x, cand, D, R, A0, width=R + 1, alpha_max=AMAX, alpha_step=step)
    got = cng.prune(dev(x), dev_ids(cand), dev(f32_of(D)), R, A0, 0.0, width=R + 1,
                    alpha_max=AMAX, alpha_step=step)
    torch.cuda.synchronize()
    assert (host_ids(got) == want).all()


def test_prune_adaptive_hand_worked():
    g = json.load(open(os.path.join(GOLD, "adaptive_alpha.json")))
    for case in g["cases"]:
        x = np.array(case["points"], np.float32)
        n, c = len(x), len(case["cand0"])
        cand = np.full((n, c), NONE, np.uint32)
        cD = np.full((n, c), np.inf, np.float32)
        cand[0] = case["cand0"]
        cD[0] = [oracle.dist_f32(x[0], x[v]) for v in case["cand0"]]
        for run in case["runs"]:
            got = cng.prune(dev(x), dev_ids(cand), dev(cD), run["M"], run.get("alpha0", A0), 0.0,
                            alpha_max=run["alpha_max"], alpha_step=run.get("alpha_step", STEP))
            torch.cuda.synchronize()
            assert [int(v) for v in host_ids(got)[0] if v != NONE] == run["row0"], run


@pytest.mark.parametrize("case", [(1, 10000, 24, 64), (2, 5000, 32, 128), (4, 4000, 32, 128)])
def test_build_adaptive_backward_bit_exact(case):
    cfg, n, R, C = case
    print(f"adaptive build cfg{cfg} n={n}", flush=True)
    x, _ = workloads.generate(cfg, n=n, nq=1)
    oadj, oe, oadded = oracle.build(x, R, C, A0, alpha_max=AMAX, alpha_step=STEP, backward=True)
    g = cng.build(dev(x), R, C, A0, alpha_max=AMAX, alpha_step=STEP, backward=True)
    assert g.entry == oe
    assert (host_ids(g.adj) == oadj).all()
    assert g.stats["connect_added"] == oadded


def test_backward_adaptive_stage():
    x, _ = workloads.generate(1, n=3000, nq=1)
    cand, D = oracle.knn(x, x, 64, exclude_self=True)
    pruned = oracle.prune(x, cand, D, 24, A0, width=25, alpha_max=AMAX, alpha_step=STEP)
    want = oracle.backward(x, pruned, 24, 64, A0, alpha_max=AMAX, alpha_step=STEP)
    a = dev_ids(pruned)
    cng.backward(dev(x), a, 24, 64, A0, alpha_max=AMAX, alpha_step=STEP)
    torch.cuda.synchronize()
    assert (host_ids(a) == want).all()
