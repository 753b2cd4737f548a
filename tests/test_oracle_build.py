"""Pins for the oracle's build stages: exact candidates, the pruning rule
(Definition 2 / Eq. (1), Algorithm 2), the entry point (centroid rule of
Algorithm 3) and connectivity (Algorithm 3, phase 4)."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NONE = oracle.NONE


def exact_d2(a, b):
    a = a.astype(np.float64)
    b = b.astype(np.float64)
    return ((a[:, None, :] - b[None, :, :]) ** 2).sum(-1)


# ---------------------------------------------------------------- candidates
@pytest.mark.parametrize("mode", [oracle.FP32, oracle.FP64])
def test_knn_is_brute_force(mode):
    x, q = workloads.uniform_cube(300, 40, 6, seed=2)
    ids, D = oracle.knn(q, x, 17, mode=mode)
    E = exact_d2(q, x)
    for i in range(len(q)):
        want = np.lexsort((np.arange(len(x)), E[i]))[:17]
        assert list(ids[i]) == list(want)
        np.testing.assert_allclose(D[i], E[i][want], rtol=1e-6)


def test_knn_excludes_self_keeps_duplicates_and_pads():
    x, _ = workloads.uniform_cube(50, 1, 4, seed=3)
    x[7] = x[3]                       # an exact duplicate of point 3
    ids, D = oracle.knn(x, x, 5, exclude_self=True)
    assert all(i not in row for i, row in enumerate(ids))
    assert ids[3][0] == 7 and D[3][0] == 0.0 and ids[7][0] == 3
    ids2, D2 = oracle.knn(x[:4], x[:4], 6, exclude_self=True)   # only 3 others exist
    assert (ids2[:, 3:] == NONE).all() and np.isinf(D2[:, 3:]).all()


def test_knn_ties_break_by_id():
    x = np.array([[0.0], [1.0], [-1.0], [2.0], [-2.0]], np.float32)
    ids, _ = oracle.knn(np.zeros((1, 1), np.float32), x, 5)
    assert list(ids[0]) == [0, 1, 2, 3, 4]


# ---------------------------------------------------------------- pruning
def test_prune_hand_worked_cases():
    g = json.load(open(os.path.join(GOLD, "prune_line.json")))
    pts = np.array(g["points"], np.float32)
    cand = np.array([[1, 2, 3, 4]], np.uint32)
    for mode in (oracle.FP32, oracle.FP64):
        D = np.array([[oracle.dist_f64(pts[0], pts[c]) for c in cand[0]]])
        for case in g["cases"]:
            # prune only row 0; other rows get empty candidate lists
            C = np.full((len(pts), 4), NONE, np.uint32)
            CD = np.full((len(pts), 4), np.inf)
            C[0], CD[0] = cand[0], D[0]
            adj = oracle.prune(pts, C, CD, R=4, alpha=case["alpha"], tau=case["tau"], mode=mode)
            got = [int(v) for v in adj[0] if v != NONE]
            assert got == case["expect"], (mode, case)


def test_prune_near_tie_keeps_tau():
    """Float32 near-ties of Eq. (1) are re-decided in float64 with the same tau.
    p = 0, u = 3, v = 1 on a line: d(p,u) = 3, d(u,v) = 2, alpha = 1, so the
    right side is 2 + 2 tau.  tau = 0.5 is an exact tie (u kept); tau just below
    0.5 rounds to 0.5 in float32, so only the float64 re-check with the given tau
    prunes u."""
    pts = np.array([[0.0], [1.0], [3.0]], np.float32)
    C = np.full((3, 2), NONE, np.uint32)
    CD = np.full((3, 2), np.inf)
    C[0] = [1, 2]
    CD[0] = [1.0, 9.0]
    for mode in (oracle.FP32, oracle.FP64):
        for tau, expect in ((0.5, [1, 2]), (0.499999999, [1]), (0.500000001, [1, 2]),
                            (0.0, [1])):
            adj = oracle.prune(pts, C, CD, R=2, alpha=1.0, tau=tau, mode=mode)
            assert [int(v) for v in adj[0] if v != NONE] == expect, (mode, tau)


def _prune_setup(n=400, d=8, C=40, seed=4):
    x, _ = workloads.uniform_cube(n, 1, d, seed=seed)
    cand, D = oracle.knn(x, x, C, exclude_self=True, mode=oracle.FP64)
    return x, cand, D


def _decides(x, p, u, v, alpha, tau):
    """Eq. (1) in double precision: returns (prunes, margin)."""
    a = np.linalg.norm(x[p].astype(np.float64) - x[u])
    b = np.linalg.norm(x[u].astype(np.float64) - x[v])
    rhs = alpha * b + (alpha + 1) * tau
    return a > rhs, abs(a - rhs) / max(a, 1e-300)


@pytest.mark.parametrize("alpha,tau", [(1.2, 0.0), (1.5, 0.02), (1.0, 0.0), (0.9, 0.0)])
def test_prune_invariants(alpha, tau):
    """(i) no kept edge is prunable by an earlier kept one; (ii) every dropped
    candidate seen before the cap is prunable by an earlier kept one; (iii) rows
    follow candidate order, hold no self loop or duplicate, length <= R."""
    x, cand, D = _prune_setup()
    R = 12
    adj = oracle.prune(x, cand, D, R=R, alpha=alpha, tau=tau, mode=oracle.FP64)
    for p in range(len(x)):
        kept = [int(v) for v in adj[p] if v != NONE]
        assert len(kept) <= R and len(set(kept)) == len(kept) and p not in kept
        order = {int(u): j for j, u in enumerate(cand[p])}
        assert [order[v] for v in kept] == sorted(order[v] for v in kept)
        S = []
        for u in cand[p]:
            u = int(u)
            if len(S) == len(kept):
                break
            hits = [_decides(x, p, u, v, alpha, tau) for v in S]
            if u in kept:
                assert u == kept[len(S)]
                assert not any(h for h, m in hits if m > 1e-9)
                S.append(u)
            else:
                assert any(h for h, m in hits) or any(m <= 1e-9 for h, m in hits)


def test_prune_huge_alpha_is_exact_rnn():
    """alpha -> infinity prunes nothing: rows are the first R candidates."""
    x, cand, D = _prune_setup(seed=5)
    adj = oracle.prune(x, cand, D, R=10, alpha=1e30, tau=0.0)
    assert (adj == cand[:, :10]).all()
    adj = oracle.prune(x, cand, D, R=10, alpha=1.2, tau=1e9)   # tau >= diameter: same
    assert (adj == cand[:, :10]).all()


def test_prune_alpha1_tau0_is_mrng_rule():
    """alpha = 1, tau = 0 is the MRNG / HNSW-heuristic rule: keep u unless a kept v
    (closer to p) is closer to u than p is."""
    x, cand, D = _prune_setup(seed=6)
    adj = oracle.prune(x, cand, D, R=1000, alpha=1.0, tau=0.0, mode=oracle.FP64)
    for p in range(0, len(x), 7):
        S = []
        for u in cand[p]:
            du = np.linalg.norm(x[p].astype(np.float64) - x[u])
            if all(np.linalg.norm(x[u].astype(np.float64) - x[v]) >= du for v in S):
                S.append(int(u))
        assert [int(v) for v in adj[p] if v != NONE] == S


def test_prune_lune_form():
    """Eq. (1) equals membership of v in B(p, d(p,u)) and B(u, r), with
    r = (d(p,u) - (alpha+1) tau) / alpha (Section 3.1, Fig. 1d)."""
    x, cand, D = _prune_setup(seed=7)
    alpha, tau = 1.3, 0.01
    adj = oracle.prune(x, cand, D, R=1000, alpha=alpha, tau=tau, mode=oracle.FP64)
    xd = x.astype(np.float64)
    for p in range(0, len(x), 5):
        kept = [int(v) for v in adj[p] if v != NONE]
        for u in cand[p]:
            u = int(u)
            dpu = np.linalg.norm(xd[p] - xd[u])
            r = (dpu - (alpha + 1) * tau) / alpha
            earlier = [v for v in kept if np.linalg.norm(xd[p] - xd[v]) <= dpu and v != u]
            in_lune = [v for v in earlier if np.linalg.norm(xd[u] - xd[v]) < r]
            assert (u in kept) == (len(in_lune) == 0)


def test_prune_fp32_matches_fp64_away_from_ties():
    x, _ = workloads.generate(1, n=2000, nq=1)
    cand, D32 = oracle.knn(x, x, 32, exclude_self=True, mode=oracle.FP32)
    cand64, D64 = oracle.knn(x, x, 32, exclude_self=True, mode=oracle.FP64)
    assert (cand == cand64).mean() > 0.999
    a32 = oracle.prune(x, cand, D32, R=16, alpha=1.2, mode=oracle.FP32)
    a64 = oracle.prune(x, cand, D64, R=16, alpha=1.2, mode=oracle.FP64)
    same = (a32 == a64).all(axis=1)
    assert same.mean() > 0.995


# ---------------------------------------------------------------- entry
def test_medoid_is_point_nearest_centroid():
    for seed, (n, d) in enumerate([(5000, 16), (9000, 3), (100, 128)]):
        x, _ = workloads.uniform_cube(n, 1, d, seed=seed)
        c = x.astype(np.float64).mean(0)
        dd = ((x.astype(np.float64) - c) ** 2).sum(1)
        order = np.argsort(dd)
        assert dd[order[1]] - dd[order[0]] > 1e-9 * dd[order[0]]
        assert oracle.medoid(x) == order[0]


def test_medoid_tiny_hand_worked():
    """Points 1, 3, 8: centroid 4, nearest point 3 (id 1); a centroid of the sum
    (12) or of sum / (n - 1) (6) would pick 8 (id 2)."""
    assert oracle.medoid(np.array([[1.0], [3.0], [8.0]], np.float32)) == 1
    x = np.array([[1.0, 0.0], [3.0, 1.0], [8.0, -1.0]], np.float32)   # centroid (4, 0)
    assert oracle.medoid(x) == 1


def test_medoid_tie_goes_to_smaller_id():
    x = np.array([[1.0], [-1.0], [3.0], [-3.0]], np.float32)   # centroid 0, ids 0 and 1 tie
    assert oracle.medoid(x) == 0


# ---------------------------------------------------------------- connectivity
def test_connect_reaches_everything_using_free_slots_only():
    x, _ = workloads.generate(1, n=3000, nq=1)
    cand, D = oracle.knn(x, x, 32, exclude_self=True)
    R, W = 12, 13
    pruned = oracle.prune(x, cand, D, R=R, alpha=1.2, width=W)
    s = oracle.medoid(x)
    assert oracle.reachable(pruned, s).mean() < 1.0          # clusters are disconnected
    adj, added, rounds = oracle.connect(x, pruned, s, Lc=32)
    assert oracle.reachable(adj, s).all()
    assert added >= 1 and rounds >= 1
    deg0 = (pruned != NONE).sum(1)
    # pruned edges are untouched; new edges only fill slots that were empty
    for p in range(len(x)):
        assert (adj[p, :deg0[p]] == pruned[p, :deg0[p]]).all()
    assert ((adj != NONE).sum() - (pruned != NONE).sum()) == added
    # every added edge points to a point that had no path from the entry before
    before = oracle.reachable(pruned, s)
    new_targets = adj[(adj != pruned)]
    assert not before[new_targets].any()


def test_connect_noop_when_connected():
    x, _ = workloads.uniform_cube(500, 1, 4, seed=8)
    cand, D = oracle.knn(x, x, 20, exclude_self=True)
    pruned = oracle.prune(x, cand, D, R=20, alpha=1e30, width=21)
    s = oracle.medoid(x)
    if oracle.reachable(pruned, s).all():
        adj, added, rounds = oracle.connect(x, pruned, s, Lc=20)
        assert added == 0 and rounds == 0 and (adj == pruned).all()


def test_connect_capacity_error():
    # rows of width 1 that are all full and a cycle that cannot reach point 3
    x = np.array([[0.0], [1.0], [2.0], [10.0]], np.float32)
    adj = np.array([[1], [2], [0], [2]], np.uint32)
    with pytest.raises(RuntimeError):
        oracle.connect(x, adj, 0, Lc=4)


def test_threads_do_not_change_results():
    x, q = workloads.generate(1, n=2000, nq=50)
    oracle.set_threads(1)
    a1, e1, _ = oracle.build(x, 12, 24, 1.2)
    r1 = oracle.search(x, a1, q, 10, 32, e1)
    oracle.set_threads(max(2, oracle.max_threads()))
    a2, e2, _ = oracle.build(x, 12, 24, 1.2)
    r2 = oracle.search(x, a2, q, 10, 32, e2)
    assert e1 == e2 and (a1 == a2).all()
    for u, v in zip(r1, r2):
        assert (u == v).all()


@pytest.mark.parametrize("mode", [oracle.FP32, oracle.FP64])
def test_connect_hand_traced_cases(mode):
    """Hand-traced rounds of the connectivity phase (Alg. 3 phase 4): which
    unreached points are attached in a round (the smallest id of every strongly
    connected component of the unreached subgraph that no other unreached
    point enters), to which row (the first search result with a free slot,
    else the nearest reached point with one), and in what order competing
    points are applied."""
    g = json.load(open(os.path.join(GOLD, "connect_cases.json")))
    for c in g["cases"]:
        adj, added, rounds = oracle.connect(np.array(c["points"], np.float32),
                                            np.array(c["adj"], np.uint32), c["entry"], c["Lc"],
                                            mode=mode)
        assert adj.tolist() == c["expect_adj"], c["name"]
        assert added == c["expect_added"] and rounds == c["expect_rounds"], c["name"]
