"""Oracle: Algorithm 3 phase 3 (backward edges with lazy pruning, Section 4.3).

Pinned against a hand-worked case, against the set definition of the phase
(own out-neighbours plus reverse sources, ordered by (D, id), cut to Cb) built
here independently, the symmetry it gives when no row has to be pruned, and the
pruning invariants of Eq. (1) on the rows that are pruned."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

NONE = oracle.NONE
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(adj):
    return [[int(v) for v in r if v != NONE] for r in adj]


def _pad(adj, W):
    out = np.full((adj.shape[0], W), NONE, np.uint32)
    out[:, : adj.shape[1]] = adj
    return out


def _setup(n=500, d=5, C=40, R=10, alpha=1.2, seed=11):
    x, _ = workloads.uniform_cube(n, 1, d, seed=seed)
    cand, D = oracle.knn(x, x, C, exclude_self=True, mode=oracle.FP64)
    adj = oracle.prune(x, cand, D, R=R, alpha=alpha, mode=oracle.FP64, width=R + 1)
    return x, adj


def _union_sorted(x, rows, p):
    """Own out-neighbours plus sources of in-edges, a set, by (D64, id)."""
    V = set(rows[p]) | {u for u, r in enumerate(rows) if p in r}
    key = [(float(oracle.dist_f64(x[p], x[v])), v) for v in V]
    return [v for _, v in sorted(key)]


def test_hand_worked_line():
    g = json.load(open(os.path.join(GOLD, "backward_line.json")))
    x = np.array(g["points"], np.float32)
    for case in g["cases"]:
        R = case["R"]
        adj = np.full((len(x), R + 1), NONE, np.uint32)
        for u, r in enumerate(g["adj_before"]):
            adj[u, : len(r)] = r
        for mode in (oracle.FP32, oracle.FP64):
            out = _rows(oracle.backward(x, adj, R, case["Cb"], case["alpha"], mode=mode))
            assert out[0] == case["row0"], (case, mode)
            assert all(out[u] == [0] for u in range(1, len(x))), (case, mode)


def test_without_pruning_rows_are_the_sorted_union():
    x, adj = _setup()
    rows = _rows(adj)
    W = 400  # no candidate set reaches this: nothing is pruned or cut
    new = _rows(oracle.backward(x, _pad(adj, W), W, W, 1.2, mode=oracle.FP64))
    for p in range(len(x)):
        assert new[p] == _union_sorted(x, rows, p), p
    # every phase-2 edge now has its reverse
    for u, r in enumerate(rows):
        for v in r:
            assert u in new[v] and v in new[u]


@pytest.mark.parametrize("R,Cb", [(10, 40), (8, 12), (10, 10)])
def test_pruned_rows_follow_eq1_over_the_cut_union(R, Cb):
    alpha = 1.2
    x, adj = _setup(R=R)
    rows = _rows(adj)
    new = _rows(oracle.backward(x, adj, R, Cb, alpha, mode=oracle.FP64))
    xd = x.astype(np.float64)
    pruned_rows = 0
    for p in range(len(x)):
        V = _union_sorted(x, rows, p)[:Cb]
        if len(V) <= R:
            assert new[p] == V, p
            continue
        pruned_rows += 1
        kept = new[p]
        assert len(kept) <= R and set(kept) <= set(V)
        pos = {v: j for j, v in enumerate(V)}
        assert [pos[v] for v in kept] == sorted(pos[v] for v in kept)  # candidate order
        S = []
        for u in V:
            if len(S) == len(kept):
                break
            a = np.linalg.norm(xd[p] - xd[u])
            hits = [a > alpha * np.linalg.norm(xd[u] - xd[v]) for v in S]
            if u in kept:
                assert u == kept[len(S)] and not any(hits), (p, u)
                S.append(u)
            else:
                assert any(hits), (p, u)
    assert (pruned_rows > 0) == (Cb > R)


def test_empty_and_isolated_rows():
    x = np.array([[0.0], [1.0], [5.0]], np.float32)
    adj = np.full((3, 3), NONE, np.uint32)
    adj[1, 0] = 0  # 1 -> 0 only; 2 has no edges in or out
    out = _rows(oracle.backward(x, adj, 2, 4, 1.2))
    assert out == [[1], [0], []]


def test_build_with_backward_edges_is_connected_and_bounded():
    x, _ = workloads.generate(1, n=3000, nq=1)
    adj, e, _ = oracle.build(x, 16, 48, 1.2, backward=True)
    assert oracle.reachable(adj, e).all()
    deg = (adj != NONE).sum(1)
    assert deg.max() <= 17
    # more in-edges than the build without the phase
    adj0, _, _ = oracle.build(x, 16, 48, 1.2)
    assert (adj != NONE).sum() > (adj0 != NONE).sum()
