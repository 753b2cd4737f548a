"""Pins for the sub-quadratic candidate phases of Algorithm 3 (Section 4.1):
phase 1, an approximate K-NN graph by NN-descent (synchronous rounds over
neighbours of neighbours, started from SplitMix64 draws), and phase 2, each
point's local-neighbour set = the C nearest of the points a beam search on
that graph evaluates."""
import numpy as np
import pytest

import oracle
import workloads

NONE = oracle.NONE


def test_splitmix_reference_outputs():
    """The first outputs of SplitMix64 seeded with 0, as published with the
    generator (0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, ...)."""
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert [oracle.splitmix(0, i) for i in range(4)] == want


def _check_rows(x, ids, D):
    n, K = ids.shape
    for p in range(n):
        row = [int(v) for v in ids[p] if v != NONE]
        assert p not in row and len(set(row)) == len(row)
        assert all(v == NONE for v in ids[p][len(row):])
        keys = [(float(D[p, j]), row[j]) for j in range(len(row))]
        assert keys == sorted(keys)
        for j, v in enumerate(row):
            assert D[p, j] == float(oracle.dist_f32(x[p], x[v]))


def test_nndescent_rows_and_start():
    x, _ = workloads.generate(1, n=500, nq=1)
    K, seed = 8, 77
    ids, D, r = oracle.nndescent(x, K, seed, 0)
    assert r == 0
    _check_rows(x, ids, D)
    # round 0: the K nearest of the distinct draws splitmix(seed, pK + j) mod n
    for p in (0, 123, 499):
        draws = {oracle.splitmix(seed, p * K + j) % 500 for j in range(K)} - {p}
        best = sorted(draws, key=lambda v: (float(oracle.dist_f32(x[p], x[v])), v))[:K]
        assert [int(v) for v in ids[p] if v != NONE] == best


def test_nndescent_one_round_is_synchronous():
    """One round: each list becomes the K nearest of itself and its members'
    lists, all taken from the previous round (numpy brute force over that
    candidate set)."""
    x, _ = workloads.generate(1, n=400, nq=1)
    K, seed = 6, 5
    ids0, _, _ = oracle.nndescent(x, K, seed, 0)
    ids1, D1, r = oracle.nndescent(x, K, seed, 1)
    assert r == 1
    _check_rows(x, ids1, D1)
    for p in range(0, 400, 7):
        cand = set(int(v) for v in ids0[p] if v != NONE)
        for u in list(cand):
            cand |= set(int(v) for v in ids0[u] if v != NONE)
        cand.discard(p)
        best = sorted(cand, key=lambda v: (float(oracle.dist_f32(x[p], x[v])), v))[:K]
        assert [int(v) for v in ids1[p] if v != NONE] == best


def test_nndescent_monotone_and_converges_to_exact_on_tiny_sets():
    x, _ = workloads.uniform_cube(40, 1, 3, seed=3)
    K = 39
    prev = None
    for r in range(4):
        ids, D, _ = oracle.nndescent(x, K, 11, r)
        if prev is not None:   # every rank's key can only improve
            for p in range(40):
                for j in range(K):
                    a = (prev[1][p, j], int(prev[0][p, j]))
                    b = (D[p, j], int(ids[p, j]))
                    assert b <= a
        prev = (ids, D)
    ids, D, r = oracle.nndescent(x, K, 11, 50)
    assert r < 50                        # stopped: a round changed nothing
    gt, gD = oracle.knn(x, x, K, exclude_self=True)
    assert (ids == gt).all()


def test_nndescent_quality_on_the_mixture():
    x, _ = workloads.generate(1, n=5000, nq=1)
    ids, _, r = oracle.nndescent(x, 16, 1, 12)
    gt, _ = oracle.knn(x, x, 16, exclude_self=True)
    rec = np.mean([len(set(a) & set(b)) / 16 for a, b in zip(ids.tolist(), gt.tolist())])
    assert rec >= 0.9, rec


def test_graph_candidates_full_beam_is_exact():
    """On a graph whose reachable set is everything, a beam as large as the
    set evaluates every point, so the candidates are the exact C nearest."""
    x, _ = workloads.uniform_cube(600, 1, 4, seed=9)
    g0, _ = oracle.knn(x, x, 12, exclude_self=True)
    s = oracle.medoid(x)
    assert oracle.reachable(g0, s).all()
    cand, cD = oracle.graph_candidates(x, g0, s, 600, 20)
    gt, gD = oracle.knn(x, x, 20, exclude_self=True)
    assert (cand == gt).all() and (cD == gD).all()


def test_graph_candidates_are_the_nearest_visited_and_own_row():
    """With a small beam: the C nearest, p excluded, of the result of
    beam-search(G0, x_p, s, L, C + 1) (the search independently called)
    together with p's own G0 row."""
    x, _ = workloads.generate(1, n=1500, nq=1)
    g0, _, _ = oracle.nndescent(x, 10, 3, 6)
    s = oracle.medoid(x)
    C, L = 16, 24
    cand, cD = oracle.graph_candidates(x, g0, s, L, C)
    for p in range(0, 1500, 37):
        ids, dists, _, _ = oracle.search(x, g0, x[p:p + 1], C + 1, L, s)
        pool = set(int(v) for v in ids[0] if v != NONE) | set(int(v) for v in g0[p] if v != NONE)
        pool.discard(p)
        want = sorted(pool, key=lambda v: (float(oracle.dist_f32(x[p], x[v])), v))[:C]
        assert [int(v) for v in cand[p] if v != NONE] == want
        assert all(cD[p, j] == float(oracle.dist_f32(x[p], x[v])) for j, v in enumerate(want))


def test_graph_candidates_keep_own_row_across_clusters():
    """Ten separated clusters: G0 does not lead from s to the other clusters,
    and the own G0 row keeps every point's candidates in its cluster."""
    x, _ = workloads.generate(1, n=2000, nq=1)
    g0, _, _ = oracle.nndescent(x, 16, 2, 8)
    s = oracle.medoid(x)
    assert oracle.reachable(g0, s).mean() < 0.5
    cand, _ = oracle.graph_candidates(x, g0, s, 32, 16)
    gt, _ = oracle.knn(x, x, 16, exclude_self=True)
    rec = np.mean([len(set(a) & set(b)) / 16 for a, b in zip(cand.tolist(), gt.tolist())])
    assert rec >= 0.9, rec


def test_build_with_graph_candidates():
    """The sub-quadratic build: every point reachable; with a good K-NN graph
    and a beam that evaluates everything it equals the exact-candidate build."""
    x, q = workloads.generate(1, n=2000, nq=50)
    a, e, _ = oracle.build(x, 16, 32, 1.2, knn_K=24, knn_seed=1, knn_rounds=10, cand_L=2000)
    b, e2, _ = oracle.build(x, 16, 32, 1.2)
    g0, _, _ = oracle.nndescent(x, 24, 1, 10)
    if oracle.reachable(g0, e).all():
        assert e == e2 and (a == b).all()
    c, _, _ = oracle.build(x, 16, 32, 1.2, knn_K=16, knn_seed=1, knn_rounds=8, cand_L=48)
    assert oracle.reachable(c, e).all()
    ids, _, _, _ = oracle.search(x, c, q, 10, 32, e)
    gt, _ = oracle.knn(q, x, 10)
    rec = np.mean([len(set(u) & set(v)) / 10 for u, v in zip(ids.tolist(), gt.tolist())])
    assert rec >= 0.9, rec
