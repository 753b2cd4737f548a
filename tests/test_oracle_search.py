"""Pins for the oracle's beam search (Algorithm 1) and for the guarantees of the
alpha-convergent graph (Lemma 3, Lemma 5, alpha-shortcut reachability;
Section 3.2-3.3)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NONE = oracle.NONE


@pytest.mark.parametrize("mode", [oracle.FP32, oracle.FP64])
def test_hand_traced_line(mode):
    g = json.load(open(os.path.join(GOLD, "beam_line.json")))
    pts = np.array(g["points"], np.float32)
    adj = np.array(g["adj"], np.uint32)
    q = np.array([g["query"]], np.float32)
    ids, dists, hops, ndc = oracle.search(pts, adj, q, g["k"], g["L"], g["entry"], mode=mode)
    assert list(ids[0]) == g["expect_ids"]
    assert list(dists[0]) == g["expect_dists"]
    assert hops[0] == len(g["expect_hops"]) and ndc[0] == g["expect_ndc"]
    _, _, trace = oracle.search_trace(pts, adj, q[0], g["k"], g["L"], g["entry"], mode=mode)
    assert list(trace) == g["expect_hops"]


def test_large_beam_returns_exact_knn_of_reachable_set():
    x, q = workloads.generate(1, n=1500, nq=30)
    adj, s, _ = oracle.build(x, 10, 20, 1.2)
    assert oracle.reachable(adj, s).all()
    ids, dists, hops, ndc = oracle.search(x, adj, q, 10, 1500, s)
    gt, gD = oracle.knn(q, x, 10)
    assert (ids == gt).all()
    assert (hops == 1500).all() and (ndc == 1500).all()          # everything explored
    np.testing.assert_array_equal(dists, np.sqrt(gD.astype(np.float32)).astype(np.float64))


def test_unreachable_points_never_returned_and_padding():
    x, q = workloads.uniform_cube(50, 5, 3, seed=1)
    adj = np.full((50, 2), NONE, np.uint32)
    adj[0] = [1, 2]
    adj[1] = [2, NONE]
    ids, dists, hops, ndc = oracle.search(x, adj, q, 5, 8, 0)
    assert set(ids[:, :3].ravel()) <= {0, 1, 2}
    assert (ids[:, 3:] == NONE).all() and np.isinf(dists[:, 3:]).all()
    assert (hops == 3).all() and (ndc == 3).all()


def test_k_greater_than_L_widens_beam():
    x, q = workloads.generate(1, n=800, nq=10)
    adj, s, _ = oracle.build(x, 10, 20, 1.2)
    a = oracle.search(x, adj, q, 20, 5, s)
    b = oracle.search(x, adj, q, 20, 20, s)
    for u, v in zip(a, b):
        assert (u == v).all()


def test_entries_per_query():
    x, q = workloads.generate(1, n=800, nq=10)
    adj, s, _ = oracle.build(x, 10, 20, 1.2)
    ents = np.arange(10, dtype=np.uint32) * 7
    ids, _, _, _ = oracle.search(x, adj, q, 5, 16, ents)
    for i in range(10):
        one, _, _, _ = oracle.search(x, adj, q[i:i + 1], 5, 16, int(ents[i]))
        assert (one[0] == ids[i]).all()


# ------------------------------------------------------- alpha-CG guarantees
def _alpha_cg(n, d, alpha, tau, seed):
    """alpha-CG (Section 3.2): Algorithm 2 with V = P minus p for every p, no cap."""
    x, _ = workloads.uniform_cube(n, 1, d, seed=seed, scale=10.0)
    cand, D = oracle.knn(x, x, n - 1, exclude_self=True, mode=oracle.FP64)
    adj = oracle.prune(x, cand, D, R=n - 1, alpha=alpha, tau=tau, mode=oracle.FP64)
    return x.astype(np.float64), x, adj


def _no_near_ties(xd, adj, alpha, tau, eps=1e-9):
    """True if no pruning comparison of the graph is within eps (relative)."""
    n = len(xd)
    E = np.sqrt(((xd[:, None] - xd[None]) ** 2).sum(-1))
    for p in range(n):
        # every (u, v) pair with v kept and v closer to p than u
        kept = [int(v) for v in adj[p] if v != NONE]
        if not kept:
            continue
        a = E[p][:, None]
        rhs = alpha * E[:, kept] + (alpha + 1) * tau
        rel = np.abs(a - rhs) / np.maximum(a, 1e-300)
        rel[p] = np.inf
        if (rel < eps).any():
            return False
    return True


def _queries_near_points(xd, tau, m, seed):
    """q = v + r * unit with r < tau; kept only if v is the unique NN by a margin."""
    g = np.random.default_rng(seed)
    out = []
    while len(out) < m:
        v = g.integers(len(xd))
        u = g.standard_normal(xd.shape[1])
        u /= np.linalg.norm(u)
        q = xd[v] + g.uniform(0, 0.99 * tau) * u
        dd = np.sqrt(((xd - q) ** 2).sum(1))
        o = np.argsort(dd)
        if o[0] == v and dd[o[1]] - dd[o[0]] > 1e-6 * dd[o[1]]:
            out.append((q.astype(np.float32), int(v)))
    return out


CASES = [(120, 2, 1.3, 0.4, 1), (150, 3, 1.2, 0.5, 2), (100, 8, 1.5, 1.0, 3)]


@pytest.mark.parametrize("n,d,alpha,tau_frac,seed", CASES)
def test_alpha_cg_exact_nn_from_every_entry(n, d, alpha, tau_frac, seed):
    """Lemma 5 / Theorem 4 (first bullet): with d(q, v*) <= tau, greedy routing
    (L = 1) on the alpha-CG finds v* from every entry; per-hop contraction by
    alpha holds for all but the last two hops, and the hop count obeys
    l <= log_alpha(d(p1,q)/d(p_{l-1},q)) + 2."""
    xd0, _, _ = _alpha_cg(n, d, alpha, 0.0, seed)
    nn = np.sort(np.sqrt(((xd0[:, None] - xd0[None]) ** 2).sum(-1)), axis=1)[:, 1]
    tau = tau_frac * float(np.median(nn))
    xd, x, adj = _alpha_cg(n, d, alpha, tau, seed)
    assert _no_near_ties(xd, adj, alpha, tau)
    for q, vstar in _queries_near_points(xd, tau, 8, seed):
        dq = np.sqrt(((xd - q.astype(np.float64)) ** 2).sum(1))
        for s in range(0, n, max(1, n // 15)):
            ids, _, trace = oracle.search_trace(x, adj, q, 1, 1, s, mode=oracle.FP64)
            assert ids[0] == vstar
            path = [int(t) for t in trace]
            assert path[0] == s and path[-1] == vstar
            ell = len(path)
            for i in range(ell - 2):
                assert dq[path[i + 1]] <= dq[path[i]] / alpha * (1 + 1e-12)
            if ell >= 2 and dq[path[-2]] > 0:
                assert ell <= math.log(dq[path[0]] / dq[path[-2]], alpha) + 2 + 1e-9


@pytest.mark.parametrize("n,d,alpha,tau_frac,seed", CASES)
def test_alpha_reducible_property(n, d, alpha, tau_frac, seed):
    """Lemma 3: for every p != v*, either v* is an out-neighbour of p or some
    out-neighbour p' has d(p', q) <= d(p, q) / alpha."""
    xd0, _, _ = _alpha_cg(n, d, alpha, 0.0, seed)
    nn = np.sort(np.sqrt(((xd0[:, None] - xd0[None]) ** 2).sum(-1)), axis=1)[:, 1]
    tau = tau_frac * float(np.median(nn))
    xd, x, adj = _alpha_cg(n, d, alpha, tau, seed)
    for q, vstar in _queries_near_points(xd, tau, 8, seed + 10):
        dq = np.sqrt(((xd - q.astype(np.float64)) ** 2).sum(1))
        for p in range(n):
            if p == vstar:
                continue
            nb = [int(v) for v in adj[p] if v != NONE]
            assert vstar in nb or min(dq[nb]) <= dq[p] / alpha * (1 + 1e-12)


@pytest.mark.parametrize("n,d,alpha,tau_frac,seed", CASES)
def test_alpha_shortcut_reachability(n, d, alpha, tau_frac, seed):
    """Every non-edge (p, z) has an edge (p, p') with
    d(p', z) < (d(p, z) - (alpha+1) tau) / alpha  (Section 3.3)."""
    xd0, _, _ = _alpha_cg(n, d, alpha, 0.0, seed)
    nn = np.sort(np.sqrt(((xd0[:, None] - xd0[None]) ** 2).sum(-1)), axis=1)[:, 1]
    tau = tau_frac * float(np.median(nn))
    xd, x, adj = _alpha_cg(n, d, alpha, tau, seed)
    E = np.sqrt(((xd[:, None] - xd[None]) ** 2).sum(-1))
    for p in range(n):
        nb = [int(v) for v in adj[p] if v != NONE]
        for z in range(n):
            if z == p or z in nb:
                continue
            assert E[nb, z].min() < (E[p, z] - (alpha + 1) * tau) / alpha
