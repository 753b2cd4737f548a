"""Parity at full size: the 1M x 128 integer-valued (SIFT-shaped) workload with
R = 32, C = 128, alpha = 1.2, searched with the 10k-query batch in the launch
configuration the benchmark times.  The oracle checks sampled outputs one by one
(candidate rows, pruned rows, search results) and the stages it can afford in
full (entry point, connectivity on the GPU's pruned graph).

Equality is bit for bit throughout (ids, adjacency, float32 distances)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2510_05975_amd as cng
import workloads
from gpu_util import dev, f32_of, host_ids, oracle_qsearch, same_f32

pytestmark = pytest.mark.gpu

R, C, ALPHA, K = 32, 128, 1.2, 10


@pytest.fixture(scope="module")
def full():
    print("fullscale: generate sift_like 1M x 128 + 10k queries", flush=True)
    x, q = workloads.generate(2)
    xd, qd = dev(x), dev(q)
    print("fullscale: cng_build", flush=True)
    g = cng.build(xd, R, C, ALPHA)
    torch.cuda.synchronize()
    rng = np.random.default_rng(20251007)
    rows = np.unique(np.concatenate([[0, len(x) - 1], rng.integers(0, len(x), 30)]))
    qs = np.unique(np.concatenate([[0, len(q) - 1], rng.integers(0, len(q), 190)]))
    return dict(x=x, q=q, xd=xd, qd=qd, g=g, adj=host_ids(g.adj), rows=rows, qs=qs)


def test_entry_point_full(full):
    assert full["g"].entry == oracle.medoid(full["x"])


def test_candidates_pruning_connectivity_full(full):
    x, rows = full["x"], full["rows"]
    n = len(x)
    print("fullscale: cng_knn + cng_prune on all rows", flush=True)
    ids_t, D_t, ovf = cng.knn(full["xd"], full["xd"], C, exclude_self=True)
    pruned_t = cng.prune(full["xd"], ids_t, D_t, R, ALPHA, 0.0, width=R + 1)
    torch.cuda.synchronize()
    ids = host_ids(ids_t)
    D = D_t.cpu().numpy()
    pruned = host_ids(pruned_t)
    del ids_t, D_t, pruned_t

    # candidate rows: the first C of P \ {p} by (D, id), from C + 1 of P minus p
    print(f"fullscale: oracle knn on {len(rows)} rows", flush=True)
    oids, oD = oracle.knn(x[rows], x, C + 1)
    for j, p in enumerate(rows):
        keep = oids[j] != p
        exp_ids, exp_D = oids[j][keep][:C], oD[j][keep][:C]
        assert (ids[p] == exp_ids).all(), p
        assert same_f32(D[p], f32_of(exp_D)), p

    # pruned rows (Alg. 2 on the oracle's candidate lists of the sampled rows)
    print("fullscale: oracle prune on the sampled rows", flush=True)
    cand = np.full((n, C), oracle.NONE, np.uint32)
    candD = np.full((n, C), np.inf)
    for j, p in enumerate(rows):
        keep = oids[j] != p
        cand[p], candD[p] = oids[j][keep][:C], oD[j][keep][:C]
    oadj = oracle.prune(x, cand, candD, R, ALPHA, 0.0, width=R + 1)
    del cand, candD
    assert (pruned[rows] == oadj[rows]).all()

    # connectivity in full on the GPU's pruned graph, against the whole build
    print("fullscale: oracle connect on the pruned graph", flush=True)
    cadj, added, rounds = oracle.connect(x, pruned, full["g"].entry, C)
    assert (full["adj"] == cadj).all()
    assert full["g"].stats["connect_added"] == added
    assert oracle.reachable(full["adj"], full["g"].entry).all()


@pytest.mark.parametrize("L", [16, 96, 256])
def test_search_sampled_full(full, L):
    """Whole 10k batch in the benchmark's launch configuration (default visited
    table), sampled queries against the oracle."""
    ids_t, d_t, _, _ = cng.search(full["xd"], full["g"].adj, full["qd"], K, L, full["g"].entry)
    _, _, hops_t, _ = cng.search(full["xd"], full["g"].adj, full["qd"], K, L, full["g"].entry,
                                 stats=True)
    torch.cuda.synchronize()
    ids, dists, hops = host_ids(ids_t), d_t.cpu().numpy(), hops_t.cpu().numpy()
    qs = full["qs"]
    oids, od, ohops, _ = oracle.search(full["x"], full["adj"], full["q"][qs], K, L,
                                       full["g"].entry)
    assert (ids[qs] == oids).all()
    assert same_f32(dists[qs], f32_of(od))
    assert (hops[qs] == ohops).all()


@pytest.mark.parametrize("dtype", [cng.BF16, cng.FP8])
def test_search_quantized_sampled_full(full, dtype):
    store = cng.quantize(full["xd"], dtype)
    ids_t, d_t, _, _ = cng.search_quantized(full["xd"], store, full["g"].adj, full["qd"], K, 96,
                                            full["g"].entry)
    torch.cuda.synchronize()
    ids, dists = host_ids(ids_t), d_t.cpu().numpy()
    qs = full["qs"]
    oids, od, _, _ = oracle_qsearch(dtype, full["x"], full["adj"], full["q"][qs], K, 96,
                                    full["g"].entry)
    assert (ids[qs] == oids).all()
    assert same_f32(dists[qs], f32_of(od))


def test_adaptive_and_backward_sampled_full(full):
    """The paper's alpha-CNG stages at full size: adaptive pruning (Algorithm 4)
    on sampled rows against the oracle, the backward-edge phase on sampled rows
    against its definition (own row plus in-edge sources, by (D, id), cut to C,
    pruned adaptively when longer than R), connectivity in full, and sampled
    searches on the finished graph."""
    x, rows = full["x"], full["rows"]
    n = len(x)
    A0, AMAX, STEP = 0.9, 1.6, 0.05
    print("fullscale: adaptive prune + backward on the GPU", flush=True)
    ids_t, D_t, _ = cng.knn(full["xd"], full["xd"], C, exclude_self=True)
    p2_t = cng.prune(full["xd"], ids_t, D_t, R, A0, 0.0, width=R + 1, alpha_max=AMAX,
                     alpha_step=STEP)
    p3_t = p2_t.clone()
    cng.backward(full["xd"], p3_t, R, C, A0, 0.0, alpha_max=AMAX, alpha_step=STEP)
    torch.cuda.synchronize()
    ids, D = host_ids(ids_t), D_t.cpu().numpy()
    p2, p3 = host_ids(p2_t), host_ids(p3_t)
    del ids_t, D_t, p2_t, p3_t

    def oracle_rows(cands):
        """Adaptive pruning of the given candidate lists (row -> ids by (D, id))."""
        width = max(len(v) for v in cands.values())
        cand = np.full((n, width), oracle.NONE, np.uint32)
        candD = np.full((n, width), np.inf)
        for p, v in cands.items():
            cand[p, : len(v)] = v
            candD[p, : len(v)] = [oracle.dist_f32(x[p], x[u]) for u in v]
        return oracle.prune(x, cand, candD, R, A0, width=R + 1, alpha_max=AMAX, alpha_step=STEP)

    # phase 2 on sampled rows (the candidate lists checked in full elsewhere)
    o2 = oracle_rows({int(p): [int(u) for u in ids[p]] for p in rows})
    assert (p2[rows] == o2[rows]).all()
    assert all(float(D[p][j]) == float(np.float32(oracle.dist_f32(x[p], x[ids[p][j]])))
               for p in rows[:4] for j in range(0, C, 17))

    # phase 3 on sampled rows: own row plus sources of in-edges (a set), by (D, id)
    valid = p2 != oracle.NONE
    src_u = np.repeat(np.arange(n, dtype=np.int64), valid.sum(1))
    dst_v = p2[valid].astype(np.int64)
    cands, short = {}, {}
    for p in rows:
        V = set(int(v) for v in p2[p] if v != oracle.NONE) | set(src_u[dst_v == p].tolist())
        V = sorted(V, key=lambda u: (float(oracle.dist_f32(x[p], x[u])), u))[:C]
        (cands if len(V) > R else short)[int(p)] = V
    if cands:
        o3 = oracle_rows(cands)
        for p in cands:
            assert (p3[p] == o3[p]).all(), p
    for p, V in short.items():
        assert [int(v) for v in p3[p] if v != oracle.NONE] == V, p

    # connectivity in full on the GPU's phase-3 graph, against the whole build
    g = cng.build(full["xd"], R, C, A0, alpha_max=AMAX, alpha_step=STEP, backward=True)
    torch.cuda.synchronize()
    gadj = host_ids(g.adj)
    cadj, added, _ = oracle.connect(x, p3, g.entry, C)
    assert (gadj == cadj).all() and g.stats["connect_added"] == added

    # sampled searches on the finished graph
    qs = full["qs"]
    ids_t, d_t, _, _ = cng.search(full["xd"], g.adj, full["qd"], K, 96, g.entry)
    torch.cuda.synchronize()
    oids, od, _, _ = oracle.search(x, gadj, full["q"][qs], K, 96, g.entry)
    assert (host_ids(ids_t)[qs] == oids).all()
    assert same_f32(d_t.cpu().numpy()[qs], f32_of(od))
