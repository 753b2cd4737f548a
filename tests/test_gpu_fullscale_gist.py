"""Parity at full size on the 1M x 960 GIST-shaped workload (R = 48, C = 192,
alpha = 1.2): the streamed hi/lo-split candidate filter runs in eight passes of
131072 rows there, so this covers row offsets past zero and the pass loop at
the real shape.  The oracle checks sampled outputs one by one: candidate rows
(first, last, and rows inside later passes), pruned rows, the entry point, and
sampled queries of the 1000-query batch at the beam width that reaches
recall@10 0.95 on this graph, float32 and bf16 storage with float32 re-rank.

Equality is bit for bit (ids, adjacency, float32 distances)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2510_05975_amd as cng
import workloads
from gpu_util import dev, f32_of, host_ids, same_f32

pytestmark = pytest.mark.gpu

R, C, ALPHA, K, L = 48, 192, 1.2, 10, 352


@pytest.fixture(scope="module")
def gist():
    print("fullscale gist: generate 1M x 960 + 1000 queries", flush=True)
    x, q = workloads.generate(3)
    xd, qd = dev(x), dev(q)
    print("fullscale gist: cng_knn (all rows) + cng_prune", flush=True)
    ids_t, D_t, ovf = cng.knn(xd, xd, C, exclude_self=True)
    pruned_t = cng.prune(xd, ids_t, D_t, R, ALPHA, 0.0, width=R + 1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(960)
    n = len(x)
    # first and last row, the first and last row of the second and last pass
    # (passes of 131072 rows), and random rows
    rows = np.unique(np.concatenate([[0, n - 1, 131071, 131072, 7 * 131072, 7 * 131072 + 1],
                                     rng.integers(0, n, 10)]))
    out = dict(x=x, q=q, xd=xd, qd=qd, rows=rows, ids=host_ids(ids_t)[rows],
               D=D_t.cpu().numpy()[rows], pruned=host_ids(pruned_t))
    del ids_t, D_t, pruned_t
    print("fullscale gist: cng_build", flush=True)
    g = cng.build(xd, R, C, ALPHA)
    torch.cuda.synchronize()
    out.update(g=g, adj=host_ids(g.adj))
    return out


def test_gist_candidates_and_pruned_rows(gist):
    x, rows = gist["x"], gist["rows"]
    n = len(x)
    print(f"fullscale gist: oracle knn on {len(rows)} rows", flush=True)
    oids, oD = oracle.knn(x[rows], x, C + 1)
    cand = np.full((n, C), oracle.NONE, np.uint32)
    candD = np.full((n, C), np.inf)
    for j, p in enumerate(rows):
        keep = oids[j] != p
        exp_ids, exp_D = oids[j][keep][:C], oD[j][keep][:C]
        assert (gist["ids"][j] == exp_ids).all(), p
        assert same_f32(gist["D"][j], f32_of(exp_D)), p
        cand[p], candD[p] = exp_ids, exp_D
    oadj = oracle.prune(x, cand, candD, R, ALPHA, 0.0, width=R + 1)
    assert (gist["pruned"][rows] == oadj[rows]).all()


def test_gist_build_entry_and_connectivity(gist):
    g, adj, pruned = gist["g"], gist["adj"], gist["pruned"]
    assert g.entry == oracle.medoid(gist["x"])
    # the build's pruned columns are the stage outputs; connectivity only
    # fills spare slots, and everything is reachable from the entry
    valid = pruned != oracle.NONE
    assert (adj[valid] == pruned[valid]).all()
    assert oracle.reachable(adj, g.entry).all()
    assert int(((adj != oracle.NONE) & ~valid).sum()) == g.stats["connect_added"]


@pytest.mark.parametrize("store", [None, cng.BF16])
def test_gist_search_sampled(gist, store):
    g, adj = gist["g"], gist["adj"]
    if store is None:
        ids_t, d_t, _, _ = cng.search(gist["xd"], g.adj, gist["qd"], K, L, g.entry)
    else:
        st = cng.quantize(gist["xd"], store)
        ids_t, d_t, _, _ = cng.search_quantized(gist["xd"], st, g.adj, gist["qd"], K, L, g.entry)
    torch.cuda.synchronize()
    rng = np.random.default_rng(352)
    qs = np.unique(np.concatenate([[0, len(gist["q"]) - 1], rng.integers(0, len(gist["q"]), 46)]))
    if store is None:
        oids, od, _, _ = oracle.search(gist["x"], adj, gist["q"][qs], K, L, g.entry)
    else:
        deq, _ = oracle.dequantized(gist["x"], store)
        oids, od, _, _ = oracle.search_rerank(deq, gist["x"], adj, gist["q"][qs], K, L, g.entry)
    assert (host_ids(ids_t)[qs] == oids).all()
    assert same_f32(d_t.cpu().numpy()[qs], f32_of(od))
