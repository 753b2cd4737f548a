"""Sub-quadratic candidates on the GPU (Algorithm 3, phases 1-2) against the
oracle, bit for bit: the NN-descent K-NN graph (ids, float32 D, rounds run),
the candidate lists from a beam search on it, and whole builds with the
CNG_BUILD_GRAPH_CANDIDATES flag (fixed and adaptive alpha, backward edges),
including the 10k x 32 mixture workload in full."""
import numpy as np
import pytest
import torch

import oracle
import paper_2510_05975_amd as cng
import workloads
from gpu_util import dev, dev_ids, f32_of, host_ids, same_f32

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", [(1, 3000, 16, 0), (1, 3000, 16, 1), (1, 3000, 16, 8),
                                  (2, 2000, 32, 6), (3, 700, 8, 4), (4, 2000, 64, 5),
                                  (2, 6000, 64, 2)])
def test_nndescent_vs_oracle(case):
    """Case (2, 6000, 64, 2) offers up to 4096 candidates per point in a round,
    more than the 2048-slot visited table holds: forgotten ids come again and
    must not enter the list twice."""
    cfg, n, K, rounds = case
    print(f"nndescent cfg{cfg} n={n} K={K} rounds={rounds}", flush=True)
    x, _ = workloads.generate(cfg, n=n, nq=1)
    ids_t, D_t, r = cng.nndescent(dev(x), K, 12345 + cfg, rounds)
    torch.cuda.synchronize()
    oids, oD, orr = oracle.nndescent(x, K, 12345 + cfg, rounds)
    assert r == orr
    assert (host_ids(ids_t) == oids).all(), np.argwhere(host_ids(ids_t) != oids)[:5]
    assert same_f32(D_t.cpu().numpy(), f32_of(oD))


@pytest.mark.parametrize("d", [3, 5, 33])
def test_nndescent_odd_dims_and_tiny(d):
    x, _ = workloads.uniform_cube(300, 1, d, seed=d)
    ids_t, D_t, r = cng.nndescent(dev(x), 20, 7, 30)
    oids, oD, orr = oracle.nndescent(x, 20, 7, 30)
    assert r == orr and (host_ids(ids_t) == oids).all()
    assert same_f32(D_t.cpu().numpy(), f32_of(oD))
    x2 = x[:10]                          # K above n - 1: rows padded
    ids_t, D_t, _ = cng.nndescent(dev(x2), 12, 1, 3)
    oids, oD, _ = oracle.nndescent(x2, 12, 1, 3)
    assert (host_ids(ids_t) == oids).all() and np.isinf(D_t.cpu().numpy()[:, 9:]).all()


@pytest.mark.parametrize("case", [(1, 3000, 16, 24, 32), (2, 2000, 24, 100, 64), (3, 600, 8, 48, 48)])
def test_graph_candidates_vs_oracle(case):
    cfg, n, K, L, C = case
    x, _ = workloads.generate(cfg, n=n, nq=1)
    g0, g0D, _ = oracle.nndescent(x, K, 3, 5)
    s = oracle.medoid(x)
    ids_t, D_t = cng.graph_candidates(dev(x), dev_ids(g0), dev(f32_of(g0D)), s, L, C)
    torch.cuda.synchronize()
    oids, oD = oracle.graph_candidates(x, g0, s, L, C)
    assert (host_ids(ids_t) == oids).all(), np.argwhere(host_ids(ids_t) != oids)[:5]
    assert same_f32(D_t.cpu().numpy(), f32_of(oD))


@pytest.mark.parametrize("case", [(1, 10000, 24, 64, dict()),
                                  (2, 4000, 32, 128, dict()),
                                  (1, 5000, 24, 64, dict(alpha_max=1.6, alpha_step=0.05,
                                                         backward=True)),
                                  (4, 3000, 32, 96, dict())])
def test_build_graph_candidates_vs_oracle(case):
    """Whole builds with phases 1-2 (K = 32, 10 rounds, beam C); case 0 is
    the 10k x 32 mixture workload in full (R = 24, C = 64)."""
    cfg, n, R, C, kw = case
    print(f"graph-candidate build cfg{cfg} n={n} {kw}", flush=True)
    x, q = workloads.generate(cfg, n=n, nq=100)
    alpha = 0.9 if kw.get("alpha_step") else 1.2
    g = cng.build(dev(x), R, C, alpha, graph_candidates=True, knn_K=32, knn_rounds=10,
                  knn_seed=99, **kw)
    torch.cuda.synchronize()
    oadj, oe, oadded = oracle.build(x, R, C, alpha, knn_K=32, knn_seed=99, knn_rounds=10,
                                    cand_L=C, **kw)
    assert g.entry == oe
    assert (host_ids(g.adj) == oadj).all(), np.argwhere(host_ids(g.adj) != oadj)[:5]
    assert g.stats["connect_added"] == oadded and g.stats["knn_rounds_run"] >= 1
    ids_t, d_t, _, _ = cng.search(dev(x), g.adj, dev(q), 10, 48, g.entry)
    oids, od, _, _ = oracle.search(x, oadj, q, 10, 48, oe)
    assert (host_ids(ids_t) == oids).all() and same_f32(d_t.cpu().numpy(), f32_of(od))
