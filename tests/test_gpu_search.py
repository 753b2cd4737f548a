"""GPU beam search (Algorithm 1) against the CPU oracle on the same graph:
ids, distances, hops and distance-evaluation counts bit for bit."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2510_05975_amd as cng
import workloads
from gpu_util import dev, dev_ids, f32_of, host_ids, same_f32

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gpu_search(x, adj, q, k, L, entries, vlog2=14):
    if isinstance(entries, (int, np.integer)):
        ent = int(entries)
    else:
        ent = dev_ids(np.asarray(entries, np.uint32))
    ids, d, h, n = cng.search(dev(x), dev_ids(adj), dev(q), k, L, ent, visited_log2=vlog2, stats=True)
    torch.cuda.synchronize()
    return host_ids(ids), d.cpu().numpy(), h.cpu().numpy().astype(np.uint32), n.cpu().numpy().astype(np.uint32)


def assert_same(g, o, check_ndc=True):
    ids, d, h, n = g
    oids, od, oh, on = o
    assert (ids == oids).all(), np.argwhere(ids != oids)[:5]
    assert same_f32(d, f32_of(od))
    assert (h == oh).all()
    if check_ndc:
        assert (n == on).all()


@pytest.fixture(scope="module")
def cfg1():
    x, q = workloads.generate(1)
    adj, e, _ = oracle.build(x, 24, 64, 1.2)
    return x, q, adj, e


@pytest.mark.parametrize("L", [1, 8, 32, 64, 100, 256])
def test_cfg1_bit_exact(cfg1, L):
    x, q, adj, e = cfg1
    print(f"search cfg1 L={L}", flush=True)
    assert_same(gpu_search(x, adj, q, 10, L, e), oracle.search(x, adj, q, 10, L, e))


def test_small_visited_table_same_results(cfg1):
    """A table that forgets changes only the number of distance evaluations."""
    x, q, adj, e = cfg1
    o = oracle.search(x, adj, q, 10, 64, e)
    g = gpu_search(x, adj, q, 10, 64, e, vlog2=6)
    assert_same(g, o, check_ndc=False)
    assert (g[3] >= o[3]).all() and (g[3] > o[3]).any()


def test_k_above_L_and_large_k(cfg1):
    x, q, adj, e = cfg1
    for k, L in [(20, 5), (64, 64), (100, 16), (512, 512)]:
        assert_same(gpu_search(x, adj, q, k, L, e), oracle.search(x, adj, q, k, L, e))


def test_per_query_entries(cfg1):
    x, q, adj, e = cfg1
    ents = (np.arange(len(q), dtype=np.uint32) * 97) % len(x)
    assert_same(gpu_search(x, adj, q, 10, 32, ents), oracle.search(x, adj, q, 10, 32, ents))


def test_hand_traced_line():
    g = json.load(open(os.path.join(GOLD, "beam_line.json")))
    pts = np.array(g["points"], np.float32)
    adj = np.array(g["adj"], np.uint32)
    q = np.array([g["query"]], np.float32)
    ids, d, h, n = gpu_search(pts, adj, q, g["k"], g["L"], g["entry"])
    assert list(ids[0]) == g["expect_ids"] and list(d[0]) == g["expect_dists"]
    assert h[0] == len(g["expect_hops"]) and n[0] == g["expect_ndc"]


@pytest.mark.parametrize("d", [1, 3, 5, 31, 32, 33, 64, 65, 96, 100, 128, 129, 256, 300, 960, 1500,
                               3001, 4096])
def test_dimensions(d):
    print(f"search d={d}", flush=True)
    x, q = workloads.uniform_cube(600, 20, d, seed=d)
    adj, e, _ = oracle.build(x, 10, 20, 1.2)
    assert_same(gpu_search(x, adj, q, 10, 24, e), oracle.search(x, adj, q, 10, 24, e))


@pytest.mark.parametrize("d", [300, 960])
def test_batch_size_forms(d):
    """Launches of at most 1024 queries load twice the vectors per batch for
    257 <= d <= 1024; both forms match the oracle."""
    x, q = workloads.uniform_cube(1200, 1100, d, seed=d + 1)
    adj, e, _ = oracle.build(x, 10, 20, 1.2)
    o = oracle.search(x, adj, q, 10, 24, e)
    assert_same(gpu_search(x, adj, q, 10, 24, e), o)  # 1100 queries
    small = gpu_search(x, adj, q[:100], 10, 24, e)
    assert_same(small, tuple(a[:100] for a in o))


def test_unreachable_padding_and_invalid_ids():
    x, q = workloads.uniform_cube(50, 5, 3, seed=1)
    adj = np.full((50, 3), oracle.NONE, np.uint32)
    adj[0] = [1, 2, oracle.NONE]
    adj[1] = [2, 999, 3]          # 999 >= n ends the row like a sentinel
    o = oracle.search(x, adj, q, 5, 8, 0)
    g = gpu_search(x, adj, q, 5, 8, 0)
    assert_same(g, o)
    assert (g[0][:, 3:] == oracle.NONE).all() and np.isinf(g[1][:, 3:]).all()


def test_empty_batch():
    x, q = workloads.uniform_cube(50, 1, 3, seed=1)
    adj = np.full((50, 2), oracle.NONE, np.uint32)
    ids, d, _, _ = cng.search(dev(x), dev_ids(adj), dev(q[:0]), 5, 8, 0)
    assert ids.shape == (0, 5)


def test_wide_rows_over_64():
    """Rows wider than one wavefront are read in chunks."""
    x, q = workloads.uniform_cube(400, 30, 16, seed=4)
    cand, D = oracle.knn(x, x, 150, exclude_self=True)
    adj = np.ascontiguousarray(cand[:, :150])
    assert_same(gpu_search(x, adj, q, 10, 40, 0), oracle.search(x, adj, q, 10, 40, 0))


def test_sift_like_reduced():
    x, q = workloads.generate(2, n=6000, nq=200)
    adj, e, _ = oracle.build(x, 32, 128, 1.2)
    for L in (16, 64):
        assert_same(gpu_search(x, adj, q, 10, L, e), oracle.search(x, adj, q, 10, L, e))


def test_cooperative_search_edge_cases():
    """Few queries with d > 256 run several waves per query: per-query entries,
    an invalid entry (nothing reachable: the query's wave leaves at once and
    releases its helpers), k above L."""
    x, q = workloads.uniform_cube(900, 6, 300, seed=11)
    adj, e, _ = oracle.build(x, 10, 20, 1.2)
    ents = np.array([e, 5, 17, 899, 900, 3], np.uint32)   # 900 >= n: invalid
    ids, d, _, _ = gpu_search(x, adj, q, 12, 8, ents)
    for i in range(len(q)):
        if ents[i] >= len(x):
            assert (ids[i] == oracle.NONE).all() and np.isinf(d[i]).all()
            continue
        o = oracle.search(x, adj, q[i:i + 1], 12, 8, int(ents[i]))
        assert (ids[i] == o[0][0]).all() and same_f32(d[i:i + 1], f32_of(o[1]))
