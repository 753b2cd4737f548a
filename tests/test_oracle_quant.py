"""Pins for the oracle's reduced-precision storage (bf16, fp8-E4M3 with a
per-vector scale) and for the re-ranked beam search of the precision form."""
import numpy as np
import pytest
import torch

import oracle
import workloads


def test_bf16_matches_torch_cast():
    g = np.random.default_rng(0)
    x = np.concatenate([g.standard_normal(20000) * 10.0 ** g.uniform(-30, 30, 20000),
                        np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 255.0, 257.0, 0.0])])
    x = x.astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([oracle.round_bf16(v) for v in x], np.float32)
    assert np.array_equal(got, want)


def test_e4m3_matches_torch_cast_in_range():
    g = np.random.default_rng(1)
    x = np.concatenate([g.uniform(-448, 448, 20000), g.standard_normal(5000) * 1e-2,
                        np.array([448.0, -448.0, 0.0, 2 ** -9, 2 ** -10, 3 * 2 ** -10, 17.0, 19.0])])
    x = x.astype(np.float32)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    got = np.array([oracle.round_e4m3(v) for v in x], np.float32)
    assert np.array_equal(got, want)


def test_e4m3_hand_values_and_saturation():
    # spacing 32 in [256, 512): 300 -> 288; 304 is a tie between 288 and 320 -> even mantissa 320
    assert oracle.round_e4m3(300.0) == 288.0
    assert oracle.round_e4m3(304.0) == 320.0
    assert oracle.round_e4m3(460.0) == 448.0 and oracle.round_e4m3(1e6) == 448.0
    assert oracle.round_e4m3(-1e6) == -448.0
    assert oracle.round_e4m3(0.001) == 2 ** -9          # subnormal step
    assert oracle.round_e4m3(2 ** -10) == 0.0            # tie -> even (zero)


def test_error_bounds():
    g = np.random.default_rng(2)
    x = (g.standard_normal(5000) * 100).astype(np.float32)
    for v in x:
        assert abs(oracle.round_bf16(v) - v) <= 2 ** -8 * abs(v)  # 8 significant bits
        if 2 ** -6 <= abs(v) <= 448:
            assert abs(oracle.round_e4m3(v) - v) <= 2 ** -4 * abs(v)


def test_dequantized_fp8_scale_and_values():
    g = np.random.default_rng(3)
    x = (g.standard_normal((50, 24)) * 7).astype(np.float32)
    x[7] = 0.0
    deq, sc = oracle.dequantized(x, oracle.FP8)
    m = np.abs(x).max(1)
    assert sc[7] == 1.0 and (deq[7] == 0).all()
    ok = m > 0
    np.testing.assert_array_equal(sc[ok], (m[ok] / np.float32(448)).astype(np.float32))
    # the largest element of every vector maps to 448 * s (or its rounding neighbour)
    i = np.abs(x).argmax(1)
    top = np.abs(deq[np.arange(50), i])[ok]
    np.testing.assert_allclose(top, m[ok], rtol=2 ** -4)
    # elementwise relative error of fp8 <= 2^-4 for entries in the normal range
    rel = np.abs(deq - x) / np.maximum(np.abs(x), 1e-30)
    big = np.abs(x) / sc[:, None] >= 2 ** -6
    assert (rel[big] <= 2 ** -4 + 1e-7).all()


def test_dequantized_bf16_exact_on_small_integers():
    x, _ = workloads.generate(2, n=500, nq=1)
    deq, _ = oracle.dequantized(x, oracle.BF16)
    assert np.array_equal(deq, x)


def test_rerank_with_same_vectors_is_plain_search():
    x, q = workloads.generate(1, n=2000, nq=40)
    adj, e, _ = oracle.build(x, 16, 32, 1.2)
    a = oracle.search(x, adj, q, 10, 32, e)
    b = oracle.search_rerank(x, x, adj, q, 10, 32, e)
    c = oracle.search_rerank(x, None, adj, q, 10, 32, e)
    for u, v, w in zip(a, b, c):
        assert (u == v).all() and (u == w).all()


def test_rerank_recovers_exact_distances():
    """Searching on fp8 vectors and re-ranking with float32 returns float32
    distances of the returned ids; it can only improve on the unreranked beam."""
    x, q = workloads.generate(1, n=2000, nq=40)
    adj, e, _ = oracle.build(x, 16, 32, 1.2)
    deq, _ = oracle.dequantized(x, oracle.FP8)
    ids, dists, _, _ = oracle.search_rerank(deq, x, adj, q, 10, 32, e)
    for i in range(len(q)):
        exact = [np.sqrt(np.float32(oracle.dist_f32(q[i], x[j]))) for j in ids[i]]
        assert np.array_equal(np.float32(exact), dists[i].astype(np.float32))
        assert (np.diff(dists[i]) >= 0).all()


def test_rerank_hand_traced_whole_beam():
    """The re-rank covers every entry of the final beam (not only its first
    k) and nothing outside it: hand-traced in tests/golden/rerank_line.json."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rerank_line.json")))
    sp = np.array(g["search_points"], np.float32)
    rp = np.array(g["rerank_points"], np.float32)
    adj = np.array(g["adj"], np.uint32)
    q = np.array([g["query"]], np.float32)
    for c in g["cases"]:
        for mode in (oracle.FP32, oracle.FP64):
            ids, dists, hops, ndc = oracle.search_rerank(sp, rp, adj, q, c["k"], g["L"], g["entry"],
                                                         mode=mode)
            assert ids[0].tolist() == c["expect_ids"]
            assert dists[0].tolist() == c["expect_dists"]
            assert hops[0] == 3 and ndc[0] == 4
