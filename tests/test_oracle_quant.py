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


# ---------------------------------------------------------------- fp8 dot form of the score
def _fp8_score(enc, q, v):
    """The oracle's fp8 score, checked to be what its search ranks by (a
    one-point search: the entry's row is empty)."""
    s = float(oracle.fp8_score(enc, q, v))
    adj = np.full((len(enc[0]), 1), oracle.NONE, np.uint32)
    ids, dists, _, _ = oracle.search_fp8(enc, None, adj, np.asarray(q, np.float32)[None], 1, 1, v)
    assert ids[0, 0] == v and dists[0, 0] == float(np.sqrt(np.float32(s)))
    return s


def test_fp8_encode_matches_dequantized_values():
    x, _ = workloads.generate(1, n=300, nq=1)
    x[5] = 0.0
    c, sc, n2 = oracle.fp8_encode(x)
    deq, sc2 = oracle.dequantized(x, oracle.FP8)
    assert np.array_equal(sc, sc2)
    assert np.array_equal((c * sc[:, None]).astype(np.float32), deq)
    assert sc[5] == 1.0 and n2[5] == 0.0
    # n2 = fl(fl(s s) dot(c, c)) with the fixed-order dot
    for p in (0, 7, 299):
        assert n2[p] == np.float32(np.float32(sc[p] * sc[p]) * oracle.dot_f32(c[p], c[p]))


def test_fp8_score_is_squared_distance_when_exact():
    """Scale a power of two, stored values exact in E4M3, small integer query:
    every float32 step is exact, so the dot form equals |q - x|^2 exactly."""
    x = np.array([[448.0, -224.0, 96.0, 0.0, 12.0, -3.0, 7.0, 1.0],
                  [224.0, 112.0, -56.0, 28.0, 14.0, 0.0, -7.0, 3.5]], np.float32)
    enc = oracle.fp8_encode(x)
    assert enc[1].tolist() == [1.0, 0.5]
    assert np.array_equal(enc[0] * enc[1][:, None], x)
    q = np.array([5.0, -2.0, 9.0, 1.0, 0.0, 4.0, -6.0, 2.0], np.float32)
    for v in (0, 1):
        want = float(((q.astype(np.float64) - x[v]) ** 2).sum())
        assert _fp8_score(enc, q, v) == want


def test_fp8_score_error_bound_and_clamp():
    """Against |q - s c|^2 in float64 the dot form errs by at most
    gamma_{d+4} (|q|^2 + 2 s |q.c| + s^2 |c|^2) (float32 accumulation and the
    three combining steps); it never goes below zero, also for a query equal
    to a stored vector, where the exact value is 0."""
    x, q = workloads.generate(1, n=50, nq=20)
    c, sc, n2 = enc = oracle.fp8_encode(x)
    d = x.shape[1]
    u = 2.0 ** -24
    gam = (d + 4) * u / (1 - (d + 4) * u)
    deq = (c * sc[:, None]).astype(np.float64)
    for i in range(20):
        for v in range(0, 50, 7):
            exact = float(((q[i].astype(np.float64) - deq[v]) ** 2).sum())
            mag = float((q[i].astype(np.float64) ** 2).sum() + 2 * sc[v] * np.abs(q[i] @ c[v]).sum() +
                        sc[v] ** 2 * (c[v].astype(np.float64) ** 2).sum())
            assert abs(_fp8_score(enc, q[i], v) - exact) <= gam * mag
    for v in range(50):
        s0 = _fp8_score(enc, deq[v].astype(np.float32), v)
        assert 0.0 <= s0 <= gam * 4 * float((deq[v] ** 2).sum())


def test_fp8_search_large_beam_is_exact_knn():
    """A beam as large as the reachable set explores everything; the float32
    re-rank of the whole beam then returns the exact k nearest neighbours."""
    x, q = workloads.generate(1, n=600, nq=15)
    adj, e, _ = oracle.build(x, 10, 20, 1.2)
    assert oracle.reachable(adj, e).all()
    ids, dists, hops, ndc = oracle.search_fp8(oracle.fp8_encode(x), x, adj, q, 10, 600, e)
    gt, gD = oracle.knn(q, x, 10)
    assert (ids == gt).all() and (hops == 600).all()
    assert np.array_equal(dists, np.sqrt(gD.astype(np.float32)).astype(np.float64))
