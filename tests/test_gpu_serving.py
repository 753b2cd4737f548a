"""Serving loop (continuous batching on a persistent device grid): each
result is the same alone and in a mix of concurrent requests with different
k and L, equals the batched search kernels and the oracle's Algorithm 1 (plain
float32, or fp8 storage with float32 re-rank) bit for bit; admission is by
footprint (a request still in flight blocks only its own bytes); a grid that
left after an idle spell is relaunched by the next submit."""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_2510_05975_amd as cng
import workloads
from gpu_util import dev, host_ids, same_f32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def index():
    x, q = workloads.generate(2, n=30000, nq=600)
    xd = dev(x)
    g = cng.build(xd, 32, 64, 1.2)
    torch.cuda.synchronize()
    return x, q, xd, g


def batched(xd, g, q, k, L, store=None):
    if store is None:
        ids, d, _, _ = cng.search(xd, g.adj, dev(q), k, L, g.entry)
    else:
        ids, d, _, _ = cng.search_quantized(xd, store, g.adj, dev(q), k, L, g.entry)
    torch.cuda.synchronize()
    return host_ids(ids), d.cpu().numpy()


@pytest.mark.parametrize("dtype", [None, cng.FP8])
def test_alone_equals_mix_equals_batched(index, dtype):
    x, q, xd, g = index
    store = None if dtype is None else cng.quantize(xd, dtype)
    rng = np.random.default_rng(7)
    probe = q[:40]
    with cng.Server(xd, g.adj, g.entry, store=store, max_k=100) as srv:
        print(f"serving dtype={dtype}: alone", flush=True)
        alone = srv.wait(srv.submit(probe, 10, 64))
        # a mix of concurrent requests, the probe request in the middle
        reqs = []
        for i in range(60):
            if i == 30:
                reqs.append(("probe", srv.submit(probe, 10, 64), probe, 10, 64))
                continue
            nq = int(rng.integers(1, 65))
            k = int(rng.choice([1, 10, 100]))
            L = int(rng.choice([32, 64, 128, 256]))
            sel = q[rng.integers(0, len(q), nq)]
            r = srv.submit(sel, k, L)
            while r is None:  # not admitted: drain completed requests and retry
                for j, item in enumerate(reqs):
                    if item[1] is not None and len(item) == 5:
                        out = srv.poll(item[1])
                        if out is not None:
                            reqs[j] = item + (out,)
                r = srv.submit(sel, k, L)
            reqs.append(("mix", r, sel, k, L))
        print("serving: mix submitted", flush=True)
        results = []
        for item in reqs:
            out = item[5] if len(item) == 6 else srv.wait(item[1])
            results.append((item, out))
    adj = host_ids(g.adj)
    enc = None if dtype is None else oracle.fp8_encode(x)
    for (tag, _, sel, k, L, *_), (ids, dists) in results:
        bi, bd = batched(xd, g, sel, k, L, store)
        assert np.array_equal(ids, bi) and np.array_equal(dists, bd), (tag, k, L)
        if dtype is None:
            oi, od, _, _ = oracle.search(x, adj, sel, k, L, g.entry)
        else:
            oi, od, _, _ = oracle.search_fp8(enc, x, adj, sel, k, L, g.entry)
        assert np.array_equal(ids, oi) and same_f32(dists, od.astype(np.float32)), (tag, k, L)
        if tag == "probe":
            assert np.array_equal(ids, alone[0]) and np.array_equal(dists, alone[1])


def _footprint(nq, d, k):
    return -(-nq * (4 * d + 8 * k) // 64) * 64


def test_footprint_admission_long_request_does_not_block(index):
    """Arena of 64 queries at k = 10.  A (40 queries, L = 256) stays in flight
    (not polled) while B (24 queries) fills the rest; C (24 queries) is refused
    until B is retired and then takes B's bytes, although A still holds the
    bytes before them.  A request with k = 1 costs less and is admitted into a
    smaller gap."""
    x, q, xd, g = index
    d = x.shape[1]
    arena = _footprint(64, d, 10)
    with cng.Server(xd, g.adj, g.entry, max_k=10, waves=256, arena_bytes=arena) as srv:
        a = srv.submit(q[:40], 10, 256)
        b = srv.submit(q[40:64], 10, 32)
        assert a is not None and b is not None
        st = srv.stats()
        assert st["arena_used"] == _footprint(40, d, 10) + _footprint(24, d, 10) == arena
        assert srv.submit(q[64:88], 10, 32) is None          # no room while B is in flight
        assert srv.submit(q[64:65], 1, 32) is None           # not even one small query
        rb = srv.wait(b)
        c = srv.submit(q[64:88], 10, 32)                     # A is still in flight
        assert c is not None
        assert srv.stats()["in_flight"] == 2
        rc = srv.wait(c)
        e = srv.submit(q[88:104], 1, 64)                     # 16 queries, k = 1: fits B's old bytes
        assert e is not None and _footprint(16, d, 1) <= _footprint(24, d, 10)
        re_ = srv.wait(e)
        ra = srv.wait(a)
        st = srv.stats()
        assert st["arena_used"] == 0 and st["refused"] == 2 and st["in_flight"] == 0
    adj = host_ids(g.adj)
    for sel, k, L, (ids, dists) in [(q[:40], 10, 256, ra), (q[40:64], 10, 32, rb),
                                    (q[64:88], 10, 32, rc), (q[88:104], 1, 64, re_)]:
        oi, od, _, _ = oracle.search(x, adj, sel, k, L, g.entry)
        assert np.array_equal(ids, oi) and same_f32(dists, od.astype(np.float32))


def test_relaunch_after_idle_exit(index):
    """With a short idle limit the grid leaves once the ring is empty; the
    next submit launches a fresh grid, which serves the request."""
    x, q, xd, g = index
    adj = host_ids(g.adj)
    with cng.Server(xd, g.adj, g.entry, max_k=10, idle_checks=4000) as srv:
        r1 = srv.wait(srv.submit(q[:8], 10, 48))
        t0 = time.time()
        while srv.stats()["running"] and time.time() - t0 < 20:
            time.sleep(0.01)
        st = srv.stats()
        assert st["running"] == 0, "the grid did not leave after its idle limit"
        r2 = srv.wait(srv.submit(q[8:16], 10, 48), timeout=20)
        assert srv.stats()["launches"] == st["launches"] + 1
    for sel, (ids, dists) in [(q[:8], r1), (q[8:16], r2)]:
        oi, od, _, _ = oracle.search(x, adj, sel, 10, 48, g.entry)
        assert np.array_equal(ids, oi) and same_f32(dists, od.astype(np.float32))


def test_admission_refuses_then_accepts(index):
    x, q, xd, g = index
    with cng.Server(xd, g.adj, g.entry, max_k=10, waves=64, capacity=64) as srv:
        a = srv.submit(q[:50], 10, 32)
        assert a is not None
        b = srv.submit(q[50:100], 10, 32)     # 100 > 64 slots: refused
        assert b is None
        srv.wait(a)
        b = srv.submit(q[50:100], 10, 32)
        assert b is not None
        ids, _ = srv.wait(b)
        bi, _ = batched(xd, g, q[50:100], 10, 32)
        assert np.array_equal(ids, bi)


def test_per_query_entries_and_restart(index):
    x, q, xd, g = index
    ents = (np.arange(20, dtype=np.uint32) * 977) % len(x)
    for _ in range(2):
        with cng.Server(xd, g.adj, g.entry, max_k=10) as srv:
            ids, d = srv.wait(srv.submit(q[:20], 10, 48, entries=ents))
        bi, bd, _, _ = cng.search(xd, g.adj, dev(q[:20]), 10, 48,
                                  torch.from_numpy(ents.view(np.int32)).to("cuda:0"))
        assert np.array_equal(ids, host_ids(bi)) and np.array_equal(d, bd.cpu().numpy())


def test_rejects_bad_requests(index):
    x, q, xd, g = index
    with cng.Server(xd, g.adj, g.entry, max_k=10) as srv:
        with pytest.raises(cng.CngError):
            srv.submit(q[:2], 11, 32)       # k > max_k
        with pytest.raises(cng.CngError):
            srv.submit(q[:2], 10, 300)      # beam > 256
        ids, _ = srv.wait(srv.submit(q[:2], 10, 32))
        assert ids.shape == (2, 10)
