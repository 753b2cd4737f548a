"""Serving loop (continuous batching on a persistent device grid): each
result is the same alone and in a mix of concurrent requests with different
k and L, and equals the batched search kernels; admission refuses requests
that do not fit and accepts them once slots free up."""
import numpy as np
import pytest
import torch

import paper_2510_05975_amd as cng
import workloads
from gpu_util import dev, host_ids

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
    for (tag, _, sel, k, L, *_), (ids, dists) in results:
        bi, bd = batched(xd, g, sel, k, L, store)
        assert np.array_equal(ids, bi) and np.array_equal(dists, bd), (tag, k, L)
        if tag == "probe":
            assert np.array_equal(ids, alone[0]) and np.array_equal(dists, alone[1])


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
