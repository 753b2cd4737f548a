"""Helpers shared by the GPU tests (host <-> device marshalling, and the
oracle counterpart of each stored-vector form)."""
import numpy as np
import torch

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def dev_ids(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(DEV)


def host_ids(t):
    return t.cpu().numpy().view(np.uint32)


def f32_of(d64):
    """Oracle float64 values that hold float32 results -> float32."""
    return np.asarray(d64).astype(np.float32)


def same_f32(a, b):
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    return a.shape == b.shape and np.array_equal(a.view(np.uint32), b.view(np.uint32))


def oracle_qsearch(dtype, x, adj, q, k, L, entries):
    """The oracle's search over the stored form `dtype` of x (1: bf16 values by
    the fixed-order distance, 2: fp8 by the dot form) with the float32 re-rank
    of the final beam."""
    import oracle
    if dtype == 2:
        return oracle.search_fp8(oracle.fp8_encode(x), x, adj, q, k, L, entries)
    deq, _ = oracle.dequantized(x, dtype)
    return oracle.search_rerank(deq, x, adj, q, k, L, entries)
