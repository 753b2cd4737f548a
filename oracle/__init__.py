"""CPU oracle for the alpha-CNG hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library never loads it and shares no
code with it.

``cng_oracle.c`` holds the plain C implementation (double precision mode and a
fixed-reduction-order single precision mode); this module builds it with gcc and
wraps it with ctypes.  Every array argument is a host numpy array.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cng_oracle.c")
LIB = os.environ.get("CNG_ORACLE_LIB") or os.path.join(HERE, "libcng_oracle.so")

NONE = 0xFFFFFFFF
FP64 = 0
FP32 = 1

_CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-fPIC",
           "-shared", "-Wall", "-Wextra"]


def build_lib(src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle (always recompiles)."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", *_CFLAGS, "-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_lib()
        L = C.CDLL(LIB)
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        i64 = C.c_int64
        L.orc_dist_f32.restype = C.c_float
        L.orc_dist_f32.argtypes = [f32p, f32p, C.c_int]
        L.orc_dist_f64.restype = C.c_double
        L.orc_dist_f64.argtypes = [f32p, f32p, C.c_int]
        L.orc_knn.argtypes = [f32p, i64, f32p, i64, C.c_int, C.c_int, C.c_int, C.c_int, u32p, f64p]
        L.orc_prune.argtypes = [f32p, i64, C.c_int, u32p, f64p, C.c_int, C.c_int, C.c_int,
                                C.c_double, C.c_double, C.c_int, u32p]
        L.orc_prune_adaptive.argtypes = [f32p, i64, C.c_int, u32p, f64p, C.c_int, C.c_int,
                                         C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                         C.c_int, u32p]
        L.orc_medoid.restype = C.c_uint32
        L.orc_medoid.argtypes = [f32p, i64, C.c_int]
        L.orc_search.argtypes = [f32p, i64, C.c_int, u32p, C.c_int, f32p, i64, C.c_int, C.c_int,
                                 u32p, i64, C.c_int, u32p, f64p, C.c_void_p, C.c_void_p]
        L.orc_search_trace.argtypes = [f32p, i64, C.c_int, u32p, C.c_int, f32p, C.c_int, C.c_int,
                                       C.c_uint32, C.c_int, u32p, f64p, u32p, C.c_int,
                                       C.POINTER(C.c_int)]
        L.orc_connect.argtypes = [f32p, i64, C.c_int, u32p, C.c_int, C.c_uint32, C.c_int, C.c_int,
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.orc_build.argtypes = [f32p, i64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                C.c_int, u32p, C.POINTER(C.c_uint32), C.POINTER(C.c_int64)]
        L.orc_backward.argtypes = [f32p, i64, C.c_int, u32p, C.c_int, C.c_int, C.c_int,
                                   C.c_double, C.c_double, C.c_double, C.c_double, C.c_int]
        L.orc_round_bf16.restype = C.c_float
        L.orc_round_bf16.argtypes = [C.c_float]
        L.orc_round_e4m3.restype = C.c_float
        L.orc_round_e4m3.argtypes = [C.c_float]
        L.orc_dequantized.argtypes = [f32p, i64, C.c_int, C.c_int, f32p, C.c_void_p]
        L.orc_search_rerank.argtypes = [f32p, C.c_void_p, i64, C.c_int, u32p, C.c_int, f32p, i64,
                                        C.c_int, C.c_int, u32p, i64, C.c_int, u32p, f64p,
                                        C.c_void_p, C.c_void_p]
        L.orc_dot_f32.restype = C.c_float
        L.orc_dot_f32.argtypes = [f32p, f32p, C.c_int]
        L.orc_fp8_encode.argtypes = [f32p, i64, C.c_int, f32p, f32p, f32p]
        L.orc_fp8_score.restype = C.c_float
        L.orc_fp8_score.argtypes = [f32p, f32p, C.c_float, C.c_float, C.c_int]
        L.orc_search_fp8.argtypes = [f32p, f32p, f32p, C.c_void_p, i64, C.c_int, u32p, C.c_int, f32p,
                                     i64, C.c_int, C.c_int, u32p, i64, u32p, f64p, C.c_void_p,
                                     C.c_void_p]
        L.orc_splitmix.restype = C.c_uint64
        L.orc_splitmix.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_nndescent.argtypes = [f32p, i64, C.c_int, C.c_int, C.c_uint64, C.c_int, C.c_int, u32p,
                                    f64p, C.POINTER(C.c_int)]
        L.orc_graph_candidates.argtypes = [f32p, i64, C.c_int, u32p, C.c_int, C.c_uint32, C.c_int,
                                           C.c_int, C.c_int, u32p, f64p]
        L.orc_build_ex.argtypes = [f32p, i64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                   C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_int, C.c_uint64, C.c_int, C.c_int, u32p,
                                   C.POINTER(C.c_uint32), C.POINTER(C.c_int64)]
        L.orc_max_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def dist_f32(x, y) -> np.float32:
    """Fixed-order single precision squared distance."""
    x, y = _f32(x), _f32(y)
    return np.float32(lib().orc_dist_f32(x, y, x.size))


def dist_f64(x, y) -> float:
    """The same reduction order in double precision."""
    x, y = _f32(x), _f32(y)
    return float(lib().orc_dist_f64(x, y, x.size))


def dot_f32(x, y) -> np.float32:
    """Fixed-order single precision dot product (the lanes and butterfly of
    dist_f32)."""
    x, y = _f32(x), _f32(y)
    return np.float32(lib().orc_dot_f32(x, y, x.size))


def knn(rows, cols, C: int, exclude_self: bool = False, mode: int = FP32):
    """C nearest columns of every row by (D, id) -> (ids uint32, D float64)."""
    rows, cols = _f32(rows), _f32(cols)
    nr, d = rows.shape
    ids = np.empty((nr, C), np.uint32)
    D = np.empty((nr, C), np.float64)
    _check(lib().orc_knn(rows, nr, cols, cols.shape[0], d, C, int(exclude_self), mode, ids, D), "knn")
    return ids, D


def prune(points, cand, candD, R: int, alpha: float, tau: float = 0.0, mode: int = FP32,
          width: int | None = None, alpha_max: float | None = None, alpha_step: float = 0.0):
    """Alg. 2 on every candidate row, at most R kept -> adjacency (n x width,
    NONE padded).  alpha_step > 0: Alg. 4 (adaptive alpha from ``alpha`` up to
    ``alpha_max``)."""
    points = _f32(points)
    n, d = points.shape
    W = R if width is None else width
    cand = np.ascontiguousarray(cand, np.uint32)
    candD = np.ascontiguousarray(candD, np.float64)
    adj = np.empty((n, W), np.uint32)
    amax = alpha if alpha_max is None else alpha_max
    _check(lib().orc_prune_adaptive(points, n, d, cand, candD, cand.shape[1], R, W, alpha, amax,
                                    alpha_step, tau, mode, adj), "prune")
    return adj


def medoid(points) -> int:
    points = _f32(points)
    return int(lib().orc_medoid(points, points.shape[0], points.shape[1]))


def search(points, adj, queries, k: int, L: int, entries, mode: int = FP32):
    """Alg. 1 for every query -> (ids, dists, hops, ndc)."""
    points, queries = _f32(points), _f32(queries)
    n, d = points.shape
    adj = np.ascontiguousarray(adj, np.uint32)
    entries = np.ascontiguousarray(np.atleast_1d(entries), np.uint32)
    nq = queries.shape[0]
    ids = np.empty((nq, k), np.uint32)
    dists = np.empty((nq, k), np.float64)
    hops = np.empty(nq, np.uint32)
    ndc = np.empty(nq, np.uint32)
    _check(lib().orc_search(points, n, d, adj, adj.shape[1], queries, nq, k, L, entries,
                            entries.size, mode, ids, dists, hops.ctypes.data, ndc.ctypes.data),
           "search")
    return ids, dists, hops, ndc


def search_trace(points, adj, q, k: int, L: int, entry: int, mode: int = FP32, cap: int = 1 << 16):
    """One query, also returning the sequence of hop vertices."""
    points = _f32(points)
    n, d = points.shape
    adj = np.ascontiguousarray(adj, np.uint32)
    ids = np.empty(k, np.uint32)
    dists = np.empty(k, np.float64)
    trace = np.empty(cap, np.uint32)
    tl = C.c_int(0)
    _check(lib().orc_search_trace(points, n, d, adj, adj.shape[1], _f32(q), k, L, entry, mode,
                                  ids, dists, trace, cap, C.byref(tl)), "search_trace")
    return ids, dists, trace[: min(tl.value, cap)].copy()


def connect(points, adj, entry: int, Lc: int, mode: int = FP32):
    """Connectivity repair in place on a copy -> (adj, n_added, n_rounds)."""
    points = _f32(points)
    n, d = points.shape
    adj = np.array(adj, np.uint32, copy=True, order="C")
    added, rounds = C.c_int64(0), C.c_int64(0)
    _check(lib().orc_connect(points, n, d, adj, adj.shape[1], entry, Lc, mode, C.byref(added),
                             C.byref(rounds)), "connect")
    return adj, added.value, rounds.value


def backward(points, adj, R: int, Cb: int, alpha: float, tau: float = 0.0, mode: int = FP32,
             alpha_max: float | None = None, alpha_step: float = 0.0):
    """Alg. 3 phase 3 (backward edges, lazy pruning) on a copy of ``adj``."""
    points = _f32(points)
    n, d = points.shape
    adj = np.array(adj, np.uint32, copy=True, order="C")
    amax = alpha if alpha_max is None else alpha_max
    _check(lib().orc_backward(points, n, d, adj, R, adj.shape[1], Cb, alpha, amax, alpha_step,
                              tau, mode), "backward")
    return adj


def build(points, R: int, C_: int, alpha: float, tau: float = 0.0, mode: int = FP32,
          connect: bool = True, Lc: int = 0, extra: int = 1, backward: bool = False,
          alpha_max: float | None = None, alpha_step: float = 0.0, knn_K: int = 0,
          knn_seed: int = 0, knn_rounds: int = 0, cand_L: int = 0):
    """Whole build -> (adj (n x (R + extra)), entry, n_added).  alpha_step > 0:
    adaptive alpha (Alg. 4) from ``alpha`` to ``alpha_max``.  knn_K > 0:
    candidates from an NN-descent graph (K, seed, rounds) searched with beam
    cand_L (Alg. 3 phases 1-2) instead of the exact C nearest."""
    points = _f32(points)
    n, d = points.shape
    adj = np.empty((n, R + extra), np.uint32)
    entry = C.c_uint32(0)
    added = C.c_int64(0)
    amax = alpha if alpha_max is None else alpha_max
    _check(lib().orc_build_ex(points, n, d, R, extra, C_, alpha, amax, alpha_step, tau, mode,
                              int(connect), int(backward), Lc, knn_K, knn_seed, knn_rounds, cand_L,
                              adj, C.byref(entry), C.byref(added)), "build")
    return adj, int(entry.value), added.value


def splitmix(seed: int, i: int) -> int:
    """Output i of the counter-based SplitMix64 stream with seed ``seed``."""
    return int(lib().orc_splitmix(seed & (2 ** 64 - 1), i))


def nndescent(points, K: int, seed: int, rounds: int, mode: int = FP32):
    """Alg. 3 phase 1: NN-descent K-NN graph -> (ids [n, K], D [n, K], rounds run)."""
    points = _f32(points)
    n, d = points.shape
    ids = np.empty((n, K), np.uint32)
    D = np.empty((n, K), np.float64)
    rr = C.c_int(0)
    _check(lib().orc_nndescent(points, n, d, K, seed & (2 ** 64 - 1), rounds, mode, ids, D,
                               C.byref(rr)), "nndescent")
    return ids, D, rr.value


def graph_candidates(points, g0, entry: int, L: int, C_: int, mode: int = FP32):
    """Alg. 3 phase 2: the C nearest of the points a beam search on g0 from
    ``entry`` evaluates for each point (itself excluded) -> (ids, D)."""
    points = _f32(points)
    n, d = points.shape
    g0 = np.ascontiguousarray(g0, np.uint32)
    ids = np.empty((n, C_), np.uint32)
    D = np.empty((n, C_), np.float64)
    _check(lib().orc_graph_candidates(points, n, d, g0, g0.shape[1], entry, L, C_, mode, ids, D),
           "graph_candidates")
    return ids, D


def reachable(adj, entry: int) -> np.ndarray:
    """Boolean mask of the points reachable from ``entry`` (numpy BFS)."""
    adj = np.asarray(adj)
    n = adj.shape[0]
    seen = np.zeros(n, bool)
    seen[entry] = True
    frontier = np.array([entry])
    ok = np.cumprod((adj != NONE) & (adj < n), axis=1).astype(bool)  # prefix before first sentinel
    while frontier.size:
        nb = adj[frontier][ok[frontier]]
        nb = np.unique(nb)
        nb = nb[~seen[nb]]
        seen[nb] = True
        frontier = nb
    return seen


BF16 = 1
FP8 = 2


def round_bf16(x: float) -> float:
    return float(lib().orc_round_bf16(float(x)))


def round_e4m3(x: float) -> float:
    return float(lib().orc_round_e4m3(float(x)))


def dequantized(points, dtype: int):
    """float32 values of the bf16 (dtype 1) or fp8-E4M3 + per-vector scale
    (dtype 2) copy of ``points`` -> (values [n, d], scales [n] or None)."""
    points = _f32(points)
    n, d = points.shape
    out = np.empty_like(points)
    scales = np.empty(n, np.float32) if dtype == FP8 else None
    _check(lib().orc_dequantized(points, n, d, dtype, out,
                                 scales.ctypes.data if scales is not None else None), "dequantized")
    return out, scales


def search_rerank(search_points, rerank_points, adj, queries, k: int, L: int, entries,
                  mode: int = FP32):
    """Beam search on ``search_points``; the final beam re-ranked with ``rerank_points``."""
    sp, qs = _f32(search_points), _f32(queries)
    rp = _f32(rerank_points) if rerank_points is not None else None
    n, d = sp.shape
    adj = np.ascontiguousarray(adj, np.uint32)
    entries = np.ascontiguousarray(np.atleast_1d(entries), np.uint32)
    nq = qs.shape[0]
    ids = np.empty((nq, k), np.uint32)
    dists = np.empty((nq, k), np.float64)
    hops = np.empty(nq, np.uint32)
    ndc = np.empty(nq, np.uint32)
    _check(lib().orc_search_rerank(sp, rp.ctypes.data if rp is not None else None, n, d, adj,
                                   adj.shape[1], qs, nq, k, L, entries, entries.size, mode, ids,
                                   dists, hops.ctypes.data, ndc.ctypes.data), "search_rerank")
    return ids, dists, hops, ndc


def fp8_encode(points):
    """fp8 form of the stored vectors -> (E4M3 values c [n, d] unscaled,
    scales s [n], n2 [n] = fl(fl(s s) dot(c, c)))."""
    points = _f32(points)
    n, d = points.shape
    c = np.empty_like(points)
    sc = np.empty(n, np.float32)
    n2 = np.empty(n, np.float32)
    _check(lib().orc_fp8_encode(points, n, d, c, sc, n2), "fp8_encode")
    return c, sc, n2


def fp8_score(encoded, q, v: int) -> np.float32:
    """fp8 dot-form score of stored vector v (from fp8_encode) against q."""
    c, sc, n2 = encoded
    q = _f32(q)
    return np.float32(lib().orc_fp8_score(q, _f32(c[v]), float(sc[v]), float(n2[v]), q.size))


def search_fp8(encoded, rerank_points, adj, queries, k: int, L: int, entries):
    """Beam search scored by the fp8 dot form of ``encoded`` (from
    fp8_encode); the final beam re-ranked with ``rerank_points`` (float32)."""
    c, sc, n2 = (_f32(a) for a in encoded)
    qs = _f32(queries)
    rp = _f32(rerank_points) if rerank_points is not None else None
    n, d = c.shape
    adj = np.ascontiguousarray(adj, np.uint32)
    entries = np.ascontiguousarray(np.atleast_1d(entries), np.uint32)
    nq = qs.shape[0]
    ids = np.empty((nq, k), np.uint32)
    dists = np.empty((nq, k), np.float64)
    hops = np.empty(nq, np.uint32)
    ndc = np.empty(nq, np.uint32)
    _check(lib().orc_search_fp8(c, sc, n2, rp.ctypes.data if rp is not None else None, n, d, adj,
                                adj.shape[1], qs, nq, k, L, entries, entries.size, ids, dists,
                                hops.ctypes.data, ndc.ctypes.data), "search_fp8")
    return ids, dists, hops, ndc
