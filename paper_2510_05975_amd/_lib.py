"""ctypes binding of libcng.so (the gfx950 alpha-CNG library).

Argument marshalling only: torch tensors supply device memory and the current
HIP stream; every step runs in the library's kernels.  uint32 ids travel in
torch.int32 tensors (same bits; CNG_NONE reads as -1).

The library must have been built (``paper_2510_05975_amd.build_lib.build()``);
importing works without it, but every call raises if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcng.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cng.h")

NONE = 0xFFFFFFFF
BUILD_CONNECT = 1
BUILD_BACKWARD = 2
BUILD_GRAPH_CANDIDATES = 4
STATUS = {0: "CNG_OK", -1: "CNG_EINVAL", -2: "CNG_ENOMEM", -3: "CNG_EDEVICE",
          -4: "CNG_EUNSUPPORTED", -5: "CNG_ECAPACITY"}


class CngError(RuntimeError):
    def __init__(self, func: str, status: int, msg: str):
        super().__init__(f"{func}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class BuildParams(C.Structure):
    _fields_ = [("R", C.c_int32), ("extra", C.c_int32), ("C", C.c_int32), ("alpha", C.c_double),
                ("tau", C.c_double), ("flags", C.c_uint32), ("Lc", C.c_int32), ("band", C.c_int32),
                ("visited_log2", C.c_int32), ("alpha_max", C.c_double), ("alpha_step", C.c_double),
                ("pass_rows", C.c_int32), ("knn_K", C.c_int32), ("knn_rounds", C.c_int32),
                ("cand_L", C.c_int32), ("knn_seed", C.c_uint64)]


class BuildStats(C.Structure):
    _fields_ = [("ms_entry", C.c_double), ("ms_candidates", C.c_double), ("ms_prune", C.c_double),
                ("ms_connect", C.c_double), ("ms_total", C.c_double),
                ("connect_rounds", C.c_int64), ("connect_added", C.c_int64),
                ("overflow_rows", C.c_int64), ("exact_integer", C.c_int32),
                ("filter_dtype", C.c_int32), ("ms_backward", C.c_double),
                ("ms_knn_graph", C.c_double), ("knn_rounds_run", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
vp, i64, i32, u32, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32, C.c_size_t

_SIGS = {
    "cng_last_error": (C.c_char_p, []),
    "cng_version": (C.c_char_p, []),
    "cng_build_workspace_size": (C.c_int, [i64, i32, C.POINTER(BuildParams), C.POINTER(sz)]),
    "cng_build": (C.c_int, [vp, i64, i32, C.POINTER(BuildParams), vp, vp, vp, sz, vp,
                            C.POINTER(BuildStats)]),
    "cng_entry_workspace_size": (sz, [i64, i32]),
    "cng_entry_point": (C.c_int, [vp, i64, i32, vp, vp, sz, vp]),
    "cng_knn_workspace_size": (C.c_int, [i64, i64, i32, i32, i32, i64, C.POINTER(sz)]),
    "cng_knn": (C.c_int, [vp, i64, vp, i64, i32, i32, i32, i32, i64, vp, vp, vp, sz, vp,
                          C.POINTER(i64)]),
    "cng_nndescent_workspace_size": (C.c_int, [i64, i32, C.POINTER(sz)]),
    "cng_nndescent": (C.c_int, [vp, i64, i32, i32, C.c_uint64, i32, vp, vp, vp, sz, vp,
                                C.POINTER(i32)]),
    "cng_graph_candidates_workspace_size": (C.c_int, [i64, i32, C.POINTER(sz)]),
    "cng_graph_candidates": (C.c_int, [vp, i64, i32, vp, vp, i32, u32, i32, i32, vp, vp, vp, sz,
                                       vp]),
    "cng_prune": (C.c_int, [vp, i64, i32, vp, vp, i32, i32, i32, C.c_double, C.c_double, vp, vp]),
    "cng_prune_adaptive": (C.c_int, [vp, i64, i32, vp, vp, i32, i32, i32, C.c_double, C.c_double,
                                     C.c_double, C.c_double, vp, vp]),
    "cng_backward_workspace_size": (C.c_int, [i64, i32, i32, C.POINTER(sz)]),
    "cng_backward": (C.c_int, [vp, i64, i32, vp, i32, i32, i32, C.c_double, C.c_double,
                               C.c_double, C.c_double, vp, sz,
                               vp]),
    "cng_connect_workspace_size": (C.c_int, [i64, i32, i32, C.POINTER(sz)]),
    "cng_connect": (C.c_int, [vp, i64, i32, vp, i32, u32, i32, i32, vp, sz, vp, C.POINTER(i64),
                              C.POINTER(i64)]),
    "cng_search": (C.c_int, [vp, i64, i32, vp, i32, vp, i64, i32, i32, vp, i64, vp, vp, vp, vp,
                             i32, vp]),
    "cng_quantized_bytes": (sz, [i64, i32, i32]),
    "cng_quantize": (C.c_int, [vp, i64, i32, i32, vp, vp, vp]),
    "cng_search_quantized": (C.c_int, [vp, vp, i32, vp, i64, i32, vp, i32, vp, i64, i32, i32, vp,
                                       i64, vp, vp, vp, vp, i32, vp]),
    "cng_kmeans_workspace_size": (sz, [i64, i32, i32]),
    "cng_kmeans": (C.c_int, [vp, i64, i32, i32, i32, vp, vp, vp, vp, sz, vp]),
    "cng_entry_labels_workspace_size": (C.c_int, [i64, i32, i64, i32, C.POINTER(sz)]),
    "cng_entry_labels": (C.c_int, [vp, i64, i32, vp, i32, u32, vp, i64, i32, vp, i32, vp, vp, sz,
                                   vp]),
    "cng_mlp_param_count": (i64, [i32, i32, i32]),
    "cng_mlp_workspace_size": (sz, [i32, i32, i32, i32]),
    "cng_mlp_input_stats_workspace_size": (sz, [i64, i32]),
    "cng_mlp_input_stats": (C.c_int, [vp, i64, i32, vp, vp, vp, sz, vp]),
    "cng_mlp_gradients": (C.c_int, [vp, i32, i32, i32, vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, sz,
                                    vp]),
    "cng_mlp_adam": (C.c_int, [vp, vp, vp, vp, i32, i32, i32, i32, C.c_float, C.c_float, C.c_float,
                               C.c_float, vp]),
    "cng_mlp_logits": (C.c_int, [vp, i32, i32, i32, vp, vp, vp, i32, i32, vp, vp, vp, sz, vp]),
    "cng_entry_predict": (C.c_int, [vp, i32, i32, i32, vp, vp, vp, i32, i32, vp, u32, C.c_float, vp,
                                    vp, vp, sz, vp]),
    "cng_entry_predict_noalloc_max_bytes": (sz, []),
    "cng_entry_predict_noalloc": (C.c_int, [vp, i32, i32, i32, vp, vp, vp, i32, i32, vp, u32,
                                            C.c_float, vp, vp, vp]),
    "cng_nearest_centre_workspace_size": (sz, [i64, i32, i32]),
    "cng_nearest_centre_entry": (C.c_int, [vp, i64, i32, vp, i32, vp, vp, vp, sz, vp]),
    "cng_serve_workspace_size": (sz, []),
    "cng_serve_start": (C.c_int, [C.c_void_p, vp, sz, C.POINTER(C.c_void_p)]),
    "cng_serve_submit": (C.c_int, [vp, vp, i32, i32, i32, vp, C.POINTER(C.c_uint64)]),
    "cng_serve_poll": (C.c_int, [vp, C.c_uint64, vp, vp, C.POINTER(i32)]),
    "cng_serve_get_stats": (C.c_int, [vp, vp]),
    "cng_serve_stop": (C.c_int, [vp]),
}


def lib():
    """Load libcng.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2510_05975_amd.build_lib")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Function names declared in include/cng.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(cng_[a-z0-9_]+)\s*\(", txt)))


def _check(func: str, st: int):
    if st != 0:
        msg = lib().cng_last_error().decode()
        raise CngError(func, st, msg)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _f32(x: torch.Tensor) -> torch.Tensor:
    if x.dtype != torch.float32 or x.dim() != 2:
        raise ValueError("expected a 2-D float32 tensor")
    return x.contiguous()


def _ids(x: torch.Tensor) -> torch.Tensor:
    if x.dtype not in (torch.int32, torch.uint32):
        raise ValueError("expected int32 ids")
    return x.contiguous()


def version() -> str:
    return lib().cng_version().decode()


@dataclass
class Graph:
    adj: torch.Tensor      # [n, W] int32 (uint32 bits)
    entry: int
    R: int
    stats: dict


def build(points: torch.Tensor, R: int, C_: int, alpha: float, tau: float = 0.0, extra: int = 1,
          connect: bool = True, Lc: int = 0, band: int = 0, visited_log2: int = 0,
          backward: bool = False, alpha_max: float | None = None,
          alpha_step: float = 0.0, pass_rows: int = 0, graph_candidates: bool = False,
          knn_K: int = 0, knn_rounds: int = 0, cand_L: int = 0, knn_seed: int = 0) -> Graph:
    """cng_build: entry point, candidates (exact, or with graph_candidates from
    an NN-descent graph and a beam search on it), pruning (adaptive alpha when
    alpha_step > 0), optional backward edges, connectivity."""
    x = _f32(points)
    n, d = x.shape
    flags = ((BUILD_CONNECT if connect else 0) | (BUILD_BACKWARD if backward else 0) |
             (BUILD_GRAPH_CANDIDATES if graph_candidates else 0))
    amax = alpha if alpha_max is None else alpha_max
    p = BuildParams(R, extra, C_, alpha, tau, flags, Lc, band, visited_log2, amax, alpha_step,
                    pass_rows, knn_K, knn_rounds, cand_L, knn_seed)
    nb = sz(0)
    _check("cng_build_workspace_size", lib().cng_build_workspace_size(n, d, C.byref(p), C.byref(nb)))
    ws = _ws(nb.value, x.device)
    adj = torch.empty((n, R + extra), dtype=torch.int32, device=x.device)
    entry = torch.empty(1, dtype=torch.int32, device=x.device)
    st = BuildStats()
    _check("cng_build", lib().cng_build(_ptr(x), n, d, C.byref(p), _ptr(adj), _ptr(entry), _ptr(ws),
                                        nb.value, _stream(), C.byref(st)))
    return Graph(adj, int(entry.item()) & 0xFFFFFFFF, R, st.as_dict())


def entry_point(points: torch.Tensor) -> int:
    x = _f32(points)
    n, d = x.shape
    nb = lib().cng_entry_workspace_size(n, d)
    ws = _ws(nb, x.device)
    out = torch.empty(1, dtype=torch.int32, device=x.device)
    _check("cng_entry_point", lib().cng_entry_point(_ptr(x), n, d, _ptr(out), _ptr(ws), nb, _stream()))
    return int(out.item()) & 0xFFFFFFFF


def knn(rows: torch.Tensor, cols: torch.Tensor, C_: int, exclude_self: bool = False, band: int = 0,
        pass_rows: int = 0):
    """cng_knn -> (ids int32 [nr, C], D float32 [nr, C], overflow_rows)."""
    r, c = _f32(rows), _f32(cols)
    nr, d = r.shape
    nc = c.shape[0]
    nb = sz(0)
    _check("cng_knn_workspace_size", lib().cng_knn_workspace_size(nr, nc, d, C_, band, pass_rows,
                                                                  C.byref(nb)))
    ws = _ws(nb.value, r.device)
    ids = torch.empty((nr, C_), dtype=torch.int32, device=r.device)
    D = torch.empty((nr, C_), dtype=torch.float32, device=r.device)
    ovf = i64(0)
    same = exclude_self and rows.data_ptr() == cols.data_ptr()
    rp = _ptr(r)
    cp = rp if same else _ptr(c)
    _check("cng_knn", lib().cng_knn(rp, nr, cp, nc, d, C_, int(exclude_self), band, pass_rows, _ptr(ids),
                                    _ptr(D), _ptr(ws), nb.value, _stream(), C.byref(ovf)))
    return ids, D, ovf.value


def nndescent(points: torch.Tensor, K: int, seed: int, rounds: int):
    """cng_nndescent -> (ids int32 [n, K], D float32 [n, K], rounds run)."""
    x = _f32(points)
    n, d = x.shape
    nb = sz(0)
    _check("cng_nndescent_workspace_size", lib().cng_nndescent_workspace_size(n, K, C.byref(nb)))
    ws = _ws(nb.value, x.device)
    ids = torch.empty((n, K), dtype=torch.int32, device=x.device)
    D = torch.empty((n, K), dtype=torch.float32, device=x.device)
    rr = i32(0)
    _check("cng_nndescent", lib().cng_nndescent(_ptr(x), n, d, K, seed, rounds, _ptr(ids), _ptr(D),
                                                _ptr(ws), nb.value, _stream(), C.byref(rr)))
    return ids, D, rr.value


def graph_candidates(points: torch.Tensor, g0: torch.Tensor, g0D: torch.Tensor, entry: int, L: int,
                     C_: int):
    """cng_graph_candidates -> (ids int32 [n, C], D float32 [n, C])."""
    x = _f32(points)
    n, d = x.shape
    g0 = _ids(g0)
    nb = sz(0)
    _check("cng_graph_candidates_workspace_size",
           lib().cng_graph_candidates_workspace_size(n, C_, C.byref(nb)))
    ws = _ws(nb.value, x.device)
    ids = torch.empty((n, C_), dtype=torch.int32, device=x.device)
    D = torch.empty((n, C_), dtype=torch.float32, device=x.device)
    _check("cng_graph_candidates", lib().cng_graph_candidates(
        _ptr(x), n, d, _ptr(g0), _ptr(g0D.contiguous()), g0.shape[1], entry, L, C_, _ptr(ids),
        _ptr(D), _ptr(ws), nb.value, _stream()))
    return ids, D


def prune(points: torch.Tensor, cand: torch.Tensor, candD: torch.Tensor, R: int, alpha: float,
          tau: float = 0.0, width: int | None = None, alpha_max: float | None = None,
          alpha_step: float = 0.0) -> torch.Tensor:
    """cng_prune (fixed alpha) or, with alpha_step > 0, cng_prune_adaptive."""
    x = _f32(points)
    n, d = x.shape
    cand, candD = _ids(cand), candD.contiguous()
    W = R if width is None else width
    adj = torch.empty((n, W), dtype=torch.int32, device=x.device)
    if alpha_step > 0:
        amax = alpha if alpha_max is None else alpha_max
        _check("cng_prune_adaptive", lib().cng_prune_adaptive(
            _ptr(x), n, d, _ptr(cand), _ptr(candD), cand.shape[1], R, W, alpha, amax, alpha_step,
            tau, _ptr(adj), _stream()))
    else:
        _check("cng_prune", lib().cng_prune(_ptr(x), n, d, _ptr(cand), _ptr(candD), cand.shape[1],
                                            R, W, alpha, tau, _ptr(adj), _stream()))
    return adj


def backward(points: torch.Tensor, adj: torch.Tensor, R: int, Cb: int, alpha: float,
             tau: float = 0.0, alpha_max: float | None = None, alpha_step: float = 0.0) -> None:
    """cng_backward in place on adj (backward edges with lazy pruning)."""
    x = _f32(points)
    n, d = x.shape
    adj = _ids(adj)
    W = adj.shape[1]
    nb = sz(0)
    _check("cng_backward_workspace_size", lib().cng_backward_workspace_size(n, W, Cb, C.byref(nb)))
    ws = _ws(nb.value, x.device)
    amax = alpha if alpha_max is None else alpha_max
    _check("cng_backward", lib().cng_backward(_ptr(x), n, d, _ptr(adj), W, R, Cb, alpha, amax,
                                              alpha_step, tau, _ptr(ws), nb.value, _stream()))


def connect(points: torch.Tensor, adj: torch.Tensor, entry: int, Lc: int, visited_log2: int = 0):
    """cng_connect in place on adj -> (rounds, added)."""
    x = _f32(points)
    n, d = x.shape
    adj = _ids(adj)
    W = adj.shape[1]
    nb = sz(0)
    _check("cng_connect_workspace_size", lib().cng_connect_workspace_size(n, W, Lc, C.byref(nb)))
    ws = _ws(nb.value, x.device)
    rounds, added = i64(0), i64(0)
    _check("cng_connect", lib().cng_connect(_ptr(x), n, d, _ptr(adj), W, entry, Lc, visited_log2,
                                            _ptr(ws), nb.value, _stream(), C.byref(rounds),
                                            C.byref(added)))
    return rounds.value, added.value


def search(points: torch.Tensor, adj: torch.Tensor, queries: torch.Tensor, k: int, L: int,
           entries, visited_log2: int = 0, stats: bool = False, out=None):
    """cng_search -> (ids int32 [nq, k], dists float32 [nq, k], hops, ndc)."""
    x, q = _f32(points), _f32(queries)
    n, d = x.shape
    nq = q.shape[0]
    adj = _ids(adj)
    if isinstance(entries, int):
        entries = torch.tensor([entries & 0xFFFFFFFF], dtype=torch.int64).to(torch.int32).to(x.device)
    entries = _ids(entries)
    if out is None:
        ids = torch.empty((nq, k), dtype=torch.int32, device=x.device)
        dists = torch.empty((nq, k), dtype=torch.float32, device=x.device)
        hops = torch.empty(nq, dtype=torch.int32, device=x.device) if stats else None
        ndc = torch.empty(nq, dtype=torch.int32, device=x.device) if stats else None
    else:
        ids, dists, hops, ndc = out
    _check("cng_search", lib().cng_search(_ptr(x), n, d, _ptr(adj), adj.shape[1], _ptr(q), nq, k, L,
                                          _ptr(entries), entries.numel(), _ptr(ids), _ptr(dists),
                                          _ptr(hops), _ptr(ndc), visited_log2, _stream()))
    return ids, dists, hops, ndc


F32, BF16, FP8 = 0, 1, 2


@dataclass
class Store:
    """Reduced-precision copy of the base vectors (cng_quantize)."""
    dtype: int
    vecs: torch.Tensor          # uint16 bf16 bits / uint8 fp8 codes, [n, d]
    scales: torch.Tensor | None  # fp8 only, [n, 2] float32: scale s and n2 = s^2 |c|^2


def quantize(points: torch.Tensor, dtype: int) -> Store:
    x = _f32(points)
    n, d = x.shape
    if dtype == BF16:
        vecs = torch.empty((n, d), dtype=torch.uint16, device=x.device)
        scales = None
    elif dtype == FP8:
        vecs = torch.empty((n, d), dtype=torch.uint8, device=x.device)
        scales = torch.empty((n, 2), dtype=torch.float32, device=x.device)
    else:
        raise ValueError("dtype must be BF16 or FP8")
    _check("cng_quantize", lib().cng_quantize(_ptr(x), n, d, dtype, _ptr(vecs), _ptr(scales),
                                              _stream()))
    return Store(dtype, vecs, scales)


def search_quantized(points: torch.Tensor, store: Store, adj: torch.Tensor, queries: torch.Tensor,
                     k: int, L: int, entries, visited_log2: int = 0, stats: bool = False):
    """cng_search_quantized -> (ids, float32-exact dists, hops, ndc)."""
    x, q = _f32(points), _f32(queries)
    n, d = x.shape
    nq = q.shape[0]
    adj = _ids(adj)
    if isinstance(entries, int):
        entries = torch.tensor([entries & 0xFFFFFFFF], dtype=torch.int64).to(torch.int32).to(x.device)
    entries = _ids(entries)
    ids = torch.empty((nq, k), dtype=torch.int32, device=x.device)
    dists = torch.empty((nq, k), dtype=torch.float32, device=x.device)
    hops = torch.empty(nq, dtype=torch.int32, device=x.device) if stats else None
    ndc = torch.empty(nq, dtype=torch.int32, device=x.device) if stats else None
    _check("cng_search_quantized", lib().cng_search_quantized(
        _ptr(x), _ptr(store.vecs), store.dtype, _ptr(store.scales), n, d, _ptr(adj), adj.shape[1],
        _ptr(q), nq, k, L, _ptr(entries), entries.numel(), _ptr(ids), _ptr(dists), _ptr(hops),
        _ptr(ndc), visited_log2, _stream()))
    return ids, dists, hops, ndc


# ---------------------------------------------------------------- learned entry point
def kmeans(points: torch.Tensor, K: int, iters: int, init_ids: torch.Tensor):
    """cng_kmeans -> (centers [K, d] float32, entries [K] int32)."""
    x = _f32(points)
    n, d = x.shape
    nb = lib().cng_kmeans_workspace_size(n, d, K)
    ws = _ws(nb, x.device)
    centers = torch.empty((K, d), dtype=torch.float32, device=x.device)
    entries = torch.empty(K, dtype=torch.int32, device=x.device)
    _check("cng_kmeans", lib().cng_kmeans(_ptr(x), n, d, K, iters, _ptr(_ids(init_ids)),
                                          _ptr(centers), _ptr(entries), _ptr(ws), nb, _stream()))
    return centers, entries


def entry_labels(points, adj, nav: int, queries, L: int, entries):
    x, q = _f32(points), _f32(queries)
    n, d = x.shape
    nq = q.shape[0]
    K = entries.numel()
    nb = sz(0)
    _check("cng_entry_labels_workspace_size",
           lib().cng_entry_labels_workspace_size(n, d, nq, K, C.byref(nb)))
    ws = _ws(nb.value, x.device)
    labels = torch.empty(nq, dtype=torch.int32, device=x.device)
    adj = _ids(adj)
    _check("cng_entry_labels", lib().cng_entry_labels(_ptr(x), n, d, _ptr(adj), adj.shape[1], nav,
                                                      _ptr(q), nq, L, _ptr(_ids(entries)), K,
                                                      _ptr(labels), _ptr(ws), nb.value, _stream()))
    return labels


def mlp_param_count(d: int, H: int, K: int) -> int:
    return int(lib().cng_mlp_param_count(d, H, K))


def mlp_input_stats(X):
    """cng_mlp_input_stats -> (x_mean [d], x_scale [1]) device float32."""
    X = _f32(X)
    n, d = X.shape
    nb = lib().cng_mlp_input_stats_workspace_size(n, d)
    ws = _ws(nb, X.device)
    mean = torch.empty(d, dtype=torch.float32, device=X.device)
    scale = torch.empty(1, dtype=torch.float32, device=X.device)
    _check("cng_mlp_input_stats", lib().cng_mlp_input_stats(_ptr(X), n, d, _ptr(mean), _ptr(scale),
                                                            _ptr(ws), nb, _stream()))
    return mean, scale


def mlp_gradients(params, d, H, K, X, labels, batch_ids, B, precision, grads, loss=None, ws=None,
                  affine=None):
    """affine: (x_mean, x_scale) device tensors, or None for raw inputs."""
    X = _f32(X)
    xm, xs = affine if affine is not None else (None, None)
    nb = lib().cng_mlp_workspace_size(d, H, K, B)
    if ws is None or ws.numel() < nb:
        ws = _ws(nb, X.device)
    _check("cng_mlp_gradients", lib().cng_mlp_gradients(
        _ptr(params), d, H, K, _ptr(X), _ptr(xm), _ptr(xs), _ptr(_ids(labels)),
        _ptr(batch_ids) if batch_ids is not None else None, B, precision, _ptr(grads),
        _ptr(loss), _ptr(ws), ws.numel(), _stream()))
    return ws


def mlp_adam(params, grads, m1, m2, d, H, K, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check("cng_mlp_adam", lib().cng_mlp_adam(_ptr(params), _ptr(grads), _ptr(m1), _ptr(m2), d, H,
                                              K, step, lr, beta1, beta2, eps, _stream()))


def mlp_logits(params, d, H, K, X, precision, affine=None, hidden=False):
    """cng_mlp_logits -> Z [B, K] (and the hidden activations [2, B, H] with
    ``hidden``)."""
    X = _f32(X)
    xm, xs = affine if affine is not None else (None, None)
    B = X.shape[0]
    nb = lib().cng_mlp_workspace_size(d, H, K, B)
    ws = _ws(nb, X.device)
    Z = torch.empty((B, K), dtype=torch.float32, device=X.device)
    Hd = torch.empty((2, B, H), dtype=torch.float32, device=X.device) if hidden else None
    _check("cng_mlp_logits", lib().cng_mlp_logits(_ptr(params), d, H, K, _ptr(X), _ptr(xm), _ptr(xs),
                                                  B, precision, _ptr(Z), _ptr(Hd), _ptr(ws), nb,
                                                  _stream()))
    return (Z, Hd) if hidden else Z


def entry_predict(params, d, H, K, X, precision, entries, fallback: int, theta: float,
                  affine=None):
    X = _f32(X)
    xm, xs = affine if affine is not None else (None, None)
    B = X.shape[0]
    nb = lib().cng_mlp_workspace_size(d, H, K, B)
    ws = _ws(nb, X.device)
    out = torch.empty(B, dtype=torch.int32, device=X.device)
    conf = torch.empty(B, dtype=torch.float32, device=X.device)
    _check("cng_entry_predict", lib().cng_entry_predict(_ptr(params), d, H, K, _ptr(X), _ptr(xm),
                                                        _ptr(xs), B, precision,
                                                        _ptr(_ids(entries)), fallback, theta,
                                                        _ptr(out), _ptr(conf), _ptr(ws), nb,
                                                        _stream()))
    return out, conf


def entry_predict_noalloc(params, d, H, K, X, precision, entries, fallback: int, theta: float,
                          affine=None, out=None):
    """cng_entry_predict_noalloc (the library's fixed scratch array, no
    workspace): out = (entries int32 [B], conf float32 [B]) or new tensors."""
    X = _f32(X)
    xm, xs = affine if affine is not None else (None, None)
    B = X.shape[0]
    if out is None:
        out = (torch.empty(B, dtype=torch.int32, device=X.device),
               torch.empty(B, dtype=torch.float32, device=X.device))
    _check("cng_entry_predict_noalloc", lib().cng_entry_predict_noalloc(
        _ptr(params), d, H, K, _ptr(X), _ptr(xm), _ptr(xs), B, precision, _ptr(_ids(entries)),
        fallback, theta, _ptr(out[0]), _ptr(out[1]), _stream()))
    return out


def nearest_centre_entry(queries, centers, entries):
    q, c = _f32(queries), _f32(centers)
    nq, d = q.shape
    K = c.shape[0]
    nb = lib().cng_nearest_centre_workspace_size(nq, d, K)
    ws = _ws(nb, q.device)
    out = torch.empty(nq, dtype=torch.int32, device=q.device)
    _check("cng_nearest_centre_entry", lib().cng_nearest_centre_entry(
        _ptr(q), nq, d, _ptr(c), K, _ptr(_ids(entries)), _ptr(out), _ptr(ws), nb, _stream()))
    return out


# ---------------------------------------------------------------- serving
class ServeConfig(C.Structure):
    _fields_ = [("points", C.c_void_p), ("vecs", C.c_void_p), ("dtype", C.c_int32),
                ("scales", C.c_void_p), ("n", C.c_int64), ("d", C.c_int32), ("adj", C.c_void_p),
                ("W", C.c_int32), ("entry", C.c_uint32), ("waves", C.c_int32),
                ("capacity", C.c_int32), ("max_k", C.c_int32), ("visited_log2", C.c_int32),
                ("arena_bytes", C.c_int64), ("idle_checks", C.c_int32)]


class ServeStats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("submitted", C.c_int64), ("completed", C.c_int64),
                ("refused", C.c_int64), ("in_flight", C.c_int64), ("arena_bytes", C.c_int64),
                ("arena_used", C.c_int64), ("running", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Server:
    """Continuous-batching search server (cng_serve_*): a persistent device
    grid fed through pinned host rings.  Host arrays in, host arrays out."""

    def __init__(self, points: torch.Tensor, adj: torch.Tensor, entry: int, store: "Store | None" = None,
                 max_k: int = 100, waves: int = 0, capacity: int = 0, visited_log2: int = 0,
                 arena_bytes: int = 0, idle_checks: int = 0):
        import numpy as np  # noqa: F401
        x = _f32(points)
        self._keep = [x, _ids(adj), store]
        self.d = x.shape[1]
        cfg = ServeConfig(x.data_ptr(), (store.vecs if store else x).data_ptr(),
                          store.dtype if store else F32,
                          store.scales.data_ptr() if (store and store.scales is not None) else None,
                          x.shape[0], self.d, _ids(adj).data_ptr(), adj.shape[1], entry, waves,
                          capacity, max_k, visited_log2, arena_bytes, idle_checks)
        self._ws = _ws(lib().cng_serve_workspace_size(), x.device)
        torch.cuda.synchronize()
        h = C.c_void_p(0)
        _check("cng_serve_start", lib().cng_serve_start(C.byref(cfg), _ptr(self._ws),
                                                        self._ws.numel(), C.byref(h)))
        self._h = h
        self.pending = {}

    def submit(self, queries, k: int, L: int, entries=None):
        """Returns a request id, or None when the request is not admitted now."""
        import numpy as np
        q = np.ascontiguousarray(queries, dtype=np.float32)
        ent = None if entries is None else np.ascontiguousarray(entries, dtype=np.uint32)
        rid = C.c_uint64(0)
        st = lib().cng_serve_submit(self._h, q.ctypes.data, q.shape[0], k, L,
                                    None if ent is None else ent.ctypes.data, C.byref(rid))
        if st == -5:
            return None
        _check("cng_serve_submit", st)
        self.pending[rid.value] = (q.shape[0], k)
        return rid.value

    def poll(self, req: int):
        """(ids uint32 [nq, k], dists float32 [nq, k]) once complete, else None."""
        import numpy as np
        nq, k = self.pending[req]
        ids = np.empty((nq, k), np.uint32)
        dists = np.empty((nq, k), np.float32)
        done = C.c_int32(0)
        _check("cng_serve_poll", lib().cng_serve_poll(self._h, req, ids.ctypes.data,
                                                      dists.ctypes.data, C.byref(done)))
        if not done.value:
            return None
        del self.pending[req]
        return ids, dists

    def stats(self) -> dict:
        st = ServeStats()
        _check("cng_serve_get_stats", lib().cng_serve_get_stats(self._h, C.byref(st)))
        return st.as_dict()

    def wait(self, req: int, timeout: float = 30.0):
        import time
        t0 = time.time()
        while True:
            r = self.poll(req)
            if r is not None:
                return r
            if time.time() - t0 > timeout:
                raise TimeoutError(f"request {req} not complete after {timeout}s")

    def stop(self):
        if self._h:
            _check("cng_serve_stop", lib().cng_serve_stop(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()


def u32(t: torch.Tensor):
    """Device int32 ids -> host numpy uint32."""
    return t.cpu().numpy().view("uint32")
