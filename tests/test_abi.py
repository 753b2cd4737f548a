"""Host-side checks of the C ABI: the library loads, exports every function the
header declares, and rejects invalid arguments before any device work."""
import ctypes as C

import pytest

import paper_2510_05975_amd as cng
from paper_2510_05975_amd import _lib


def test_exports_every_declared_symbol():
    L = cng.lib()
    names = _lib.header_symbols()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert cng.version().startswith("cng-gfx950")


def _params(**kw):
    p = dict(R=32, extra=1, C=128, alpha=1.2, tau=0.0, flags=1, Lc=0, band=0, visited_log2=0,
             alpha_max=1.2, alpha_step=0.0, pass_rows=0, knn_K=0, knn_rounds=0, cand_L=0,
             knn_seed=0)
    p.update(kw)
    return _lib.BuildParams(*[p[f] for f, _ in _lib.BuildParams._fields_])


@pytest.mark.parametrize("bad", [dict(R=0), dict(extra=-1), dict(C=0), dict(alpha=0.0),
                                 dict(alpha=float("nan")), dict(tau=-1.0), dict(Lc=-1),
                                 dict(visited_log2=3), dict(visited_log2=20),
                                 dict(alpha_step=-0.05), dict(alpha_step=0.05, alpha_max=1.0),
                                 dict(alpha_step=0.05, alpha_max=float("inf")), dict(pass_rows=-1)])
def test_build_params_rejected(bad):
    nb = C.c_size_t(0)
    st = cng.lib().cng_build_workspace_size(1000, 32, C.byref(_params(**bad)), C.byref(nb))
    assert st == -1
    assert cng.lib().cng_last_error().decode() != ""


@pytest.mark.parametrize("bad", [dict(R=200, extra=100), dict(band=8192), dict(C=900), dict(Lc=1000),
                                 dict(alpha_step=1e-6, alpha_max=2.0)])
def test_build_params_unsupported(bad):
    nb = C.c_size_t(0)
    st = cng.lib().cng_build_workspace_size(100000, 32, C.byref(_params(**bad)), C.byref(nb))
    assert st == -4


def test_build_sizes():
    nb = C.c_size_t(0)
    assert cng.lib().cng_build_workspace_size(1, 32, C.byref(_params()), C.byref(nb)) == -1  # n < 2
    assert cng.lib().cng_build_workspace_size(1000, 0, C.byref(_params()), C.byref(nb)) == -1
    assert cng.lib().cng_build_workspace_size(1000, 5000, C.byref(_params()), C.byref(nb)) == -1
    assert cng.lib().cng_build_workspace_size(10000, 32, C.byref(_params()), C.byref(nb)) == 0
    small = nb.value
    assert cng.lib().cng_build_workspace_size(20000, 32, C.byref(_params()), C.byref(nb)) == 0
    assert nb.value > small > 0
    assert cng.lib().cng_last_error().decode() == ""


def test_search_rejects_before_launch():
    L = cng.lib()
    fake = C.c_void_p(0x1000)
    # k = 0
    assert L.cng_search(fake, 100, 8, fake, 4, fake, 1, 0, 10, fake, 1, fake, fake, None, None, 0,
                        None) == -1
    # max(L, k) > 512
    assert L.cng_search(fake, 100, 8, fake, 4, fake, 1, 10, 600, fake, 1, fake, fake, None, None,
                        0, None) == -4
    # n_entries neither 1 nor nq
    assert L.cng_search(fake, 100, 8, fake, 4, fake, 5, 10, 10, fake, 3, fake, fake, None, None, 0,
                        None) == -1
    # W too large
    assert L.cng_search(fake, 100, 8, fake, 300, fake, 1, 10, 10, fake, 1, fake, fake, None, None,
                        0, None) == -4
    # NULL queries
    assert L.cng_search(fake, 100, 8, fake, 4, None, 1, 10, 10, fake, 1, fake, fake, None, None, 0,
                        None) == -1
    # nq = 0 is a no-op
    assert L.cng_search(fake, 100, 8, fake, 4, None, 0, 10, 10, fake, 1, fake, fake, None, None, 0,
                        None) == 0


def test_other_stages_reject():
    L = cng.lib()
    fake = C.c_void_p(0x1000)
    nb = C.c_size_t(0)
    assert L.cng_knn_workspace_size(10, 10, 8, 0, 0, 0, C.byref(nb)) == -1
    assert L.cng_knn_workspace_size(10, 10, 8, 900, 0, 0, C.byref(nb)) == -4
    assert L.cng_knn_workspace_size(10, 10, 8, 4, 0, -1, C.byref(nb)) == -1
    # smaller passes need less band memory
    big, small = C.c_size_t(0), C.c_size_t(0)
    assert L.cng_knn_workspace_size(100000, 100000, 32, 64, 0, 0, C.byref(big)) == 0
    assert L.cng_knn_workspace_size(100000, 100000, 32, 64, 0, 1000, C.byref(small)) == 0
    assert small.value < big.value
    # exclude_self with different row and column arrays
    assert L.cng_knn(fake, 10, C.c_void_p(0x2000), 10, 8, 4, 1, 0, 0, fake, fake, fake, 1 << 30,
                     None, None) == -1
    assert L.cng_prune(fake, 10, 8, fake, fake, 4, 5, 4, 1.2, 0.0, fake, None) == -1  # W < R
    assert L.cng_prune(fake, 10, 8, fake, fake, 4, 4, 4, -1.0, 0.0, fake, None) == -1
    assert L.cng_connect(fake, 10, 8, fake, 4, 10, 8, 0, fake, 1 << 30, None, None, None) == -1
    # workspace too small
    assert L.cng_entry_point(fake, 10, 8, fake, fake, 1, None) == -2


def test_serve_config_rejected_before_any_device_call():
    from paper_2510_05975_amd._lib import ServeConfig
    L = cng.lib()
    fake = 0x1000
    out = C.c_void_p(0)

    def start(**kw):
        f = dict(points=fake, vecs=fake, dtype=0, scales=None, n=100, d=8, adj=fake, W=4, entry=0,
                 waves=0, capacity=0, max_k=10, visited_log2=0, arena_bytes=0, idle_checks=0)
        f.update(kw)
        cfg = ServeConfig(*[f[k] for k, _ in ServeConfig._fields_])
        return L.cng_serve_start(C.byref(cfg), C.c_void_p(fake), 1 << 20, C.byref(out))

    assert start(visited_log2=14) == -1   # 6 .. 13 or 0
    assert start(visited_log2=5) == -1
    assert start(d=6) == -4               # d % 4
    assert start(max_k=300) == -4
    assert start(entry=100) == -1
    assert start(dtype=2) == -1           # fp8 without scales
    assert start(arena_bytes=-1) == -1
    assert start(idle_checks=-1) == -1
    assert start(arena_bytes=16) == -1    # smaller than one query
    assert start(arena_bytes=1 << 40) == -4
