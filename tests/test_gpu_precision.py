"""Precision form on the GPU against the oracle: bf16 / fp8-E4M3 storage,
reduced-precision scoring and the float32 re-rank of the final beam.  The
stored values, the beam and the re-ranked outputs are all bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_2510_05975_amd as cng
import workloads
from gpu_util import dev, dev_ids, f32_of, host_ids, oracle_qsearch, same_f32

pytestmark = pytest.mark.gpu


def e4m3_values(codes) -> np.ndarray:
    """E4M3 values of uint8 codes (decoded on the host)."""
    codes = np.asarray(codes).astype(np.uint32)
    e, m, sgn = (codes >> 3) & 0xF, codes & 7, np.where(codes & 0x80, -1.0, 1.0)
    val = np.where(e == 0, m * 2.0 ** -9, (8 + m) * 2.0 ** (e.astype(np.int64) - 10)) * sgn
    return val.astype(np.float32)


def stored_values(st: cng.Store) -> np.ndarray:
    """float32 values the device copy stands for (decoded on the host)."""
    if st.dtype == cng.BF16:
        b = st.vecs.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        return b.view(np.float32)
    val = e4m3_values(st.vecs.cpu().numpy())
    return (val * st.scales.cpu().numpy()[:, 0:1]).astype(np.float32)


@pytest.mark.parametrize("dtype", [cng.BF16, cng.FP8])
@pytest.mark.parametrize("cfg,n", [(1, 3000), (3, 500), (4, 2000), (2, 1000)])
def test_quantize_matches_oracle(dtype, cfg, n):
    x, _ = workloads.generate(cfg, n=n, nq=1)
    x[3] = 0.0
    st = cng.quantize(dev(x), dtype)
    torch.cuda.synchronize()
    want, sc = oracle.dequantized(x, dtype)
    assert same_f32(stored_values(st), want)
    if dtype == cng.FP8:
        c, s, n2 = oracle.fp8_encode(x)
        sn = st.scales.cpu().numpy()
        assert same_f32(e4m3_values(st.vecs.cpu().numpy()), c)
        assert same_f32(sn[:, 0], s) and same_f32(sn[:, 1], n2)


def test_fp8_codes_saturate_and_keep_sign():
    x = np.array([[448.0, -448.0, 1e-3, -1e-3, 0.0, 300.0, -304.0, 2.0 ** -10]], np.float32)
    st = cng.quantize(dev(x), cng.FP8)
    want, _ = oracle.dequantized(x, cng.FP8)
    assert same_f32(stored_values(st), want)
    assert same_f32(st.scales.cpu().numpy()[:, 1], oracle.fp8_encode(x)[2])


def gpu_qsearch(x, st, adj, q, k, L, e, vlog2=14):
    ids, d, h, n = cng.search_quantized(dev(x), st, dev_ids(adj), dev(q), k, L, e,
                                        visited_log2=vlog2, stats=True)
    torch.cuda.synchronize()
    return host_ids(ids), d.cpu().numpy(), h.cpu().numpy().astype(np.uint32), n.cpu().numpy().astype(np.uint32)


@pytest.mark.parametrize("dtype", [cng.BF16, cng.FP8])
@pytest.mark.parametrize("cfg,n,R,C", [(1, 6000, 24, 64), (3, 1500, 24, 48), (4, 4000, 32, 64)])
def test_quantized_search_bit_exact(dtype, cfg, n, R, C):
    print(f"qsearch dtype={dtype} cfg{cfg}", flush=True)
    x, q = workloads.generate(cfg, n=n, nq=120)
    adj, e, _ = oracle.build(x, R, C, 1.2)
    st = cng.quantize(dev(x), dtype)
    for L, k in [(32, 10), (64, 10), (8, 20)]:
        g = gpu_qsearch(x, st, adj, q, k, L, e)
        o = oracle_qsearch(dtype, x, adj, q, k, L, e)
        assert (g[0] == o[0]).all(), np.argwhere(g[0] != o[0])[:5]
        assert same_f32(g[1], f32_of(o[1]))
        assert (g[2] == o[2]).all() and (g[3] == o[3]).all()


@pytest.mark.parametrize("d", [5, 33, 100, 300, 1500, 4096])
def test_quantized_search_dims(d):
    x, q = workloads.uniform_cube(800, 30, d, seed=d)
    adj, e, _ = oracle.build(x, 10, 20, 1.2)
    for dtype in (cng.BF16, cng.FP8):
        st = cng.quantize(dev(x), dtype)
        g = gpu_qsearch(x, st, adj, q, 10, 24, e)
        o = oracle_qsearch(dtype, x, adj, q, 10, 24, e)
        assert (g[0] == o[0]).all() and same_f32(g[1], f32_of(o[1]))


def test_bf16_on_small_integers_equals_float32_search():
    x, q = workloads.generate(2, n=4000, nq=100)
    adj, e, _ = oracle.build(x, 32, 64, 1.2)
    st = cng.quantize(dev(x), cng.BF16)
    g = gpu_qsearch(x, st, adj, q, 10, 48, e)
    o = oracle.search(x, adj, q, 10, 48, e)
    assert (g[0] == o[0]).all() and same_f32(g[1], f32_of(o[1]))
