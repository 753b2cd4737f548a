"""The allocation-free entry prediction (cng_entry_predict_noalloc, scratch
in the library's fixed device array) against cng_entry_predict with a
workspace, through the C ABI: identical entries and confidences on two calls
in a row, the second with a smaller batch; shapes beyond the array refused
before any launch."""
import numpy as np
import pytest
import torch

import paper_2510_05975_amd as cng
from paper_2510_05975_amd import _lib as L, learned
from gpu_util import dev, dev_ids

pytestmark = pytest.mark.gpu


def test_noalloc_predict_equals_workspace_predict():
    d, H, K = 96, 256, 1024
    g = np.random.default_rng(21)
    P = dev(learned.init_params(d, H, K, seed=9)[None])[0]
    ents = dev_ids((np.arange(K, dtype=np.uint32) * 13 + 5) % 100000)
    X = g.standard_normal((800, d)).astype(np.float32) * 3 + 1
    xd = dev(X)
    aff = L.mlp_input_stats(xd)
    for B, prec, th in [(800, 1, 0.002), (300, 1, 0.0), (77, 0, 0.001)]:
        q = xd[:B].contiguous()
        e1, c1 = L.entry_predict(P, d, H, K, q, prec, ents, 424242, th, affine=aff)
        e2, c2 = L.entry_predict_noalloc(P, d, H, K, q, prec, ents, 424242, th, affine=aff)
        torch.cuda.synchronize()
        assert torch.equal(e1, e2) and torch.equal(c1, c2), (B, prec)


def test_noalloc_refuses_shapes_beyond_the_array():
    d, H, K = 96, 256, 1024
    cap = L.lib().cng_entry_predict_noalloc_max_bytes()
    assert cap == 16 << 20
    B = 8192
    assert L.lib().cng_mlp_workspace_size(d, H, K, B) > cap
    P = torch.zeros(L.mlp_param_count(d, H, K), device="cuda:0")
    X = torch.zeros((B, d), device="cuda:0")
    with pytest.raises(cng.CngError) as ei:
        L.entry_predict_noalloc(P, d, H, K, X, 1, torch.zeros(K, dtype=torch.int32, device="cuda:0"),
                                0, 0.0)
    assert ei.value.status == -4
