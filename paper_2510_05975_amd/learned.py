"""Learned entry point: k-means entry nodes, labels from the plain search,
MLP training and gated prediction.  This module only sequences library calls;
every computation runs in libcng's kernels (the input standardisation too:
its statistics come from cng_mlp_input_stats and every network call applies
it).  Random draws (initial weights, k-means seeds, epoch permutations) come
from numpy generators on the host and are passed in as inputs."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L


def init_params(d: int, H: int, K: int, seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, in the library's parameter order."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, fan_out in ((d, H), (H, H), (H, K)):
        parts.append((g.standard_normal((fan_in, fan_out)) * np.sqrt(2.0 / fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == L.mlp_param_count(d, H, K)
    return p


@dataclass
class EntryModel:
    d: int
    H: int
    K: int
    params: torch.Tensor
    entries: torch.Tensor          # [K] entry node ids
    centers: torch.Tensor          # [K, d] k-means centres
    fallback: int                  # navigating node
    theta: float = 0.0
    precision: int = 1             # 1: bf16 products, 0: float32
    affine: tuple | None = None    # (x_mean [d], x_scale [1]) of the input standardisation
    history: list = field(default_factory=list)

    def predict(self, queries: torch.Tensor, theta: float | None = None):
        th = self.theta if theta is None else theta
        return L.entry_predict(self.params, self.d, self.H, self.K, queries, self.precision,
                               self.entries, self.fallback, th, affine=self.affine)

    def logits(self, queries: torch.Tensor):
        return L.mlp_logits(self.params, self.d, self.H, self.K, queries, self.precision,
                            affine=self.affine)


def kmeans_entries(points: torch.Tensor, K: int, iters: int = 20, seed: int = 1):
    g = np.random.Generator(np.random.PCG64(seed))
    init = g.permutation(points.shape[0])[:K].astype(np.int32)
    return L.kmeans(points, K, iters, torch.from_numpy(init).to(points.device))


def train(model: EntryModel, X: torch.Tensor, labels: torch.Tensor, epochs: int = 4,
          batch: int = 1024, lr: float = 1e-3, seed: int = 2, log_every: int = 0,
          standardize: bool = True):
    """Adam on mini-batches drawn by a seeded permutation per epoch.

    With ``standardize`` the network sees (x - mean) / scale, the statistics
    of the training queries (cng_mlp_input_stats); the model keeps them and
    prediction applies the same map.  Data of large magnitude (e.g. integers
    in [0, 255]) does not train otherwise."""
    n = X.shape[0]
    dev = X.device
    model.affine = L.mlp_input_stats(X) if standardize else None
    P = model.params
    G = torch.empty_like(P)
    m1 = torch.zeros_like(P)
    m2 = torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    rng = np.random.Generator(np.random.PCG64(seed))
    ws = None
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(dev)
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            ws = L.mlp_gradients(P, model.d, model.H, model.K, X, labels, idx, batch,
                                 model.precision, G, loss, ws, affine=model.affine)
            step += 1
            L.mlp_adam(P, G, m1, m2, model.d, model.H, model.K, step, lr)
            if log_every and step % log_every == 0:
                model.history.append((step, float(loss.item())))
        model.history.append((step, float(loss.item())))
    return model
