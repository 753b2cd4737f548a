"""Float64 oracle of the learned entry point's network -- TEST INFRASTRUCTURE ONLY.

Multilayer perceptron d -> H -> H -> K with ReLU hidden layers, softmax
cross-entropy loss averaged over the batch, and Adam, written out plainly in
numpy float64.  Parameter layout (one flat vector): W1 [d x H], b1 [H],
W2 [H x H], b2 [H], W3 [H x K], b3 [K], with y = x W + b.

``rnd`` (optional) is applied to both operands of every matrix product and
nothing else: with ``round_bf16`` it describes the bf16 form of the network
(operands rounded to bfloat16, products summed exactly, everything else in
float64).  Without it the network is plain float64.
"""
from __future__ import annotations

import numpy as np


def unpack(p, d, H, K):
    p = np.asarray(p, np.float64)
    sizes = [d * H, H, H * H, H, H * K, K]
    parts = np.split(p, np.cumsum(sizes)[:-1])
    W1, b1, W2, b2, W3, b3 = parts
    return W1.reshape(d, H), b1, W2.reshape(H, H), b2, W3.reshape(H, K), b3


def round_bf16(a):
    """Nearest bfloat16 (8 significant bits, ties to even) of the float32
    value of each element, returned as float64."""
    b = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32)).view(np.uint32)
    b = b.astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(A, B, rnd):
    return (rnd(A) @ rnd(B)) if rnd is not None else A @ B


def forward(p, d, H, K, X, rnd=None):
    W1, b1, W2, b2, W3, b3 = unpack(p, d, H, K)
    X = np.asarray(X, np.float64)
    A1 = _mm(X, W1, rnd) + b1
    H1 = np.maximum(A1, 0.0)
    A2 = _mm(H1, W2, rnd) + b2
    H2 = np.maximum(A2, 0.0)
    Z = _mm(H2, W3, rnd) + b3
    return H1, H2, Z


def standardized(X, mean, scale):
    """The network's input (x - mean) / scale, elementwise in float32."""
    return ((np.asarray(X, np.float32) - np.asarray(mean, np.float32)) /
            np.float32(scale)).astype(np.float32)


def loss_and_grads(p, d, H, K, X, y, rnd=None):
    """Mean softmax cross-entropy and its gradient (flat, same layout as p)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, d, H, K)
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.int64)
    B = X.shape[0]
    H1, H2, Z = forward(p, d, H, K, X, rnd)
    m = Z.max(1, keepdims=True)
    E = np.exp(Z - m)
    S = E.sum(1, keepdims=True)
    P = E / S
    loss = float(np.mean((m[:, 0] + np.log(S[:, 0])) - Z[np.arange(B), y]))
    dZ = P.copy()
    dZ[np.arange(B), y] -= 1.0
    dZ /= B
    gW3 = _mm(H2.T, dZ, rnd)
    gb3 = dZ.sum(0)
    dH2 = _mm(dZ, W3.T, rnd) * (H2 > 0)
    gW2 = _mm(H1.T, dH2, rnd)
    gb2 = dH2.sum(0)
    dH1 = _mm(dH2, W2.T, rnd) * (H1 > 0)
    gW1 = _mm(X.T, dH1, rnd)
    gb1 = dH1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def loss_only(p, d, H, K, X, y):
    _, _, Z = forward(p, d, H, K, X)
    y = np.asarray(y, np.int64)
    m = Z.max(1, keepdims=True)
    return float(np.mean(m[:, 0] + np.log(np.exp(Z - m).sum(1)) - Z[np.arange(len(y)), y]))


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (Kingma & Ba)."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
