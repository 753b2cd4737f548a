"""Pins for the float64 MLP oracle of the learned entry point: central finite
differences, an independent autograd implementation (torch, float64, CPU) and
softmax/Adam identities."""
import numpy as np
import torch

from oracle import mlp
import workloads


def small(seed=0, d=7, H=11, K=5, B=9):
    g = np.random.default_rng(seed)
    n = d * H + H + H * H + H + H * K + K
    p = g.standard_normal(n) * 0.5
    X = g.standard_normal((B, d))
    y = g.integers(0, K, B)
    return p, X, y, (d, H, K)


def test_gradients_match_finite_differences():
    p, X, y, (d, H, K) = small()
    loss, g = mlp.loss_and_grads(p, d, H, K, X, y)
    assert abs(loss - mlp.loss_only(p, d, H, K, X, y)) < 1e-12
    h = 1e-6
    rng = np.random.default_rng(1)
    for i in rng.choice(p.size, 60, replace=False):
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_only(p + e, d, H, K, X, y) - mlp.loss_only(p - e, d, H, K, X, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))


def test_gradients_match_torch_autograd():
    p, X, y, (d, H, K) = small(seed=3, d=12, H=16, K=9, B=20)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    sizes = [d * H, H, H * H, H, H * K, K]
    W1, b1, W2, b2, W3, b3 = torch.split(pt, sizes)
    Xt = torch.tensor(X)
    h1 = torch.relu(Xt @ W1.view(d, H) + b1)
    h2 = torch.relu(h1 @ W2.view(H, H) + b2)
    z = h2 @ W3.view(H, K) + b3
    loss = torch.nn.functional.cross_entropy(z, torch.tensor(y))
    loss.backward()
    l2, g = mlp.loss_and_grads(p, d, H, K, X, y)
    assert abs(loss.item() - l2) < 1e-12
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_output_gradient_rows_sum_to_zero():
    # d(loss)/d(b3) summed over classes is zero for softmax cross-entropy
    p, X, y, (d, H, K) = small(seed=5)
    _, g = mlp.loss_and_grads(p, d, H, K, X, y)
    assert abs(g[-K:].sum()) < 1e-12


def test_adam_first_step_moves_by_lr():
    # with bias correction the first step is lr * sign(g) (up to eps)
    g = np.array([0.3, -2.0, 1e-3])
    p1, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    np.testing.assert_allclose(p1, -0.01 * np.sign(g), rtol=1e-4)


def test_fresh_queries_share_the_distribution():
    x, _ = workloads.generate(1, n=3000, nq=1)
    t = workloads.fresh_queries(1, 3000, stream=7)
    t2 = workloads.fresh_queries(1, 3000, stream=8)
    assert not np.array_equal(t, t2)
    # same centres: the per-cluster means of the base set explain the new queries
    assert abs(np.linalg.norm(x.mean(0)) - np.linalg.norm(t.mean(0))) < 0.5


def test_adam_second_step_closed_forms():
    """Two bias-corrected steps, worked out by hand.  A constant gradient g
    gives m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so every step moves by
    lr * sign(g) (up to eps).  Gradients +1 then -1 give m_2 = -(1 - b1)^2 and
    v_2 = 1 - b2^2, so the second step adds lr (1 - b1) / (1 + b1) (= lr / 19
    at b1 = 0.9)."""
    lr = 0.01
    g = np.array([0.7, -3.0])
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in (1, 2, 3):
        p, m, v = mlp.adam_step(p, g, m, v, t, lr)
        np.testing.assert_allclose(p, -t * lr * np.sign(g), rtol=1e-6)
    p1, m, v = mlp.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 1, lr)
    p2, m, v = mlp.adam_step(p1, -np.ones(1), m, v, 2, lr)
    np.testing.assert_allclose(m, [-(0.1 ** 2)], rtol=1e-12)
    np.testing.assert_allclose(v, [1 - 0.999 ** 2], rtol=1e-12)
    np.testing.assert_allclose(p2, p1 + lr / 19, rtol=1e-7)
