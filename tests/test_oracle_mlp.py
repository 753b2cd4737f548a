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


def test_round_bf16_matches_c_oracle_and_is_identity_on_bf16_values():
    import oracle
    g = np.random.default_rng(9)
    v = np.concatenate([g.standard_normal(300) * 10.0 ** g.integers(-6, 6, 300),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 255.0, 257.0]])
    r = mlp.round_bf16(v)
    assert all(r[i] == oracle.round_bf16(float(np.float32(v[i]))) for i in range(len(v)))
    assert (mlp.round_bf16(r) == r).all()
    assert mlp.round_bf16([1.0 + 2 ** -8])[0] == 1.0           # tie to even
    assert mlp.round_bf16([1.0 + 3 * 2 ** -8])[0] == 1.0 + 2 ** -6


def test_bf16_form_equals_float64_on_bf16_representable_operands():
    """With operands that bf16 holds exactly (small dyadic values) and
    activations that stay so, the bf16 form is the float64 network."""
    g = np.random.default_rng(4)
    d, H, K, B = 4, 6, 5, 7
    n = d * H + H + H * H + H + H * K + K
    p = g.integers(-3, 4, n) / 4.0
    X = g.integers(-2, 3, (B, d)).astype(np.float64)
    y = g.integers(0, K, B)
    _, _, Z = mlp.forward(p, d, H, K, X)
    _, _, Zb = mlp.forward(p, d, H, K, X, rnd=mlp.round_bf16)
    H1, H2, _ = mlp.forward(p, d, H, K, X)
    assert (mlp.round_bf16(H1) == H1).all() and (mlp.round_bf16(H2) == H2).all()
    assert (Z == Zb).all()
    # and rounding changes the result where the operands are not bf16 values
    p2 = p + 1e-3
    _, _, Z2 = mlp.forward(p2, d, H, K, X)
    _, _, Z2b = mlp.forward(p2, d, H, K, X, rnd=mlp.round_bf16)
    assert not (Z2 == Z2b).all()
    l1, g1 = mlp.loss_and_grads(p, d, H, K, X, y)
    l2, g2 = mlp.loss_and_grads(p, d, H, K, X, y, rnd=lambda a: np.asarray(a, np.float64))
    assert l1 == l2 and (g1 == g2).all()


def test_standardized_is_float32_elementwise():
    X = np.array([[1.0, 2.0], [3.0, 7.0]], np.float32)
    m = np.array([2.0, 4.5], np.float32)
    s = np.float32(3.0)
    out = mlp.standardized(X, m, s)
    assert out.dtype == np.float32
    assert out[0, 0] == np.float32(-1.0) / np.float32(3.0)
    assert out[1, 1] == np.float32(2.5) / np.float32(3.0)
