"""Learned entry point on the GPU: network gradients and Adam against the
float64 oracle, prediction and gating, k-means entry nodes, labels from the
plain search, and what the trained network gains over the fixed entry."""
import numpy as np
import pytest
import torch

import oracle
import paper_2510_05975_amd as cng
import workloads
from oracle import mlp as omlp
from paper_2510_05975_amd import _lib as L, learned
from gpu_util import dev, dev_ids, host_ids
import mlp_bounds
from mlp_bounds import U

pytestmark = pytest.mark.gpu

D, H, K = 96, 256, 1024


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def split(g, d, H, K):
    sizes = [d * H, H, H * H, H, H * K, K]
    return np.split(np.asarray(g), np.cumsum(sizes)[:-1])


@pytest.fixture(scope="module")
def net():
    g = np.random.default_rng(0)
    p = learned.init_params(D, H, K, seed=3)
    p[D * H: D * H + H] = g.standard_normal(H) * 0.1            # non-zero biases
    X = g.standard_normal((64, D)).astype(np.float32)
    y = g.integers(0, K, 64).astype(np.uint32)
    return p, X, y


def test_gradients_fp32_vs_oracle(net):
    """float32 products: every gradient tensor within 1e-5 (relative 2-norm)
    of the float64 network, the loss within 1e-5 relative."""
    p, X, y = net
    P = dev(p[None])[0]
    G = torch.empty_like(P)
    loss = torch.zeros(1, device="cuda:0")
    L.mlp_gradients(P, D, H, K, dev(X), dev_ids(y), None, 64, 0, G, loss)
    torch.cuda.synchronize()
    l64, g64 = omlp.loss_and_grads(p, D, H, K, X, y)
    assert abs(loss.item() - l64) <= 1e-5 * abs(l64)
    for a, b in zip(split(G.cpu().numpy().astype(np.float64), D, H, K), split(g64, D, H, K)):
        assert rel(a, b) <= 1e-5


@pytest.mark.parametrize("standardize", [False, True])
def test_gradients_bf16_layerwise_vs_oracle(net, standardize):
    """One bf16 training step, product by product: from the library's own
    operands (its stored intermediates H1, H2, Z, dZ, dH2, dH1, documented in
    cng_mlp_gradients), every product, ReLU mask, softmax and bias sum against
    the oracle's exact product of the same bf16 operands, within the float32
    accumulation bound (tests/mlp_bounds.py).  With standardize the input
    affine of cng_mlp_input_stats is applied on the device."""
    p, X, y = net
    B = len(X)
    Xin = X * 40.0 + 100.0 if standardize else X
    xd = dev(Xin)
    aff = L.mlp_input_stats(xd) if standardize else None
    P = dev(p[None])[0]
    G = torch.empty_like(P)
    loss = torch.zeros(1, device="cuda:0")
    ws = L.mlp_gradients(P, D, H, K, xd, dev_ids(y), None, B, 1, G, loss, affine=aff)
    torch.cuda.synchronize()
    w = ws[: (4 * B * H + 2 * B * K + B) * 4].view(torch.float32).cpu().numpy().astype(np.float64)
    H1, H2, dH2, dH1 = (w[i * B * H:(i + 1) * B * H].reshape(B, H) for i in range(4))
    Z = w[4 * B * H: 4 * B * H + B * K].reshape(B, K)
    dZ = w[4 * B * H + B * K: 4 * B * H + 2 * B * K].reshape(B, K)
    lrow = w[4 * B * H + 2 * B * K:]
    Xs = omlp.standardized(Xin, aff[0].cpu().numpy(), aff[1].item()) if standardize else Xin
    Xs = Xs.astype(np.float64)
    W1, b1, W2, b2, W3, b3 = omlp.unpack(p, D, H, K)
    g = split(G.cpu().numpy().astype(np.float64), D, H, K)
    checks = {}
    v, e = mlp_bounds.relu_layer(Xs, W1, b1, False)
    checks["H1"] = mlp_bounds.within(H1, v, e)
    v, e = mlp_bounds.relu_layer(H1, W2, b2, False)
    checks["H2"] = mlp_bounds.within(H2, v, e)
    v, e = mlp_bounds.product(H2, W3, b3)
    checks["Z"] = mlp_bounds.within(Z, v, e)
    Pr, eP = mlp_bounds.softmax(Z)
    t = Pr.copy()
    t[np.arange(B), y] -= 1.0
    checks["dZ"] = mlp_bounds.within(dZ, t / B, (eP + U * np.abs(t)) / B)
    m = Z.max(1)
    lo = m + np.log(np.exp(Z - m[:, None]).sum(1)) - Z[np.arange(B), y]
    checks["loss"] = mlp_bounds.within(lrow, lo, mlp_bounds.gamma(K + 16) * (np.abs(m) + np.abs(lo) + np.abs(Z[np.arange(B), y])))
    for name, (A, Bm, gi) in {"W3": (H2.T, dZ, 4), "W2": (H1.T, dH2, 2), "W1": (Xs.T, dH1, 0)}.items():
        v, e = mlp_bounds.product(A, Bm)
        checks["g" + name] = mlp_bounds.within(g[gi].reshape(v.shape), v, e)
    for name, (Dm, gi) in {"b3": (dZ, 5), "b2": (dH2, 3), "b1": (dH1, 1)}.items():
        v, e = mlp_bounds.colsum(Dm)
        checks["g" + name] = mlp_bounds.within(g[gi], v, e)
    v, e = mlp_bounds.product(dZ, W3.T)
    checks["dH2"] = mlp_bounds.within(dH2, v * (H2 > 0), e * (H2 > 0))
    v, e = mlp_bounds.product(dH2, W2.T)
    checks["dH1"] = mlp_bounds.within(dH1, v * (H1 > 0), e * (H1 > 0))
    print("bf16 step, max |lib - oracle| / bound per product:",
          {k: round(r, 4) for k, (_, r) in checks.items()})
    assert all(ok for ok, _ in checks.values()), checks
    assert abs(loss.item() - lrow.mean()) <= 1e-6 * abs(lrow.mean())
    # the whole step against the oracle's own bf16 form (not from the library's
    # intermediates): close, not bit-identical -- reported, not a parity claim
    _, g_o = omlp.loss_and_grads(p, D, H, K, Xs, y, rnd=omlp.round_bf16)
    print("end to end vs the oracle's bf16 form, relative 2-norm per tensor:",
          [round(rel(a, b), 5) for a, b in zip(g, split(g_o, D, H, K))])


def test_logits_fp32_vs_oracle(net):
    p, X, _ = net
    Z = L.mlp_logits(dev(p[None])[0], D, H, K, dev(X), 0)
    _, _, Z64 = omlp.forward(p, D, H, K, X)
    assert rel(Z.cpu().numpy(), Z64) <= 1e-5


def test_input_stats_and_affine():
    """cng_mlp_input_stats against float64 numpy; the network with the input
    affine equals the network on inputs standardized beforehand (float32,
    elementwise), bit for bit, in both precisions."""
    x, _ = workloads.generate(2, n=10000, nq=1)
    xd = dev(x)
    mean, scale = L.mlp_input_stats(xd)
    m64 = x.astype(np.float64).mean(0)
    s64 = np.sqrt(((x.astype(np.float64) - m64.astype(np.float32)) ** 2).mean())
    np.testing.assert_allclose(mean.cpu().numpy(), m64, rtol=1e-6, atol=1e-6)
    assert abs(scale.item() - s64) <= 1e-6 * s64
    d, Hs, Ks = 128, 64, 48
    p = learned.init_params(d, Hs, Ks, seed=5)
    P = dev(p[None])[0]
    q = x[:96]
    xs = omlp.standardized(q, mean.cpu().numpy(), scale.item())
    for prec in (0, 1):
        Za = L.mlp_logits(P, d, Hs, Ks, dev(q), prec, affine=(mean, scale))
        Zb = L.mlp_logits(P, d, Hs, Ks, dev(xs), prec)
        assert torch.equal(Za, Zb)
    y = np.arange(96, dtype=np.uint32) % Ks
    Ga, Gb = torch.empty_like(P), torch.empty_like(P)
    L.mlp_gradients(P, d, Hs, Ks, dev(q), dev_ids(y), None, 96, 1, Ga, affine=(mean, scale))
    L.mlp_gradients(P, d, Hs, Ks, dev(xs), dev_ids(y), None, 96, 1, Gb)
    assert torch.equal(Ga, Gb)


def test_logits_bf16_layerwise_vs_oracle(net):
    """The prediction path (packed bf16 operands, cng_mlp_logits with its
    hidden activations) layer by layer against the oracle's exact products of
    the same bf16 operands: each hidden layer within the float32 accumulation
    bound plus its own bf16 rounding, the logits within the accumulation bound,
    and the argmax equal wherever the top-2 gap exceeds twice the bound."""
    p, X, _ = net
    g = np.random.default_rng(11)
    Xb = np.concatenate([X, g.standard_normal((448, D)).astype(np.float32)]).astype(np.float64)
    Zt, Ht = L.mlp_logits(dev(p[None])[0], D, H, K, dev(Xb), 1, hidden=True)
    Z = Zt.cpu().numpy().astype(np.float64)
    H1, H2 = (h.astype(np.float64) for h in Ht.cpu().numpy())
    W1, b1, W2, b2, W3, b3 = omlp.unpack(p, D, H, K)
    assert (omlp.round_bf16(H1) == H1).all() and (omlp.round_bf16(H2) == H2).all()
    v, e = mlp_bounds.relu_layer(Xb, W1, b1, True)
    ok1, r1 = mlp_bounds.within(H1, v, e)
    v, e = mlp_bounds.relu_layer(H1, W2, b2, True)
    ok2, r2 = mlp_bounds.within(H2, v, e)
    Zo, eZ = mlp_bounds.product(H2, W3, b3)
    ok3, r3 = mlp_bounds.within(Z, Zo, eZ)
    print(f"bf16 prediction path, max |lib - oracle| / bound: H1 {r1:.3g} H2 {r2:.3g} Z {r3:.3g}; "
          f"median logit bound {np.median(eZ):.3g} of median |z| {np.median(np.abs(Zo)):.3g}")
    assert ok1 and ok2 and ok3
    rows = np.arange(len(Zo))
    top2 = np.argsort(-Zo, axis=1)[:, :2]
    gap = Zo[rows, top2[:, 0]] - Zo[rows, top2[:, 1]]
    decided = gap > 2 * (eZ[rows, top2[:, 0]] + eZ[rows, top2[:, 1]])
    assert decided.mean() > 0.9
    assert (Z.argmax(1)[decided] == top2[decided, 0]).all()
    # end to end against the oracle's own bf16 form: report how often the
    # argmax agrees (bf16 rounding of the hidden layers can flip either way)
    _, _, Ze = omlp.forward(p, D, H, K, Xb, rnd=omlp.round_bf16)
    print(f"argmax agreement with the oracle's bf16 form: {(Ze.argmax(1) == Z.argmax(1)).mean():.4f}, "
          f"with float64: {(omlp.forward(p, D, H, K, Xb)[2].argmax(1) == Z.argmax(1)).mean():.4f}")


def test_batch_ids_gather_rows(net):
    p, X, y = net
    P = dev(p[None])[0]
    idx = np.arange(63, -1, -2, dtype=np.uint32)  # 32 rows, reversed, every other one
    G1, G2 = torch.empty_like(P), torch.empty_like(P)
    L.mlp_gradients(P, D, H, K, dev(X), dev_ids(y), dev_ids(idx), 32, 0, G1)
    L.mlp_gradients(P, D, H, K, dev(X[idx]), dev_ids(y[idx]), None, 32, 0, G2)
    torch.cuda.synchronize()
    assert torch.equal(G1, G2)


def test_adam_vs_oracle():
    g = np.random.default_rng(4)
    n = omlp.unpack(np.zeros(L.mlp_param_count(8, 16, 4)), 8, 16, 4)[0].size
    cnt = L.mlp_param_count(8, 16, 4)
    p, gr = g.standard_normal(cnt).astype(np.float32), g.standard_normal(cnt).astype(np.float32)
    m, v = (g.standard_normal(cnt) * 0.1).astype(np.float32), np.abs(g.standard_normal(cnt) * 0.1).astype(np.float32)
    P, Gt, M, V = (dev(a[None])[0] for a in (p, gr, m, v))
    L.mlp_adam(P, Gt, M, V, 8, 16, 4, 7, 1e-3)
    torch.cuda.synchronize()
    p2, m2, v2 = omlp.adam_step(p, gr, m, v, 7, 1e-3)
    # float32 state against the float64 step: float32 resolution (2^-24 ~ 6e-8)
    assert rel(P.cpu().numpy(), p2) <= 1e-6 and rel(M.cpu().numpy(), m2) <= 1e-6
    assert rel(V.cpu().numpy(), v2) <= 1e-6 and n == 8 * 16
    # and the step itself, resolved to float32 rounding of the parameters
    step = P.cpu().numpy().astype(np.float64) - p
    assert np.abs(step - (p2 - p)).max() <= 2 * 2.0 ** -24 * np.abs(p2).max()


def test_predict_and_gate(net):
    """cng_entry_predict uses the logits of cng_mlp_logits (the same packed
    kernels): the entry of their argmax (ties to the lower index), and the
    softmax probability within its float32 bound; with a threshold the gate
    falls back to the navigating node exactly where that probability is below
    it (rows within the bound of the threshold are skipped)."""
    p, X, _ = net
    P = dev(p[None])[0]
    ents = (np.arange(K, dtype=np.uint32) * 7 + 1)
    Z = L.mlp_logits(P, D, H, K, dev(X), 1).cpu().numpy().astype(np.float64)
    Pr, eP = mlp_bounds.softmax(Z)
    top = Z.argmax(1)
    rows = np.arange(len(X))
    conf_o, econf = Pr[rows, top], eP[rows, top]
    out, conf = L.entry_predict(P, D, H, K, dev(X), 1, dev_ids(ents), 999999, 0.0)
    assert (host_ids(out) == ents[top]).all()
    assert (np.abs(conf.cpu().numpy() - conf_o) <= econf).all()
    th = float(np.median(conf_o))
    out2, _ = L.entry_predict(P, D, H, K, dev(X), 1, dev_ids(ents), 999999, th)
    want = np.where(conf_o >= th, ents[top], 999999)
    sure = np.abs(conf_o - th) > econf
    assert sure.sum() >= len(X) - 2
    assert (host_ids(out2)[sure] == want[sure]).all()


def test_kmeans_entries_and_init():
    x, _ = workloads.generate(4, n=20000, nq=1)
    init = np.random.default_rng(1).permutation(len(x))[:64].astype(np.uint32)
    c0, e0 = L.kmeans(dev(x), 64, 0, dev_ids(init))
    assert np.array_equal(c0.cpu().numpy(), x[init])
    c, e = L.kmeans(dev(x), 64, 10, dev_ids(init))
    torch.cuda.synchronize()
    cc = c.cpu().numpy()
    oids, _ = oracle.knn(cc, x, 1)
    assert (host_ids(e) == oids[:, 0]).all()
    # Lloyd never increases the within-cluster sum of squares
    def wcss(cent):
        ids, D2 = oracle.knn(x, cent, 1)
        return D2.sum()
    assert wcss(cc) <= wcss(x[init])


def test_entry_labels_vs_oracle():
    x, q = workloads.generate(1, n=5000, nq=300)
    adj, s, _ = oracle.build(x, 16, 32, 1.2)
    ents = np.random.default_rng(2).permutation(len(x))[:32].astype(np.uint32)
    lab = L.entry_labels(dev(x), dev_ids(adj), s, dev(q), 32, dev_ids(ents))
    top, _, _, _ = oracle.search(x, adj, q, 1, 32, s)
    want, _ = oracle.knn(x[top[:, 0]], x[ents], 1)
    assert (host_ids(lab) == want[:, 0]).all()


def test_learned_entry_beats_fixed_entry():
    """On ten well separated clusters the fixed entry must cross between
    clusters through few repair edges; a trained network starting near the
    query's cluster recovers recall at small beams (a held-out split)."""
    x, _ = workloads.generate(1, n=10000, nq=1)
    ev = workloads.fresh_queries(1, 500, stream=11)
    tr = workloads.fresh_queries(1, 30000, stream=12)
    xd = dev(x)
    g = cng.build(xd, 24, 64, 1.2)
    cent, ents = learned.kmeans_entries(xd, 64, iters=15, seed=1)
    lab = L.entry_labels(xd, g.adj, g.entry, dev(tr), 64, ents)
    model = learned.EntryModel(32, 128, 64, dev(learned.init_params(32, 128, 64, 5)[None])[0],
                               ents, cent, g.entry, theta=0.0, precision=1)
    learned.train(model, dev(tr), lab, epochs=6, batch=256, lr=2e-3, seed=3)
    assert model.history[-1][1] < 0.7 * np.log(64)   # well below a uniform guess
    evd = dev(ev)
    gt, _ = oracle.knn(ev, x, 10)
    pe, conf = model.predict(evd)
    ce = L.nearest_centre_entry(evd, cent, ents)

    def recall(entries, Lb):
        ids, _, _, ndc = cng.search(xd, g.adj, evd, 10, Lb, entries, stats=True)
        r = np.mean([len(set(a) & set(b)) / 10 for a, b in zip(host_ids(ids).tolist(), gt.tolist())])
        return r, float(ndc.float().mean())

    r_med, n_med = recall(g.entry, 12)
    r_mlp, n_mlp = recall(pe, 12)
    r_cen, _ = recall(ce, 12)
    print(f"recall@10 L=12: medoid {r_med:.3f} ({n_med:.0f} ndc), mlp {r_mlp:.3f} ({n_mlp:.0f} ndc), "
          f"nearest centre {r_cen:.3f}", flush=True)
    assert r_mlp >= r_med + 0.05
