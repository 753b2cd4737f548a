"""Seeded synthetic workloads for the alpha-CNG build and search.

This module only draws random numbers: it holds none of the method's
arithmetic (no distances, no pruning, no search).  Both the CPU oracle's tests
and the GPU path's tests, benchmarks and smoke check take their inputs from
here, so the two sides see byte-identical arrays.

The paper evaluates on public datasets (SIFT, GIST, DEEP, BIGANN ...; paper
Section 5.1, Table 2) that are not available here.  Each generator below is a
stand-in with the same shape, value range and low intrinsic dimension:

* ``mixture``   -- 10 isotropic Gaussians in 32 dims (small CPU-feasible case).
* ``sift_like`` -- d=128, integer values in [0, 255] (SIFT/BIGANN-shaped):
  ``rint(255 * sigmoid(z @ W + eps))`` with a 16-dim latent ``z``.
* ``gist_like`` -- d=960 from a 32-dim latent map plus small noise (GIST-shaped).
* ``vmf``       -- unit vectors in 96 dims from a 100-centre von Mises-Fisher
  mixture with kappa=50 (DEEP-shaped, angular).

Every generator uses one ``numpy.random.Generator(PCG64(seed))`` and draws in
the order written in its docstring.  Large arrays are drawn in row chunks of
``CHUNK`` rows; the chunking is part of the recipe, so a given (seed, n, nq)
always yields the same bytes.
"""
from __future__ import annotations

import numpy as np

CHUNK = 65536

# Workload table: sizes and parameters of the five standard cases.
#   C: candidate pool size, R: out-degree cap, L: beam widths to sweep.
CONFIGS = {
    1: dict(name="mixture10k", gen="mixture", n=10_000, d=32, nq=100, C=64, R=24,
            alpha=1.2, tau=0.0, k=10, L=[32]),
    2: dict(name="sift_like_1m", gen="sift_like", n=1_000_000, d=128, nq=10_000, C=128, R=32,
            alpha=1.2, tau=0.0, k=10, L=[16, 24, 32, 48, 64, 96, 128, 192, 256]),
    3: dict(name="gist_like_1m", gen="gist_like", n=1_000_000, d=960, nq=1_000, C=192, R=48,
            alpha=1.2, tau=0.0, k=10, L=[16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512]),
    4: dict(name="vmf_10m", gen="vmf", n=10_000_000, d=96, nq=10_000, C=128, R=32,
            alpha=1.2, tau=0.0, k=10, L=[32, 48, 64, 96, 128, 192, 256, 384, 512]),
    5: dict(name="sift_like_10m", gen="sift_like", n=10_000_000, d=128, nq=10_000, C=128, R=32,
            alpha=1.2, tau=0.0, k=10, L=[32, 64, 128, 256]),
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def mixture(n: int, nq: int, seed: int = 0, d: int = 32, n_centres: int = 10,
            centre_sigma: float = 2.0):
    """Gaussian mixture.  Draw order: centres (n_centres x d, N(0, centre_sigma^2)),
    then per base chunk: labels (uniform over centres) and N(0,1) offsets, then the
    same for the queries."""
    g = _rng(seed)
    centres = g.standard_normal((n_centres, d)) * centre_sigma

    def draw(m):
        out = np.empty((m, d), np.float32)
        for a in range(0, m, CHUNK):
            b = min(m, a + CHUNK)
            lab = g.integers(0, n_centres, size=b - a)
            out[a:b] = (centres[lab] + g.standard_normal((b - a, d))).astype(np.float32)
        return out

    return draw(n), draw(nq)


def sift_like(n: int, nq: int, seed: int = 0, d: int = 128, latent: int = 16,
              noise: float = 0.5):
    """Integer-valued vectors in [0, 255].  Draw order: W (latent x d, N(0, 1/latent)),
    then per chunk: z (rows x latent, N(0,1)) and eps (rows x d, N(0, noise^2));
    x = rint(255 * sigmoid(z @ W + eps)) with round-half-even.  Queries follow the
    base set in the same stream."""
    g = _rng(seed)
    W = g.standard_normal((latent, d)) / np.sqrt(latent)

    def draw(m):
        out = np.empty((m, d), np.float32)
        for a in range(0, m, CHUNK):
            b = min(m, a + CHUNK)
            z = g.standard_normal((b - a, latent))
            eps = g.standard_normal((b - a, d)) * noise
            v = 255.0 / (1.0 + np.exp(-(z @ W + eps)))
            out[a:b] = np.rint(v).astype(np.float32)
        return out

    return draw(n), draw(nq)


def gist_like(n: int, nq: int, seed: int = 0, d: int = 960, latent: int = 32,
              noise: float = 0.1):
    """Low-rank real vectors.  Draw order: W (latent x d, N(0, 1/latent)), then per
    chunk z (rows x latent) and noise (rows x d, N(0, noise^2)); x = z @ W + noise."""
    g = _rng(seed)
    W = g.standard_normal((latent, d)) / np.sqrt(latent)

    def draw(m):
        out = np.empty((m, d), np.float32)
        for a in range(0, m, CHUNK):
            b = min(m, a + CHUNK)
            z = g.standard_normal((b - a, latent))
            out[a:b] = (z @ W + g.standard_normal((b - a, d)) * noise).astype(np.float32)
        return out

    return draw(n), draw(nq)


def _vmf_cosines(g: np.random.Generator, m: int, p: int, kappa: float) -> np.ndarray:
    """Wood (1994) rejection sampler for the cosine w between a vMF(mu, kappa)
    sample on S^{p-1} and its mean direction."""
    b = (-2.0 * kappa + np.sqrt(4.0 * kappa * kappa + (p - 1.0) ** 2)) / (p - 1.0)
    x0 = (1.0 - b) / (1.0 + b)
    c = kappa * x0 + (p - 1.0) * np.log(1.0 - x0 * x0)
    out = np.empty(m)
    filled = 0
    while filled < m:
        want = int((m - filled) * 1.2) + 16
        z = g.beta((p - 1.0) / 2.0, (p - 1.0) / 2.0, size=want)
        u = g.random(want)
        w = (1.0 - (1.0 + b) * z) / (1.0 - (1.0 - b) * z)
        ok = kappa * w + (p - 1.0) * np.log(1.0 - x0 * w) - c >= np.log(u)
        w = w[ok][: m - filled]
        out[filled:filled + w.size] = w
        filled += w.size
    return out


def vmf(n: int, nq: int, seed: int = 0, d: int = 96, n_centres: int = 100,
        kappa: float = 50.0, query_seed: int | None = None):
    """Unit vectors from a von Mises-Fisher mixture.  Draw order: centres
    (normalised Gaussians), then per chunk: labels, cosines (Wood's sampler),
    tangent Gaussians.  Rows are normalised in float64, cast to float32 and
    normalised again in float32.  Queries come from ``query_seed`` (default
    seed + 1) with the same centres."""
    g = _rng(seed)
    centres = g.standard_normal((n_centres, d))
    centres /= np.linalg.norm(centres, axis=1, keepdims=True)

    def draw(gen, m):
        out = np.empty((m, d), np.float32)
        for a in range(0, m, CHUNK):
            b = min(m, a + CHUNK)
            lab = gen.integers(0, n_centres, size=b - a)
            mu = centres[lab]
            w = _vmf_cosines(gen, b - a, d, kappa)
            v = gen.standard_normal((b - a, d))
            v -= np.sum(v * mu, axis=1, keepdims=True) * mu
            v /= np.linalg.norm(v, axis=1, keepdims=True)
            x = w[:, None] * mu + np.sqrt(np.maximum(0.0, 1.0 - w * w))[:, None] * v
            x /= np.linalg.norm(x, axis=1, keepdims=True)
            x32 = x.astype(np.float32)
            x32 /= np.linalg.norm(x32, axis=1, keepdims=True).astype(np.float32)
            out[a:b] = x32
        return out

    base = draw(g, n)
    q = draw(_rng(seed + 1 if query_seed is None else query_seed), nq)
    return base, q


GENERATORS = dict(mixture=mixture, sift_like=sift_like, gist_like=gist_like, vmf=vmf)


def generate(cfg: int, n: int | None = None, nq: int | None = None, seed: int = 0):
    """Base points and queries of standard case ``cfg`` (optionally resized)."""
    c = CONFIGS[cfg]
    gen = GENERATORS[c["gen"]]
    return gen(c["n"] if n is None else n, c["nq"] if nq is None else nq, seed=seed, d=c["d"])


def uniform_cube(n: int, nq: int, d: int, seed: int = 0, scale: float = 1.0):
    """Plain uniform points in [0, scale)^d (tiny property tests)."""
    g = _rng(seed)
    return ((g.random((n, d)) * scale).astype(np.float32),
            (g.random((nq, d)) * scale).astype(np.float32))


def fresh_queries(cfg: int, nq: int, stream: int, seed: int = 0):
    """nq new queries from the same distribution as standard case ``cfg`` (the
    same centres / latent map, drawn first from ``seed``), sampled from an
    independent generator keyed by (seed, stream) -- e.g. training queries that
    share no draws with the base set or the evaluation queries."""
    c = CONFIGS[cfg]
    gname, d = c["gen"], c["d"]
    qg = _rng(1_000_003 * (seed + 1) + stream)
    if gname == "vmf":
        return vmf(0, nq, seed=seed, d=d, query_seed=1_000_003 * (seed + 1) + stream)[1]
    g = _rng(seed)
    out = np.empty((nq, d), np.float32)
    if gname == "mixture":
        centres = g.standard_normal((10, d)) * 2.0
        for a in range(0, nq, CHUNK):
            b = min(nq, a + CHUNK)
            lab = qg.integers(0, 10, size=b - a)
            out[a:b] = (centres[lab] + qg.standard_normal((b - a, d))).astype(np.float32)
    elif gname == "sift_like":
        W = g.standard_normal((16, d)) / np.sqrt(16)
        for a in range(0, nq, CHUNK):
            b = min(nq, a + CHUNK)
            z = qg.standard_normal((b - a, 16))
            eps = qg.standard_normal((b - a, d)) * 0.5
            out[a:b] = np.rint(255.0 / (1.0 + np.exp(-(z @ W + eps)))).astype(np.float32)
    else:
        W = g.standard_normal((32, d)) / np.sqrt(32)
        for a in range(0, nq, CHUNK):
            b = min(nq, a + CHUNK)
            z = qg.standard_normal((b - a, 32))
            out[a:b] = (z @ W + qg.standard_normal((b - a, d)) * 0.1).astype(np.float32)
    return out
