"""Error bounds for the bf16 form of the entry network (test helper).

Each matrix product of the library's bf16 path rounds both float32 operands
to bfloat16 (nearest even) and accumulates in float32.  Given the library's
own operands (its inputs, weights and stored intermediates), the oracle forms
the same product exactly in float64 from the same bf16 operands
(``oracle.mlp.round_bf16``), so the two differ only by float32 accumulation:
at most gamma_n = n u / (1 - n u) (u = 2^-24, n = inner length + 2 for the
bias addition and the final rounding) times the sum of the terms' magnitudes.
A result that the library rounds to bf16 itself (the hidden layers of the
prediction path) may in addition be off by that rounding, at most 2^-8 of its
magnitude.  Softmax probabilities computed in float32 err by at most
p (gamma_{K+8} + 8 u + 2 u |z - max z|) (the shifted logits, the exps, their
sum and the reciprocal).  Checking every product this way pins each kernel's
arithmetic; nothing is propagated from layer to layer, so the bounds stay at
float32 resolution."""
import numpy as np

from oracle import mlp

U = 2.0 ** -24


def gamma(n):
    return n * U / (1.0 - n * U)


def product(A, B, bias=None):
    """Exact product of the bf16-rounded operands (+ bias) and its float32
    accumulation bound."""
    Ab, Bb = mlp.round_bf16(A), mlp.round_bf16(B)
    C = Ab @ Bb
    mag = np.abs(Ab) @ np.abs(Bb)
    if bias is not None:
        C = C + bias
        mag = mag + np.abs(bias)
    return C, gamma(A.shape[1] + 2) * mag


def within(got, want, bound):
    got = np.asarray(got, np.float64)
    return bool((np.abs(got - want) <= bound).all()), float((np.abs(got - want) / np.maximum(bound, 1e-300)).max())


def relu_layer(A, B, bias, out_bf16):
    """ReLU(A B + bias): oracle value and bound (plus the library's own bf16
    rounding of the result when out_bf16)."""
    C, e = product(A, B, bias)
    v = np.maximum(C, 0.0)
    if out_bf16:
        e = e + 2.0 ** -8 * (v + e)
    return v, e


def softmax(Z):
    """Probabilities from float32 logits (float64) and their float32 bound."""
    Z = np.asarray(Z, np.float64)
    K = Z.shape[1]
    m = Z.max(1, keepdims=True)
    E = np.exp(Z - m)
    P = E / E.sum(1, keepdims=True)
    return P, P * (gamma(K + 8) + 8 * U + 2 * U * np.abs(Z - m))


def colsum(X):
    X = np.asarray(X, np.float64)
    return X.sum(0), gamma(X.shape[0] + 1) * np.abs(X).sum(0)
