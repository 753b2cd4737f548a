"""Pins for the oracle's distance (paper Section 2.1: Euclidean metric).

The fixed-order single precision distance is a design choice (the paper fixes
no reduction order); it is pinned here against (a) exact rational arithmetic
that applies the same order with an independently written round-to-nearest-even,
(b) a hand-worked case where the order changes the result, (c) exactness on
small integers, (d) the rounding error bound, and (e) symmetry / zero padding.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def round_f32(r: Fraction) -> Fraction:
    """Round a rational to the nearest binary32 value, ties to even."""
    if r == 0:
        return Fraction(0)
    sign = -1 if r < 0 else 1
    a = abs(r)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)                      # subnormal range shares the 2^-149 step
    ulp = Fraction(2) ** (e - 23)
    q, rem = divmod(a, ulp)
    q = int(q)
    if rem * 2 > ulp or (rem * 2 == ulp and q % 2 == 1):
        q += 1
    return sign * q * ulp


def emulate_canonical(x, y) -> Fraction:
    """The fixed order written out with exact rationals and explicit rounding."""
    d = len(x)
    acc = [Fraction(0)] * 32
    for i in range(d):
        lane = (i // 4) % 32
        t = round_f32(Fraction(float(x[i])) - Fraction(float(y[i])))
        acc[lane] = round_f32(t * t + acc[lane])      # fused multiply-add: one rounding
    off = 16
    while off >= 1:
        acc = [round_f32(acc[l] + acc[l ^ off]) for l in range(32)]
        off //= 2
    return acc[0]


@pytest.mark.parametrize("d", [1, 3, 4, 5, 31, 32, 33, 100, 128, 129, 300])
def test_matches_exact_rational_emulation(d):
    g = np.random.default_rng(d)
    for trial in range(3):
        x = (g.standard_normal(d) * 10 ** g.uniform(-3, 3)).astype(np.float32)
        y = (g.standard_normal(d) * 10 ** g.uniform(-3, 3)).astype(np.float32)
        got = oracle.dist_f32(x, y)
        assert Fraction(float(got)) == emulate_canonical(x, y)


def test_hand_worked_order_case():
    # Lane 0 holds elements 0..3, lane 1 elements 4..7.  With t = (4096, 1, 0, 0 | 0.5, 0 ...)
    # lane 0: fma(4096, 4096, 0) = 2^24, then fma(1, 1, 2^24) = 2^24 + 1 -> ties to even 2^24.
    # lane 1: 0.25.  Butterfly: only lanes 0 and 1 are non-zero, the last step adds them:
    # 2^24 + 0.25 -> 2^24.  (Summing the small terms first would give 2^24 + 2.)
    x = np.zeros(8, np.float32)
    y = np.zeros(8, np.float32)
    x[0], x[1], x[4] = 4096.0, 1.0, 0.5
    assert float(oracle.dist_f32(x, y)) == 16777216.0
    assert oracle.dist_f64(x, y) == 16777217.25


def test_exact_on_small_integers():
    g = np.random.default_rng(1)
    for d in (7, 128, 960):
        x = g.integers(0, 256, d).astype(np.float32)
        y = g.integers(0, 256, d).astype(np.float32)
        exact = int(np.sum((x.astype(np.int64) - y.astype(np.int64)) ** 2))
        if exact < 2 ** 24:
            assert float(oracle.dist_f32(x, y)) == exact
        assert oracle.dist_f64(x, y) == exact


@pytest.mark.parametrize("d", [2, 32, 128, 960])
def test_error_bound_vs_exact(d):
    u = 2.0 ** -24
    m = 2 + 4 * ((d + 127) // 128) + 5          # roundings along the longest chain
    gamma = m * u / (1 - m * u)
    g = np.random.default_rng(100 + d)
    for _ in range(5):
        x = g.standard_normal(d).astype(np.float32)
        y = g.standard_normal(d).astype(np.float32)
        exact = sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(x, y))
        got = Fraction(float(oracle.dist_f32(x, y)))
        assert abs(got - exact) <= Fraction(gamma) * exact
        got64 = Fraction(oracle.dist_f64(x, y))
        assert abs(got64 - exact) <= Fraction(m * 2.0 ** -53 * 1.01) * exact


def test_symmetric_and_zero_padding():
    g = np.random.default_rng(5)
    for d in (5, 32, 77, 128, 200):
        x = g.standard_normal(d).astype(np.float32)
        y = g.standard_normal(d).astype(np.float32)
        assert oracle.dist_f32(x, y) == oracle.dist_f32(y, x)
        # appending zero coordinates to both vectors changes nothing
        pad = (-d) % 128 + 128
        xp = np.concatenate([x, np.zeros(pad, np.float32)])
        yp = np.concatenate([y, np.zeros(pad, np.float32)])
        assert oracle.dist_f32(xp, yp) == oracle.dist_f32(x, y)
        assert oracle.dist_f32(x, x) == 0.0


def test_fp32_within_1e5_of_fp64():
    g = np.random.default_rng(9)
    for d in (32, 96, 128, 960):
        x = g.standard_normal((50, d)).astype(np.float32)
        y = g.standard_normal((50, d)).astype(np.float32)
        for a, b in zip(x, y):
            D32 = float(oracle.dist_f32(a, b))
            D64 = oracle.dist_f64(a, b)
            assert abs(np.sqrt(D32) - np.sqrt(D64)) <= 1e-5 * np.sqrt(D64)


def emulate_dot(x, y) -> Fraction:
    """The fixed-order dot product with exact rationals and explicit rounding."""
    acc = [Fraction(0)] * 32
    for i in range(len(x)):
        lane = (i // 4) % 32
        acc[lane] = round_f32(Fraction(float(x[i])) * Fraction(float(y[i])) + acc[lane])
    off = 16
    while off >= 1:
        acc = [round_f32(acc[l] + acc[l ^ off]) for l in range(32)]
        off //= 2
    return acc[0]


@pytest.mark.parametrize("d", [1, 4, 5, 33, 128, 129, 300])
def test_dot_matches_exact_rational_emulation(d):
    g = np.random.default_rng(100 + d)
    for trial in range(3):
        x = (g.standard_normal(d) * 10 ** g.uniform(-3, 3)).astype(np.float32)
        y = (g.standard_normal(d) * 10 ** g.uniform(-3, 3)).astype(np.float32)
        assert Fraction(float(oracle.dot_f32(x, y))) == emulate_dot(x, y)


def test_dot_order_hand_worked():
    """Elements 0 and 4 go to lanes 0 and 1: with x = (1, 0, 0, 0, 2^-24, ...)
    and y = x the lanes hold 1 and 2^-48 and the butterfly adds them once:
    1 + 2^-48 rounds to 1.  Elements 0 and 1 share lane 0: fma(2^-12, 2^-12, 1)
    also rounds to 1, exactly as a left-to-right sum would."""
    x = np.zeros(8, np.float32)
    x[0], x[4] = 1.0, 2.0 ** -24
    assert oracle.dot_f32(x, x) == np.float32(1.0)
    assert oracle.dot_f32(np.array([3.0, 0, 0, 0, 5.0], np.float32),
                          np.array([2.0, 0, 0, 0, -1.0], np.float32)) == np.float32(1.0)
