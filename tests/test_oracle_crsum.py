"""Pins of the oracle's correctly rounded reductions against exact rationals.

float(Fraction) rounds an exact rational to the nearest double (ties to even),
so a Fraction sum of exact products is the definition the C helper must meet.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import native


def exact_dot(x, y):
    return float(sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0)))


def _cases(rng):
    n = int(rng.integers(1, 200))
    x = rng.standard_normal(n) * np.exp2(rng.integers(-30, 30, n))
    y = rng.standard_normal(n) * np.exp2(rng.integers(-30, 30, n))
    yield x, y
    # heavy cancellation: append the negated partial products
    x2 = np.concatenate([x, x])
    y2 = np.concatenate([y, -y * (1 + 2.0 ** -40)])
    yield x2, y2
    # near ties: 1 + 2^-53 style sums
    t = np.array([1.0, 2.0 ** -53, 2.0 ** -106, -(2.0 ** -160)])
    yield t, np.ones_like(t)


def test_cr_dot_matches_exact_rounding():
    rng = np.random.default_rng(1)
    for _ in range(200):
        for x, y in _cases(rng):
            assert native.cr_dot(x, y) == exact_dot(x, y)


def test_cr_sum_half_even_ties():
    # 1 + 2^-53 is exactly half-way between 1 and 1+2^-52: ties to even -> 1
    assert native.cr_sum([1.0, 2.0 ** -53]) == 1.0
    # a hair above the tie must round up
    assert native.cr_sum([1.0, 2.0 ** -53, 2.0 ** -120]) == 1.0 + 2.0 ** -52
    # a hair below the tie must round down
    assert native.cr_sum([1.0 + 2.0 ** -52, 2.0 ** -53, -(2.0 ** -120)]) == 1.0 + 2.0 ** -52
    # order independence
    rng = np.random.default_rng(2)
    t = rng.standard_normal(500) * np.exp2(rng.integers(-60, 60, 500))
    ref = native.cr_sum(t)
    for _ in range(5):
        assert native.cr_sum(rng.permutation(t)) == ref
    assert native.cr_sum([]) == 0.0
    assert math.isinf(native.cr_sum([1.0, math.inf]))
    assert math.isnan(native.cr_sum([math.inf, -math.inf]))


def test_csr_rowsum_matches_exact():
    rng = np.random.default_rng(3)
    n = 50
    rowptr = [0]
    col = []
    for i in range(n):
        k = int(rng.integers(0, 9))
        col += sorted(rng.choice(n, size=k, replace=False).tolist())
        rowptr.append(len(col))
    rowptr = np.array(rowptr, dtype=np.int32)
    col = np.array(col, dtype=np.int32)
    val = rng.standard_normal(col.size)
    u = rng.standard_normal(n)
    w = rng.standard_normal(n)
    out = native.cr_csr_rowsum(rowptr, col, val, u, [(-0.75, u), (0.3, w)])
    for i in range(n):
        s = Fraction(0)
        for k in range(rowptr[i], rowptr[i + 1]):
            s += Fraction(val[k]) * Fraction(u[col[k]])
        s += Fraction(-0.75) * Fraction(u[i]) + Fraction(0.3) * Fraction(w[i])
        assert out[i] == float(s)


def test_rows_comb_and_gram_match_exact():
    rng = np.random.default_rng(4)
    n, d = 40, 7
    cols = [rng.standard_normal(n) * 10.0 ** rng.integers(-5, 5) for _ in range(d)]
    c = rng.standard_normal(d)
    base = rng.standard_normal(n)
    out = native.cr_rows_comb(cols, c, base)
    for i in range(n):
        s = Fraction(base[i]) + sum(Fraction(cols[a][i]) * Fraction(c[a]) for a in range(d))
        assert out[i] == float(s)
    G = native.cr_gram(cols)
    for a in range(d):
        for b in range(d):
            assert G[a, b] == exact_dot(cols[a], cols[b])
