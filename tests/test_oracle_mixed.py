"""Pins of the FP32 stages of the mixed-precision oracle (oracle/mixed.py)
against exact rational arithmetic: the FP32 matrix-powers entry is one FP32
rounding of the FP64 value its definition computes (products exact, FP64
additions in CSR order, the three-term correction and the division each one
FP64 rounding), and gram32 is the Gram of the widened FP32 columns in the
stated order of the FP64 Gram."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import mixed
from paper_1701_03989_amd.problems import CSR, graph_laplacian, poisson2d


def rn64(q: Fraction) -> Fraction:
    """Round a rational to the nearest double (Python's float(Fraction) is
    correctly rounded, ties to even)."""
    return Fraction(float(q))


def rn32(q: Fraction) -> np.float32:
    """Round a double-valued rational to FP32 (IEEE, ties to even)."""
    return np.float32(float(q))


def entry_by_definition(A, a32, u, w, i, j, basis, lmin=None, lmax=None):
    """Row i of pass j, evaluated step by step in rationals with an explicit
    rounding after every FP64 operation."""
    acc = Fraction(0)
    for k in range(int(A.rowptr[i]), int(A.rowptr[i + 1])):
        prod = Fraction(float(a32[k])) * Fraction(float(u[int(A.col[k])]))
        acc = rn64(acc + prod)  # exact product, one FP64 rounding per addition
    if basis == "monomial":
        return rn32(acc)
    c0 = rn64((Fraction(lmax) + Fraction(lmin)) / 2)
    h = rn64((Fraction(lmax) - Fraction(lmin)) / 2)
    h2 = rn64(h / 2)
    num = rn64(acc - rn64(c0 * Fraction(float(u[i]))))
    if j >= 2:
        num = rn64(num - rn64(h2 * Fraction(float(w[i]))))
    return rn32(rn64(num / (h if j == 1 else h2)))


@pytest.mark.parametrize("basis", ["monomial", "chebyshev"])
@pytest.mark.parametrize("kind", ["poisson", "graph"])
def test_mpk32_step_matches_rational_evaluation(basis, kind):
    A = poisson2d(9) if kind == "poisson" else graph_laplacian(150, 4)
    rng = np.random.default_rng(3)
    a32 = mixed.to_f32(A.val)
    u = (rng.standard_normal(A.n) * 10.0 ** rng.uniform(-2, 2, A.n)).astype(np.float32)
    w = rng.standard_normal(A.n).astype(np.float32)
    lmin, lmax = (0.05, 8.0) if kind == "poisson" else (0.01, 25.0)
    for j in (1, 2, 3):
        got = mixed.mpk32_step(A, a32, u, w, j, basis, lmin, lmax)
        for i in range(A.n):
            want = entry_by_definition(A, a32, u, w, i, j, basis, lmin, lmax)
            assert got[i] == want, (j, i, got[i], want)


def test_mpk32_sums_in_csr_order():
    """A row whose FP64 sum depends on the order of its terms: 1 + 2^-60 - 1
    is 0 in CSR order (the small term is lost) but 2^-60 the other way round."""
    big, tiny = np.float32(1.0), np.float32(2.0 ** -60)
    rowptr = np.array([0, 3, 4, 5, 6], dtype=np.int32)
    col = np.array([1, 2, 3, 1, 2, 3], dtype=np.int32)
    val = np.array([1.0, 1.0, -1.0, 1.0, 1.0, 1.0])
    A = CSR(rowptr, col, val)
    u = np.array([0.0, big, tiny, big], dtype=np.float32)
    out = mixed.mpk32_step(A, mixed.to_f32(A.val), u, None, 1, "monomial")
    assert out[0] == 0.0
    A2 = CSR(rowptr, np.array([1, 3, 2, 1, 2, 3], dtype=np.int32), val[[0, 2, 1, 3, 4, 5]])
    out2 = mixed.mpk32_step(A2, mixed.to_f32(A2.val), u, None, 1, "monomial")
    assert out2[0] == np.float32(2.0 ** -60)


def test_mpk32_basis_rounds_matrix_values_to_fp32():
    """The matrix values enter as FP32: a value 1 + 2^-30 acts as 1."""
    A = CSR(np.array([0, 1], dtype=np.int32), np.array([0], dtype=np.int32),
            np.array([1.0 + 2.0 ** -30]))
    P, R = mixed.mpk32_basis(A, 2, True, "monomial", np.array([3.0]), None)
    assert P[1][0] == np.float32(3.0) and P[2][0] == np.float32(3.0) and R == []


def test_gram32_is_the_stated_order_gram_of_widened_fp32_columns():
    from tests.test_oracle_fp64 import _gram_by_definition

    rng = np.random.default_rng(9)
    n, d = 1300, 4
    cols = [(rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 3)).astype(np.float32)
            for _ in range(d)]
    cols[3] = (cols[0] * np.float32(1.0 + 2.0 ** -20)).astype(np.float32)  # cancellation
    G = mixed.gram32(cols)
    Y = np.stack([c.astype(np.float64) for c in cols], 1)
    assert np.array_equal(G, _gram_by_definition(Y))
    tol = mixed.gram32_tolerance(cols)
    for a in range(d):
        for b in range(d):
            exact = sum((Fraction(float(x)) * Fraction(float(y)) for x, y in zip(cols[a], cols[b])),
                        Fraction(0))
            assert abs(G[a, b] - float(exact)) <= tol[a, b]
    assert np.all(tol >= 0) and np.all(np.diag(tol) > 0)
    # any FP64 summation order of the exact products stays within the tolerance
    perm = rng.permutation(n)
    plain = Y[perm].T @ Y[perm]
    assert np.all(np.abs(plain - G) <= 2 * tol)
