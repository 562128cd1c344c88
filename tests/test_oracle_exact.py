"""Exact-arithmetic pins of the oracle's Algorithms 1-3.

Section 2: in exact arithmetic s-step CG produces the same iterates as
classical CG (the coordinates of eq. coords represent the CG vectors exactly,
and alpha, beta computed from G and B equal the classical ones).  CG itself
terminates with the exact solution after at most n steps.  Running the oracle's
own code on Fractions turns both facts into equalities: a dropped term, a sign
or index slip in B, a transposed operand or a wrong coordinate start breaks
them.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import cg as ocg
from oracle import sstep
from oracle.arith import Exact
from paper_1701_03989_amd.problems import from_dense, poisson2d, random_spd_integer


def exact_solve(M, b):
    """Gaussian elimination over the rationals."""
    n = len(b)
    A = [[Fraction(M[i][j]) for j in range(n)] + [Fraction(b[i])] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [a - f * e for a, e in zip(A[r], A[c])]
    return [A[i][n] / A[i][i] for i in range(n)]


def systems():
    out = []
    for seed in range(4):
        n = 5 + seed
        M = random_spd_integer(n, seed)
        rng = np.random.default_rng(100 + seed)
        b = rng.integers(-5, 6, n).astype(float)
        if not b.any():
            b[0] = 1.0
        out.append((from_dense(M), M, b))
    A = poisson2d(3)
    M = A.to_scipy().toarray()
    out.append((A, M, np.arange(1.0, 10.0)))
    return out


@pytest.mark.parametrize("case", range(5))
def test_classical_cg_terminates_with_exact_solution(case):
    A, M, b = systems()[case]
    n = len(b)
    r = ocg.cg(A, b, np.zeros(n), max_iters=n, ar=Exact())
    assert r.status == sstep.OK and r.iters <= n
    assert r.x == exact_solve(M, b)


def _classical_iterates(A, b):
    n = len(b)
    r = ocg.cg(A, b, np.zeros(n), max_iters=n, ar=Exact(), keep_iterates=True)
    return r


def _run(A, b, opts):
    n = len(b)
    opts.max_iters = n
    return sstep.solve(A, b, np.zeros(n), opts, ar=Exact())


@pytest.mark.parametrize("case", range(5))
@pytest.mark.parametrize("s", [1, 2, 3, 4])
@pytest.mark.parametrize("basis", ["monomial", "chebyshev"])
def test_fixed_sstep_equals_classical_exactly(case, s, basis):
    A, M, b = systems()[case]
    cl = _classical_iterates(A, b)
    kw = {}
    if basis == "chebyshev":
        kw = dict(lmin=Fraction(1, 3), lmax=Fraction(int(np.abs(M).sum(1).max())))
    res = _run(A, b, sstep.Opts(mode="fixed", fixed_s=s, basis=basis, **kw))
    m = 0
    alphas, betas = [], []
    for blk in res.blocks:
        m += blk.s_k
        alphas += blk.alphas
        betas += blk.betas
    assert alphas == cl.alphas[: len(alphas)]
    assert betas == cl.betas[: len(betas)]
    assert res.x == exact_solve(M, b)


@pytest.mark.parametrize("case", range(5))
def test_block_boundaries_match_classical_iterates(case):
    """x after every block of Alg. 2/3 equals classical x_{m+1}."""
    A, M, b = systems()[case]
    cl = _classical_iterates(A, b)
    rng = np.random.default_rng(case)
    for trial in range(3):
        sched = rng.integers(1, 5, size=len(b)).tolist()
        n = len(b)
        # replay block by block to read x at each boundary
        for nb in range(1, 4):
            opts = sstep.Opts(mode="schedule", schedule=sched[:nb] + [sched[nb - 1]])
            opts.max_iters = sum(sched[:nb])
            res = sstep.solve(A, b, np.zeros(n), opts, ar=Exact())
            m = res.iters
            if m == 0 or m > cl.iters:
                continue
            if res.status == sstep.OK and m <= cl.iters:
                assert res.x == exact_solve(M, b)
            else:
                assert res.x == cl.xs[m - 1]


def test_B_satisfies_AY_underline_eq_YB_exactly():
    """eq. AVVB holds exactly in rationals for both bases and both block types."""
    A, M, b = systems()[1]
    ar = Exact()
    n = len(b)
    rng = np.random.default_rng(7)
    p = ar.vec(rng.integers(-3, 4, n).astype(float))
    r = ar.vec(rng.integers(-3, 4, n).astype(float))
    for basis, kw in [("monomial", {}), ("chebyshev", dict(lmin=Fraction(1, 2), lmax=Fraction(20)))]:
        for s in [1, 2, 3, 5]:
            for first in [True, False]:
                prm = sstep.basis_params(basis, s, ar=ar, **kw)
                Y = sstep.krylov_basis(ar, A, p, r, s, first, prm)
                B = sstep.assemble_B(ar, s, first, prm)
                d = len(Y)
                last = {s} if first else {s, 2 * s}
                for j in range(d):
                    lhs = ar.csr_comb(A, Y[j]) if j not in last else ar.zeros(n)
                    rhs = ar.rows_comb(Y, [B[a][j] for a in range(d)])
                    assert lhs == rhs, (basis, s, first, j)
