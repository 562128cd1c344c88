"""Pins of the variable-precision blocks of the oracle (reading R17 of
oracle/sstep.py; Section 6's closing remark rearranges eq. fb into a bound on
the unit round-off an outer loop may use).

What is pinned, each against something other than the oracle's own code:
  * the rule's comparison (accept on equality, previous block's gamma and
    updated residual, 2^-24, NaN -> FP64) on hand-built values;
  * an FP32 block's basis columns against exact rational evaluation of the
    three-term step from the stored FP32 columns (one FP64 rounding of the
    numerator, one of the division, one FP32 rounding);
  * the block decisions of whole solves against the rule recomputed in exact
    rationals from the logged gamma and updated residual of the block before;
  * eqs. condy thresholds with 2^-24 in FP32 blocks and 2^-53 in FP64 ones;
  * a solve whose rule never admits FP32 is the FP64 solve, bit for bit;
  * solves with FP32 blocks reach the tolerance on A x = b (true residual
    recomputed exactly in rationals) in about the FP64 solve's iterations.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import sstep
from paper_1701_03989_amd.problems import graph_laplacian, poisson2d


def rn64(q: Fraction) -> Fraction:
    return Fraction(float(q))  # float(Fraction) rounds to nearest, ties to even


def rn32(q: Fraction) -> Fraction:
    return Fraction(float(np.float32(float(q))))  # q is already a double here


def cheb_interval(N: int):
    h = 1.0 / (N + 1)
    return 8 * math.sin(math.pi * h / 2) ** 2, 8 * math.cos(math.pi * h / 2) ** 2


def test_rule_accepts_on_equality_and_uses_fp32_unit_roundoff():
    eps32 = 2.0 ** -24
    gam, rr = 3.0, 16.0  # ((2^-24 * 1) * 3) * 4 = 12 * 2^-24 exactly
    lhs = 12.0 * eps32
    assert sstep.fp32_block_allowed(1.0, gam, rr, lhs)
    assert not sstep.fp32_block_allowed(1.0, gam, rr, np.nextafter(lhs, 0.0))
    # with 2^-53 the same numbers would pass far below: the rule must not
    assert not sstep.fp32_block_allowed(1.0, gam, rr, 12.0 * 2.0 ** -53)
    # c multiplies the left-hand side
    assert not sstep.fp32_block_allowed(2.0, gam, rr, lhs)
    assert sstep.fp32_block_allowed(2.0, gam, rr, 2 * lhs)
    # a negative quadratic form is clamped at 0; NaN (no estimate) keeps FP64
    assert sstep.fp32_block_allowed(1.0, gam, -1.0, 0.0)
    assert not sstep.fp32_block_allowed(1.0, math.nan, rr, 1.0)
    assert not sstep.fp32_block_allowed(1.0, gam, math.nan, 1.0)
    assert not sstep.fp32_block_allowed(1.0, math.inf, rr, 1.0)


@pytest.mark.parametrize("basis", ["monomial", "chebyshev"])
@pytest.mark.parametrize("first", [True, False])
def test_fp32_block_columns_match_exact_evaluation(basis, first):
    A = poisson2d(7) if basis == "chebyshev" else graph_laplacian(60, 3)
    n = A.n
    rng = np.random.default_rng(11)
    p = rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 3, n)
    r = rng.standard_normal(n)
    lmin, lmax = cheb_interval(7) if basis == "chebyshev" else (None, None)
    s = 4
    ar = sstep.CR()
    prm = sstep.basis_params(basis, s, lmin, lmax, ar)
    cols = sstep.krylov_basis(ar, A, p, r, s, first, prm, fp32=True)
    theta, gamma, sigma = prm

    def seq(v0, count):
        out = [rn32(Fraction(float(x))) for x in v0]
        seq_ = [out]
        for j in range(1, count + 1):
            u = seq_[j - 1]
            w = seq_[j - 2] if j >= 2 else None
            new = []
            for i in range(n):
                acc = Fraction(0)
                for k in range(int(A.rowptr[i]), int(A.rowptr[i + 1])):
                    acc += Fraction(float(A.val[k])) * u[int(A.col[k])]
                acc -= Fraction(theta[j - 1]) * u[i]
                if j >= 2:
                    acc -= Fraction(sigma[j - 2]) * w[i]
                q = rn64(rn64(acc) / Fraction(gamma[j - 1]))
                new.append(rn32(q))
            seq_.append(new)
        return seq_

    want = seq(p, s)
    if not first:
        want += seq(r, s - 1)
    assert len(cols) == len(want)
    for a, (got, ref) in enumerate(zip(cols, want)):
        assert np.all(got.astype(np.float32).astype(np.float64) == got)  # FP32 values
        assert [Fraction(float(x)) for x in got] == ref, a


def _solve(A, b, **kw):
    return sstep.solve(A, b, np.zeros(A.n), sstep.Opts(**kw))


def _cheb_case(N=32, tol=1e-10):
    A = poisson2d(N)
    rng = np.random.default_rng(0)
    b = A.matvec(rng.uniform(-1, 1, A.n))
    lmin, lmax = cheb_interval(N)
    return A, b, dict(mode="adaptive", basis="chebyshev", s_max=8, tol=tol, lmin=lmin, lmax=lmax)


def test_block_decisions_follow_the_rule_from_the_previous_block():
    A, b, kw = _cheb_case()
    res = _solve(A, b, precision="variable", **kw)
    flags = [blk.fp32 for blk in res.blocks]
    assert flags[0] is False and any(flags), flags  # block 0 FP64; FP32 blocks occur
    eps_star = Fraction(kw["tol"]) * Fraction(float(np.sqrt(sstep.CR().dot(b, b))))
    for prev, blk in zip(res.blocks, res.blocks[1:]):
        # ((2^-24 c) gamma) ||r^|| in exact rationals, rounded as the rule rounds
        lhs = rn64(rn64(Fraction(1, 2 ** 24) * Fraction(prev.gamma)) * Fraction(prev.res_updated))
        assert blk.fp32 == (lhs <= Fraction(float(eps_star))), blk.k
    for blk in res.blocks:
        eps = 2.0 ** -24 if blk.fp32 else 2.0 ** -53
        thr = float(rn64(Fraction(float(eps_star)) / rn64(Fraction(eps) * Fraction(blk.rnorm))))
        assert blk.thr == thr, blk.k


def test_no_fp32_block_means_the_fp64_solve():
    # the monomial basis of this system is far too ill-conditioned for the rule
    A = poisson2d(32)
    rng = np.random.default_rng(0)
    b = A.matvec(rng.uniform(-1, 1, A.n))
    kw = dict(mode="adaptive", basis="monomial", s_max=8, tol=1e-10)
    v = _solve(A, b, precision="variable", **kw)
    f = _solve(A, b, **kw)
    assert not any(blk.fp32 for blk in v.blocks)
    assert np.array_equal(v.x, f.x)
    assert [blk.s_k for blk in v.blocks] == [blk.s_k for blk in f.blocks]


@pytest.mark.parametrize("tol", [1e-6, 1e-10, 1e-12])
def test_variable_precision_reaches_the_tolerance_on_ax_eq_b(tol):
    A, b, kw = _cheb_case(tol=tol)
    v = _solve(A, b, precision="variable", **kw)
    f = _solve(A, b, **kw)
    assert v.status == sstep.OK
    # true residual of the returned x, exactly in rationals
    num = Fraction(0)
    for i in range(A.n):
        acc = Fraction(float(b[i]))
        for k in range(int(A.rowptr[i]), int(A.rowptr[i + 1])):
            acc -= Fraction(float(A.val[k])) * Fraction(float(v.x[int(A.col[k])]))
        num += acc * acc
    den = sum(Fraction(float(x)) ** 2 for x in b)
    assert num <= Fraction(tol) ** 2 * den
    # FP32 blocks do not cost iterations here (at most one more block of s_max)
    assert v.iters <= f.iters + kw["s_max"]
    n32 = sum(blk.fp32 for blk in v.blocks)
    print(f"tol {tol:g}: {n32} of {len(v.blocks)} blocks FP32; iterations {v.iters} vs {f.iters}")


def test_variable_precision_options_are_checked():
    A, b, kw = _cheb_case()
    with pytest.raises(ValueError):
        _solve(A, b, precision="variable", **dict(kw, mode="fixed", fixed_s=4))
    with pytest.raises(ValueError):
        _solve(A, b, precision="half", **kw)
