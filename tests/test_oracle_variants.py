"""Pins of the oracle's method variants (CPU): the Newton basis and its Leja
shifts, and the theoretical c_{k,j} of Section 4.1.

* Newton basis in exact rational arithmetic: eq. AVVB holds exactly, and
  fixed s-step CG with it reproduces classical CG's alpha, beta and solution
  (Section 2: any polynomial basis gives the same iterates in exact arithmetic).
* Leja ordering against its definition by brute force.
* c_{k,j} = 6 N_k j kappa(A) with N_k = 7 + 2 N_A + 14 ||B_k|| / ||A|| on a hand
  example; the norm bound of B is 1 for the monomial basis (Section 4.1 says
  ||B|| = 1 there) and lambda_max for the Chebyshev basis.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import cg as ocg
from oracle import spectral, sstep
from oracle.arith import CR, Exact
from paper_1701_03989_amd import problems
from tests.test_oracle_exact import exact_solve, systems


SHIFTS = [Fraction(7, 2), Fraction(1, 3), Fraction(9, 4), Fraction(5, 1), Fraction(2, 7)]


def test_newton_B_satisfies_AY_underline_eq_YB_exactly():
    A, M, b = systems()[2]
    ar = Exact()
    n = len(b)
    rng = np.random.default_rng(3)
    p = ar.vec(rng.integers(-3, 4, n).astype(float))
    r = ar.vec(rng.integers(-3, 4, n).astype(float))
    for s in [1, 2, 3, 5]:
        for first in [True, False]:
            prm = sstep.basis_params("newton", s, ar=ar, shifts=SHIFTS)
            Y = sstep.krylov_basis(ar, A, p, r, s, first, prm)
            B = sstep.assemble_B(ar, s, first, prm)
            d = len(Y)
            last = {s} if first else {s, 2 * s}
            for j in range(d):
                lhs = ar.csr_comb(A, Y[j]) if j not in last else ar.zeros(n)
                rhs = ar.rows_comb(Y, [B[a][j] for a in range(d)])
                assert lhs == rhs, (s, first, j)


@pytest.mark.parametrize("case", range(5))
@pytest.mark.parametrize("s", [1, 2, 3, 4])
def test_newton_sstep_equals_classical_exactly(case, s):
    A, M, b = systems()[case]
    n = len(b)
    cl = ocg.cg(A, b, np.zeros(n), max_iters=n, ar=Exact(), keep_iterates=True)
    res = sstep.solve(A, b, np.zeros(n),
                      sstep.Opts(mode="fixed", fixed_s=s, basis="newton", shifts=SHIFTS,
                                 max_iters=n), ar=Exact())
    alphas, betas = [], []
    for blk in res.blocks:
        alphas += blk.alphas
        betas += blk.betas
    assert alphas == cl.alphas[: len(alphas)]
    assert betas == cl.betas[: len(betas)]
    assert res.x == exact_solve(M, b)


def brute_leja(pts):
    """Leja order by recomputing every candidate's product from scratch."""
    out = [max(range(len(pts)), key=lambda i: (abs(pts[i]), -i))]
    while len(out) < len(pts):
        best, bs = None, -1.0
        for i in range(len(pts)):
            if i in out:
                continue
            prod = 1.0
            for c in out:
                prod = prod * abs(pts[i] - pts[c])
            if prod > bs:
                best, bs = i, prod
        out.append(best)
    return [pts[i] for i in out]


@pytest.mark.parametrize("seed", range(6))
def test_leja_order_matches_definition(seed):
    rng = np.random.default_rng(seed)
    pts = sorted(rng.uniform(0.01, 10.0, size=3 + seed).tolist())
    got = spectral.leja_order(pts)
    assert got == brute_leja(pts)
    assert sorted(got) == pts and got[0] == max(pts, key=abs)
    # two points: the second is the other one; three: the farthest from the first
    assert spectral.leja_order([1.0, 4.0]) == [4.0, 1.0]
    assert spectral.leja_order([1.0, 2.0, 4.0]) == [4.0, 1.0, 2.0]


def test_newton_shifts_are_ritz_values_of_short_lanczos():
    A = problems.poisson2d(20)
    sh = spectral.newton_shifts(A, 6, 0)
    a, b = spectral.lanczos_tridiag(A, 6, 0)
    assert sorted(sh) == sorted(spectral.ritz_values(a, b).tolist())
    lo, hi = problems.poisson_interval(20, 2)
    assert all(lo - 1e-12 <= z <= hi + 1e-12 for z in sh)  # Ritz values lie in the spectrum


def test_theory_c_hand_example():
    # N_A = 5, ||B|| = 2, ||A|| = 8, kappa = 100, j = 3:
    # N_k = 7 + 10 + 14 * 0.25 = 20.5, c = 6 * 20.5 * 3 * 100 = 36900
    assert sstep.c_theory(3, 5, 2.0, 8.0, 100.0) == 36900.0
    assert sstep.c_theory(1, 0, 0.0, 1.0, 1.0) == 42.0


def test_b_norm_bound_monomial_and_chebyshev():
    for s in [2, 5, 8]:
        for first in [True, False]:
            B = sstep.assemble_B(CR(), s, first, sstep.basis_params("monomial", s, ar=CR()))
            assert sstep.b_norm_bound(B) == 1.0
    lmin, lmax = 0.5, 12.0
    for s in [3, 6]:
        B = sstep.assemble_B(CR(), s, False,
                             sstep.basis_params("chebyshev", s, lmin, lmax, ar=CR()))
        # columns: theta + gamma_0 = c0 + h, then h/2 + c0 + h/2: ||B||_1 = lambda_max;
        # row 1: gamma_0 + theta + sigma_1 = h + c0 + h/2 = lambda_max + h/2 = ||B||_inf
        h = (lmax - lmin) / 2
        assert sstep.b_norm_bound(B) == pytest.approx(np.sqrt(lmax * (lmax + h / 2)), rel=1e-15)


def test_theory_c_gives_smaller_steps_than_c_one():
    """Section 4.2: the bound's c_{k,j} overestimates the error, so it picks
    s_k no larger than c = 1 does (same problem, same basis)."""
    A, b, x1, _ = problems.poisson2d_32_system(0)
    lo, hi = problems.poisson_interval(32, 2)
    base = dict(mode="adaptive", basis="chebyshev", lmin=lo, lmax=hi, s_max=8, tol=1e-10)
    r1 = sstep.solve(A, b, x1, sstep.Opts(**base))
    rt = sstep.solve(A, b, x1, sstep.Opts(c_mode="theory", kappa_a=hi / lo, norm_a=hi, **base))
    assert rt.status == sstep.OK and r1.status == sstep.OK
    assert sum(rt.schedule) >= sum(r1.schedule) - 8
    assert max(rt.schedule[:3]) < max(r1.schedule[:3])
    assert len(rt.blocks) > len(r1.blocks)
