"""Pins of the s_k rule of Algorithm 4 that do not come from the oracle itself:
the in-loop break of eq. check, the block-start rule eq. condy at its
boundaries, and the basis growth limit s_bar_k = min(s_{k-1} + f, s_max).

The expected values are derived by hand (or with exact rational CG and a
LAPACK eigensolver written out here), not by calling the oracle's own rule."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import sstep
from paper_1701_03989_amd.problems import from_dense, graph_laplacian, poisson2d_32_system, uniform

EPS = 2.0 ** -53

# ---------------------------------------------------------------- boundaries


def test_condy_accepts_on_equality_and_check_breaks_on_equality():
    """Section 4.2: eq. condy asks sqrt(kappa) <= threshold (so equality is
    accepted) and eq. check breaks once gamma >= the right-hand side (so
    equality breaks).  Values chosen so that every operation is exact."""
    # sqrt(9) = 3 exactly: accepted at threshold 3, rejected one ulp below it
    assert sstep.condy_accepts(9.0, 3.0)
    assert not sstep.condy_accepts(9.0, math.nextafter(3.0, 0.0))
    assert sstep.condy_accepts(9.0, math.nextafter(3.0, math.inf))
    assert not sstep.condy_accepts(math.inf, 1e300)

    # rhs = eps* / (c eps sqrt(rr1)) = 2^-10 / (2^-53 * 2) = 2^42
    eps_star, c, rr1 = 2.0 ** -10, 1.0, 4.0
    rhs = 2.0 ** 42
    assert sstep.check_breaks(rhs, eps_star, c, rr1)
    assert not sstep.check_breaks(math.nextafter(rhs, 0.0), eps_star, c, rr1)
    # c_{k,j} enters the denominator: doubling c halves the right-hand side
    assert sstep.check_breaks(rhs / 2, eps_star, 2.0, rr1)
    assert not sstep.check_breaks(math.nextafter(rhs / 2, 0.0), eps_star, 2.0, rr1)
    # a quadratic form that came out negative is clamped to 0: rhs = inf, no break
    assert not sstep.check_breaks(1e300, eps_star, c, -1e-30)


# ---------------------------------------------------------------- hand case

# A = diag(1, 10, 100), b = (10, 1, 1), x_1 = 0.  Classical CG's first step
# makes the residual grow, ||r_2|| / ||r_1|| = 4.75: the situation in which
# eq. check can stop a block short of s~ (CG residuals are not monotone).
DIAG = (1, 10, 100)
RHS = (10, 1, 1)


def _exact_cg_residual_norms2(steps):
    """||r_i||^2, i = 1..steps+1, of Algorithm 1 in rational arithmetic."""
    r = [Fraction(v) for v in RHS]
    p = list(r)
    out = [sum(v * v for v in r)]
    for _ in range(steps):
        Ap = [a * v for a, v in zip(DIAG, p)]
        rr = sum(v * v for v in r)
        alpha = rr / sum(u * v for u, v in zip(p, Ap))
        r = [ri - alpha * w for ri, w in zip(r, Ap)]
        rr1 = sum(v * v for v in r)
        p = [ri + (rr1 / rr) * pi for ri, pi in zip(r, p)]
        out.append(rr1)
    return out


def _block0_gamma():
    """sqrt(kappa) of the 3 x 3 Gram matrix of [b, A b, A^2 b] (block 0, s~ = 2),
    from its exact entries and LAPACK's eigenvalues."""
    K = [[Fraction(b) * Fraction(a) ** j for j in range(3)] for a, b in zip(DIAG, RHS)]
    G = np.array([[float(sum(K[i][u] * K[i][v] for i in range(3))) for v in range(3)]
                  for u in range(3)])
    ev = np.linalg.eigvalsh(G)
    ev1 = np.linalg.eigvalsh(G[:2, :2])
    return math.sqrt(ev[-1] / ev[0]), math.sqrt(ev1[-1] / ev1[0])


def _system():
    return from_dense(np.diag(np.array(DIAG, dtype=np.float64))), np.array(RHS, float), np.zeros(3)


def test_check_breaks_after_a_residual_growth_constant_c():
    """c = 1, s_max = 2, tol = 5e-13.  By hand: thr = tol / (c eps) = 4503.6
    (x_1 = 0, so eps* = tol ||r_1||); gamma = sqrt(kappa(G_2)) = 1990.6 <= thr,
    so eq. condy takes s~ = 2.  After iteration 1, ||r_2|| = 4.75 ||r_1||, so
    eps* / (c eps ||r_2||) = thr / 4.75 = 947.5 <= gamma: eq. check breaks and
    s_0 = 1.  Testing the residual before the update (||r_1||, rhs = thr)
    would not break."""
    A, b, x1 = _system()
    tol = 5e-13
    rn2 = _exact_cg_residual_norms2(2)
    growth = math.sqrt(rn2[1] / rn2[0])
    gam, gam1 = _block0_gamma()
    thr = tol / EPS
    assert growth == pytest.approx(4.753087, rel=1e-6)
    assert gam1 <= gam <= thr  # condy accepts i = 1, 2
    assert gam >= thr / growth  # the check fires after iteration 1 ...
    assert gam < thr  # ... but would not on the pre-update residual

    res = sstep.solve(A, b, x1, sstep.Opts(mode="adaptive", s_max=2, tol=tol, c=1.0))
    blk = res.blocks[0]
    assert blk.thr == pytest.approx(thr, rel=1e-15)
    assert blk.gamma == pytest.approx(gam, rel=1e-9)
    assert blk.s_tilde == 2
    assert blk.s_k == 1
    assert blk.rr_trace[0] == pytest.approx(float(rn2[1]), rel=1e-12)
    assert res.status == sstep.OK

    # with the check switched off the same block takes both steps
    res_nc = sstep.solve(A, b, x1, sstep.Opts(mode="adaptive", s_max=2, tol=tol, c=1.0,
                                              inner_check=False))
    assert res_nc.blocks[0].s_k == 2


def test_check_uses_c_kj_of_the_step_theory_c():
    """Theoretical c_{k,j} = 6 N_k j kappa(A), N_k = 7 + 2 N_A + 14 ||B|| / ||A||
    (Section 4.1) with N_A = 1 (diagonal), ||B|| bound 1 (monomial), ||A|| = 100,
    kappa(A) = 100: N_k = 9.14, c_{k,j} = 5484 j.  eq. condy uses c_{k,s_max}
    (s_max = 4): thr = tol / (21936 eps); s0_bar = 2 and gamma <= thr give
    s~ = 2.  eq. check at j = 1 uses c_{k,1}: its right-hand side is
    4 thr / 4.75 > gamma, so no break and s_0 = 2.  With c_{k,s_max} in the
    check instead it would be thr / 4.75 < gamma and s_0 would be 1."""
    A, b, x1 = _system()
    tol = 1e-8
    nk = 7 + 2 * 1 + 14 * (1.0 / 100.0)
    c = [6 * nk * j * 100.0 for j in range(5)]
    assert c[1] == pytest.approx(5484.0) and c[4] == pytest.approx(21936.0)
    rn2 = _exact_cg_residual_norms2(2)
    growth = math.sqrt(rn2[1] / rn2[0])
    gam, _ = _block0_gamma()
    thr = tol / (c[4] * EPS)
    rhs_j1 = tol / (c[1] * EPS * growth)  # eps* / (c_{k,1} eps ||r_2||), ||r_1|| = ||b||
    rhs_wrong = tol / (c[4] * EPS * growth)
    assert gam <= thr
    assert gam < rhs_j1  # correct reading: no break after iteration 1
    assert gam >= rhs_wrong  # c_{k,s_max} in the check would break

    res = sstep.solve(A, b, x1, sstep.Opts(mode="adaptive", s_max=4, s0_bar=2, tol=tol,
                                           c_mode="theory", kappa_a=100.0, norm_a=100.0))
    blk = res.blocks[0]
    assert blk.thr == pytest.approx(thr, rel=1e-14)
    assert blk.s_bar == 2 and blk.s_tilde == 2
    assert blk.s_k == 2
    assert blk.rr_trace[0] == pytest.approx(float(rn2[1]), rel=1e-12)


# ---------------------------------------------------------------- replay


def _poisson32():
    A, b, x1, _ = poisson2d_32_system(0)
    return A, b, x1


def _graph400():
    A = graph_laplacian(400, 0)
    return A, uniform(A.n, 0), np.zeros(A.n)


def _logdiag30():
    d = np.logspace(0.0, 4.0, 30)
    return from_dense(np.diag(d)), np.random.default_rng(0).uniform(-1, 1, 30), np.zeros(30)


@pytest.mark.parametrize("system,kw,fires", [
    (_poisson32, dict(s_max=8, tol=1e-10), False),  # the 32 x 32 workload as stated
    (_poisson32, dict(s_max=8, tol=1e-10, equilibrate=True), False),
    (_graph400, dict(s_max=10, tol=1e-12, c=10.0), True),
    (_logdiag30, dict(s_max=8, tol=1e-10), True),
])
def test_inner_check_replayed_from_materialised_residuals(system, kw, fires):
    """Every block of an adaptive solve: s_k is the first inner iteration j at
    which gamma >= eps* / (c eps ||r^_{m+j+1}||) (eq. check, with the
    residual after iteration j), or s~ if there is none.  ||r^||^2 is taken
    from the materialised residual vector Y r' (numpy), not from the oracle's
    quadratic form; blocks whose margin is within 1e-6 are skipped as ties."""
    A, b, x1 = system()
    opts = sstep.Opts(mode="adaptive", **kw)
    diag = []
    res = sstep.solve(A, b, x1, opts, diag=diag)
    assert res.status == sstep.OK
    bvec = b * sstep.equilibrate(A)[1] if opts.equilibrate else b
    eps_star = opts.tol * np.linalg.norm(bvec)
    c = opts.c
    fired = 0
    for blk in res.blocks:
        steps = [d for d in diag if d["k"] == blk.k]
        assert len(steps) == blk.s_k
        expect = blk.s_tilde
        tie = False
        for d in steps:
            rn = float(np.linalg.norm(d["r"]))
            # the oracle's quadratic form is the same quantity (eq. coords), up
            # to the rounding of G and of the materialised vector:
            # |r'^T G r' - ||Y r'||^2| <= (2d + 4) eps || |Y| |r'| ||^2
            Y = np.stack(d["Y"], 1)
            mag = float(np.linalg.norm(np.abs(Y) @ np.abs(np.asarray(d["rc"], float)))) ** 2
            bound = (2 * Y.shape[1] + 4) * EPS * mag
            assert abs(blk.rr_trace[d["j"] - 1] - rn * rn) <= bound
            rhs = eps_star / (c * EPS * rn)
            if abs(blk.gamma - rhs) <= 1e-6 * rhs:
                tie = True
            if blk.gamma >= rhs:
                expect = d["j"]
                break
        if not tie:
            assert blk.s_k == expect, (blk.k, blk.s_k, expect)
        fired += blk.s_k < blk.s_tilde
    assert (fired > 0) == fires


# ---------------------------------------------------------------- growth limit


@pytest.mark.parametrize("f,s_bar,s_k", [
    # Algorithm 4: s_bar_0 = 2, s_bar_k = min(s_{k-1} + f, 6); the rank guard
    # builds min(s_bar_k, m) steps for k >= 1 (m = iterations so far), and with
    # every basis accepted s_k = that.  Written out by hand:
    #   f = 1: m = 0 -> s 2 (m 2) -> s_bar 3, s 2 (m 4) -> 3, 3 (7) -> 4, 4 (11)
    #          -> 5, 5 (16) -> 6, 6 ...
    (1, [2, 3, 3, 4, 5, 6, 6, 6], [2, 2, 3, 4, 5, 6, 6, 6]),
    #   f = 2: 2 (m 2) -> s_bar 4, s 2 (m 4) -> 4, 4 (8) -> 6, 6 ...
    (2, [2, 4, 4, 6, 6, 6, 6, 6], [2, 2, 4, 6, 6, 6, 6, 6]),
])
def test_growth_limit_sequences_by_hand(f, s_bar, s_k):
    """c = 1e-30 makes the threshold of eqs. condy and check astronomically
    large, so every finite kappa is accepted and no check fires: the schedule
    is then a function of the growth limit and the rank guard only."""
    A, b, x1, _ = poisson2d_32_system(0)
    res = sstep.solve(A, b, x1, sstep.Opts(mode="adaptive", s_max=6, s0_bar=2, f=f, c=1e-30,
                                           tol=1e-10, equilibrate=True, max_iters=40))
    got = res.blocks[:len(s_bar)]
    assert [blk.s_bar for blk in got] == s_bar
    assert [blk.s_k for blk in got] == s_k
    assert all(blk.s_tilde == blk.s_built for blk in got)


def test_growth_limit_with_default_c_converges():
    """The same growth limits with c = 1 (Section 5's default): the schedule
    still follows s_bar_k = min(s_{k-1} + f, s_max) block by block, and the
    solve reaches its tolerance."""
    A, b, x1, _ = poisson2d_32_system(0)
    for f in (1, 2, 3):
        res = sstep.solve(A, b, x1, sstep.Opts(mode="adaptive", s_max=6, s0_bar=2, f=f,
                                               tol=1e-10, equilibrate=True))
        assert res.status == sstep.OK
        prev = None
        for blk in res.blocks:
            want = 2 if prev is None else min(prev + f, 6)
            assert blk.s_bar == want
            prev = blk.s_k
