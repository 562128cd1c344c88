"""FP64 pins of the oracle: closed forms, library cross-checks, the paper's
error bounds and the structure of the s_k rule."""
import math

import numpy as np
import pytest

from oracle import cg as ocg
from oracle import kappa as okappa
from oracle import native, spectral, sstep
from oracle.arith import CR
from paper_1701_03989_amd.problems import (from_dense, poisson2d, poisson2d_32_system, poisson3d,
                                           random_spd_integer, uniform)

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    for ln in open(f"{GOLDEN}/{name}"):
        if ln.strip() and not ln.startswith("#"):
            rows.append(ln.split())
    return rows


# ---------------------------------------------------------------- Jacobi

def test_jacobi_matches_lapack_on_random_spd():
    rng = np.random.default_rng(0)
    for k in [2, 3, 5, 8, 13, 17, 21, 33]:
        X = rng.standard_normal((3 * k, k))
        G = X.T @ X
        ev, sweeps = okappa.jacobi_eigenvalues(G)
        ref = np.linalg.eigvalsh(G)
        assert np.allclose(np.sort(ev), ref, rtol=1e-12, atol=1e-12 * ref.max())
        assert sweeps < okappa.MAX_SWEEPS


def test_jacobi_relative_accuracy_on_graded_gram():
    """Columns of very different norms (like an unnormalised Krylov basis):
    every eigenvalue, the smallest included, must be accurate relative to
    itself.  Reference: the eigenvalues of the same matrix in 50-digit
    arithmetic (mpmath)."""
    import mpmath

    rng = np.random.default_rng(1)
    k = 9
    X = rng.standard_normal((50, k)) * np.exp2(np.arange(k) * 4.0)
    G = X.T @ X
    ev, _ = okappa.jacobi_eigenvalues(G)
    with mpmath.workdps(50):
        ref = mpmath.eigsy(mpmath.matrix(G.tolist()), eigvals_only=True)
        ref = np.sort(np.array([float(v) for v in ref]))
    assert np.allclose(np.sort(ev), ref, rtol=1e-13)
    # LAPACK's eigensolver is not scaling invariant: its smallest eigenvalue
    # is far less accurate here, which is why the oracle uses Jacobi
    lap = np.linalg.eigvalsh(G)
    assert abs(lap[0] - ref[0]) / ref[0] > 1e3 * abs(np.sort(ev)[0] - ref[0]) / ref[0]


def test_jacobi_two_by_two_closed_form_and_diagonal():
    a, b, c = 3.0, 1.25, -0.5
    ev, _ = okappa.jacobi_eigenvalues([[a, c], [c, b]])
    mid, rad = (a + b) / 2, math.hypot((a - b) / 2, c)
    assert np.allclose(np.sort(ev), [mid - rad, mid + rad], rtol=1e-15)
    D = np.diag([5.0, 1.0, 3.0])
    ev, sweeps = okappa.jacobi_eigenvalues(D)
    assert list(ev) == [5.0, 1.0, 3.0] and sweeps == 1
    assert okappa.kappa_spd(D) == 5.0
    assert okappa.kappa_spd([[1.0, 2.0], [2.0, 1.0]]) == math.inf  # indefinite


def test_round_robin_covers_every_pair_once_per_sweep():
    for k in [2, 3, 6, 7, 21]:
        m = k if k % 2 == 0 else k + 1
        seen = []
        for t in range(m - 1):
            pr = okappa.round_robin_pairs(k, t)
            flat = [i for p in pr for i in p]
            assert len(flat) == len(set(flat))
            seen += pr
        assert sorted(seen) == [(p, q) for p in range(k) for q in range(p + 1, k)]


# ---------------------------------------------------------------- spectral

def test_splitmix64_published_vectors():
    ref = [int(r[0], 16) for r in _golden_rows("splitmix64_seed0.txt")]
    assert [spectral.splitmix64(0, i) for i in range(len(ref))] == ref
    u = spectral.start_vector(1000, 0)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert u[0] == float(ref[0] >> 11) * 2.0 ** -52 - 1.0


def test_poisson_spectra_closed_form():
    for name, dims, N, lo, hi in _golden_rows("poisson_spectra.txt"):
        dims, N, lo, hi = int(dims), int(N), float(lo), float(hi)
        if N > 32:
            continue
        A = poisson2d(N) if dims == 2 else poisson3d(N)
        ev = np.linalg.eigvalsh(A.to_scipy().toarray())
        assert abs(ev[0] - lo) < 1e-12 and abs(ev[-1] - hi) < 1e-12
        assert spectral.gershgorin_max(A) == 4.0 * dims
        rmin, gmax = spectral.chebyshev_interval(A, m=30, seed=0)
        # Ritz values lie inside the spectrum; the Gershgorin bound above it
        assert lo - 1e-12 <= rmin and gmax >= hi


def test_lanczos_full_length_recovers_spectrum():
    d = np.array([0.5, 1.0, 2.0, 3.5, 7.0, 11.0])
    A = from_dense(np.diag(d))
    a, b = spectral.lanczos_tridiag(A, len(d), seed=3)
    rv = spectral.ritz_values(a, b)
    assert np.allclose(rv, d, rtol=1e-10)


# ---------------------------------------------------------------- basis, B, G

def _basis(A, s, first, basis, seed=0, lmin=None, lmax=None):
    ar = CR()
    n = A.n
    p = uniform(n, seed)
    r = uniform(n, seed + 1)
    prm = sstep.basis_params(basis, s, lmin, lmax, ar)
    Y = sstep.krylov_basis(ar, A, p, r, s, first, prm)
    B = np.array(sstep.assemble_B(ar, s, first, prm))
    return np.stack(Y, axis=1), B


@pytest.mark.parametrize("basis", ["monomial", "chebyshev"])
@pytest.mark.parametrize("first", [True, False])
def test_AY_underline_minus_YB_within_eq_E_bound(basis, first):
    """eq. E: ||A Y_ - Y B|| <= eps((3+N_A)||A|| ||Y_|| + 4||Y|| ||B||)."""
    A = poisson2d(16)
    M = A.to_scipy().toarray()
    s = 6
    Y, B = _basis(A, s, first, basis, lmin=0.07, lmax=8.0)
    Yu = Y.copy()
    last = [s] if first else [s, 2 * s]
    Yu[:, last] = 0.0
    E = M @ Yu - Y @ B
    NA = int(np.diff(A.rowptr).max())
    eps = sstep.EPS
    bound = eps * ((3 + NA) * np.linalg.norm(M, 2) * np.linalg.norm(Yu, 2)
                   + 4 * np.linalg.norm(Y, 2) * np.linalg.norm(B, 2))
    assert np.linalg.norm(E, 2) <= bound
    # a transposed B breaks it by orders of magnitude
    assert np.linalg.norm(M @ Yu - Y @ B.T, 2) > 1e6 * bound


def test_monomial_B_has_unit_norm():
    """Section 4.1: for the monomial basis ||B|| = 1."""
    for s in [1, 2, 4, 8, 10]:
        for first in [True, False]:
            B = np.array(sstep.assemble_B(CR(), s, first, sstep.basis_params("monomial", s)))
            assert np.linalg.norm(B, 2) == pytest.approx(1.0, abs=1e-15)


def test_chebyshev_basis_closed_form_on_diagonal_matrix():
    """rho_j(A) u = T_j((a_ii - c0)/h) u_i on a diagonal A (R11)."""
    d = np.linspace(0.3, 9.5, 40)
    A = from_dense(np.diag(d))
    lmin, lmax = 0.25, 10.0
    Y, _ = _basis(A, 8, True, "chebyshev", lmin=lmin, lmax=lmax)
    u = Y[:, 0]
    w = (d - (lmax + lmin) / 2) / ((lmax - lmin) / 2)
    for j in range(9):
        Tj = np.cos(j * np.arccos(w))
        assert np.allclose(Y[:, j], Tj * u, rtol=1e-12, atol=1e-13)


def _fma(a, b, s):
    """IEEE fused multiply-add by its definition: a * b + s exact, one rounding."""
    from fractions import Fraction

    return float(Fraction(a) * Fraction(b) + Fraction(s))


def _gram_by_definition(Y, group=1024):
    """G = Y^T Y in the stated order, written out with an exact-rational fma:
    per group of `group` rows (zero-padded) s = fma(y_ra, y_rb, s) from +0 in
    row order; the group partials zero-padded to a power of two and added by
    recursive halves."""
    n, d = Y.shape
    ng = -(-n // group)

    def halves(v):
        return v[0] if len(v) == 1 else halves(v[:len(v) // 2]) + halves(v[len(v) // 2:])

    G = np.zeros((d, d))
    for a in range(d):
        for b in range(a, d):
            parts = []
            for g in range(ng):
                s = 0.0
                for r in range(g * group, (g + 1) * group):
                    s = _fma(Y[r, a], Y[r, b], s) if r < n else _fma(0.0, 0.0, s)
                parts.append(s)
            P = 1
            while P < len(parts):
                P *= 2
            G[a, b] = G[b, a] = halves(parts + [0.0] * (P - len(parts)))
    return G


def test_gram_equals_explicit_YtY_in_the_stated_order():
    """The oracle's Gram (C helper) against its definition evaluated with
    rational fma (3 groups, the last one ragged, so the pairwise step pads to
    4), and against the exact inner products within the fma-chain bound."""
    from fractions import Fraction

    A = poisson2d(48)  # n = 2304: groups of 1024, 1024, 256
    Y, _ = _basis(A, 3, False, "monomial")
    G = np.array(CR().gram([Y[:, a] for a in range(Y.shape[1])]))
    assert np.array_equal(G, _gram_by_definition(Y))
    absb = np.abs(Y).T @ np.abs(Y)
    gam = (1024 + 2) * sstep.EPS / (1 - (1024 + 2) * sstep.EPS)  # chain of 1024 + 2 tree levels
    for a in range(Y.shape[1]):
        for b in range(Y.shape[1]):
            ex = float(sum((Fraction(x) * Fraction(y) for x, y in zip(Y[:, a], Y[:, b])),
                           Fraction(0)))
            assert abs(G[a, b] - ex) <= gam * absb[a, b]
    # the stated order is not just any order: a column pair whose sum depends on it
    big, tiny = 1.0, 2.0 ** -60
    col = np.zeros(2048)
    col[0], col[1], col[1024] = big, tiny, -big  # 1 + tiny in group 0, -1 in group 1
    G2 = np.array(CR().gram([col, np.ones(2048)]))
    assert G2[0, 1] == 0.0  # (1 + 2^-60) rounds to 1 inside group 0; then 1 + (-1)
    assert _gram_by_definition(np.stack([col, np.ones(2048)], 1))[0, 1] == 0.0


def test_sqrt_kappa_G_equals_kappa_Y_and_interlacing():
    """Section 4.2: sqrt(kappa(G_i)) = kappa(Y_i); the sub-Grams are principal
    submatrices, so kappa(G_i) cannot decrease with i (Cauchy interlacing)."""
    A, b, x1, _ = poisson2d_32_system(0)
    Y, _ = _basis(A, 6, False, "chebyshev", lmin=0.018, lmax=8.0)
    cols = [Y[:, a] for a in range(Y.shape[1])]
    G = CR().gram(cols)
    prev = 0.0
    for i in range(1, 7):
        idx = sstep.sub_indices(6, i, False)
        kG = okappa.kappa_spd(sstep.principal(G, idx))
        kY = np.linalg.cond(Y[:, idx])
        assert math.sqrt(kG) == pytest.approx(kY, rel=1e-6)
        assert kG >= prev * (1 - 1e-10)
        prev = kG


# ---------------------------------------------------------------- algorithms

def test_s_equals_one_reproduces_classical_cg():
    """Section 4.2: with s_k = 1 the variable s-step method performs classical CG."""
    A, b, x1, _ = poisson2d_32_system(0)
    cl = ocg.cg(A, b, x1, tol=1e-10, keep_iterates=True)
    res = sstep.solve(A, b, x1, sstep.Opts(mode="fixed", fixed_s=1, tol=1e-10))
    assert abs(res.iters - cl.iters) <= 1
    alphas = [a for blk in res.blocks for a in blk.alphas]
    k = min(len(alphas), 60)
    assert np.allclose(alphas[:k], cl.alphas[:k], rtol=1e-10)
    nx = np.linalg.norm(cl.x)
    assert np.linalg.norm(res.x - cl.x) / nx < 1e-9


def test_converged_solution_matches_cholesky_direct_solve():
    A, b, x1, _ = poisson2d_32_system(0)
    M = A.to_scipy().toarray()
    L = np.linalg.cholesky(M)
    xd = np.linalg.solve(L.T, np.linalg.solve(L, b))
    kap = np.linalg.cond(M)
    for opts in [sstep.Opts(mode="adaptive", s_max=8, equilibrate=True, tol=1e-10),
                 sstep.Opts(mode="fixed", fixed_s=4, equilibrate=True, tol=1e-10)]:
        res = sstep.solve(A, b, x1, opts)
        assert res.status == sstep.OK
        assert res.relres <= 1e-10
        assert np.linalg.norm(res.x - xd) / np.linalg.norm(xd) <= kap * 1e-10
        # the reported true residual is the residual of the returned x
        rel = np.linalg.norm(b - M @ res.x) / np.linalg.norm(b)
        assert rel < 2e-10


def test_adaptive_rule_replay_and_block0_decision_against_svd():
    """Replay every block's decision from its logged quantities; check block
    0's kappa list against the SVD of the explicit sub-bases."""
    A, b, x1, _ = poisson2d_32_system(0)
    opts = sstep.Opts(mode="adaptive", s_max=8, equilibrate=True, tol=1e-10)
    res = sstep.solve(A, b, x1, opts)
    assert res.status == sstep.OK
    eps = 2.0 ** -53
    m = 0
    s_prev = None
    for blk in res.blocks:
        # growth limit and rank guard
        s_bar = 8 if blk.k == 0 else min(s_prev + 8, 8)
        assert blk.s_bar == s_bar
        assert blk.s_built == (s_bar if blk.k == 0 else min(s_bar, m))
        # eq. condy as a prefix rule, default 1
        ok = [math.sqrt(kp) <= blk.thr for kp in blk.kappas]
        st = 0
        while st < len(ok) and ok[st]:
            st += 1
        assert blk.s_tilde == max(st, 1)
        assert len(blk.kappas) == min(st + 1, blk.s_built)
        assert 1 <= blk.s_k <= blk.s_tilde <= blk.s_built <= 8
        assert blk.m == m
        m += blk.s_k
        s_prev = blk.s_k
    # block 0 with x_1 = 0: thr = tol / (c eps)
    assert res.blocks[0].thr == pytest.approx(1e-10 / eps, rel=1e-14)
    # kappa list of block 0 vs explicit SVD of [P_0 .. P_i] of the scaled matrix
    As, sc = sstep.equilibrate(A)
    p = b * sc
    ar = CR()
    Y = np.stack(sstep.krylov_basis(ar, As, p, p, 8, True, sstep.basis_params("monomial", 8)), 1)
    for i, kp in enumerate(res.blocks[0].kappas, start=1):
        assert math.sqrt(kp) == pytest.approx(np.linalg.cond(Y[:, : i + 1]), rel=1e-4)


def test_adaptive_with_unreachable_tolerance_defaults_to_one():
    """Section 4.2: when the right-hand side of eq. yhk1 is below one the rule
    cannot be met and s_k = 1."""
    A, b, x1, _ = poisson2d_32_system(0)
    res = sstep.solve(A, b, x1, sstep.Opts(mode="adaptive", s_max=8, tol=1e-19, max_iters=30))
    assert res.status == sstep.NOT_CONVERGED
    assert res.blocks[0].thr < 1.0
    low = [blk for blk in res.blocks if blk.thr < 1.0]
    assert len(low) >= 3
    assert all(blk.s_tilde == 1 and blk.s_k == 1 for blk in low)


def test_adaptive_equals_its_schedule_replayed():
    """Reductions are correctly rounded, so the basis vectors and the Gram
    entries a block uses do not depend on how many extra vectors were built:
    replaying the adaptive schedule with Alg. 3 gives the same x bit for bit."""
    A, b, x1, _ = poisson2d_32_system(0)
    for basis, kw in [("monomial", {}), ("chebyshev", dict(lmin=0.018, lmax=8.0))]:
        ad = sstep.solve(A, b, x1, sstep.Opts(mode="adaptive", s_max=8, tol=1e-10, basis=basis, **kw))
        rp = sstep.solve(A, b, x1, sstep.Opts(mode="schedule", schedule=ad.schedule, tol=1e-10,
                                              basis=basis, **kw))
        assert rp.schedule == ad.schedule
        assert np.array_equal(rp.x, ad.x)


def test_huge_threshold_gives_full_blocks():
    """c -> 0 makes every basis acceptable: s_k = min(s_max, m) (rank guard)."""
    A, b, x1, _ = poisson2d_32_system(0)
    res = sstep.solve(A, b, x1, sstep.Opts(mode="adaptive", s_max=6, c=1e-300, tol=1e-10,
                                           basis="chebyshev", lmin=0.018, lmax=8.0))
    m = 0
    for blk in res.blocks:
        want = 6 if blk.k == 0 else min(6, m)
        assert blk.s_k == want
        m += blk.s_k


def test_residual_gap_growth_bound_fb():
    """eq. fb with the theoretical c_{k,j} = 6 N_k j kappa(A) holds for every
    inner iteration of every block (diagnostic materialisation)."""
    A = poisson2d(10)
    M = A.to_scipy().toarray()
    b = M @ uniform(A.n, 5)
    x1 = np.zeros(A.n)
    diag = []
    res = sstep.solve(A, b, x1, sstep.Opts(mode="fixed", fixed_s=5, tol=1e-12, max_iters=60),
                      diag=diag)
    assert res.blocks
    kA = np.linalg.cond(M)
    nA = np.linalg.norm(M, 2)
    NA = int(np.diff(A.rowptr).max())
    xs = np.linalg.solve(M, b)
    eps = sstep.EPS
    from fractions import Fraction

    def gap(x, r):
        # delta = b - A x - r, evaluated exactly then rounded
        out = np.empty(A.n)
        for i in range(A.n):
            s = Fraction(b[i]) - Fraction(r[i])
            for k in range(A.rowptr[i], A.rowptr[i + 1]):
                s -= Fraction(A.val[k]) * Fraction(x[A.col[k]])
            out[i] = float(s)
        return out

    by_block = {}
    for e in diag:
        by_block.setdefault(e["k"], []).append(e)
    starts = {0: (x1, b.copy())}
    xcur, rcur = x1, b.copy()
    for k in sorted(by_block):
        ents = by_block[k]
        d0 = gap(xcur, rcur)
        Y = np.stack(ents[0]["Y"], 1)
        kY = np.linalg.cond(Y)
        B = np.array(sstep.assemble_B(CR(), len(Y[0]) // 2 if k else len(Y[0]) - 1, k == 0,
                                      sstep.basis_params("monomial", 5)))
        tau = np.linalg.norm(B, 2) / nA
        Nk = 7 + 2 * NA + 14 * tau
        rmax = np.linalg.norm(rcur)
        for e in ents:
            j = e["j"]
            rmax = max(rmax, np.linalg.norm(e["r"]))
            ckj = 6 * Nk * j * kA
            lhs = np.linalg.norm(gap(e["x"], e["r"]) - d0)
            rhs = ckj * eps * kY * rmax + eps * nA * np.linalg.norm(xs)
            assert lhs <= rhs
        xcur, rcur = ents[-1]["x"], ents[-1]["r"]


def test_breakdown_on_indefinite_matrix():
    M = np.diag([1.0, -2.0, 3.0, 4.0])
    M[0, 1] = M[1, 0] = 0.5
    A = from_dense(M)
    b = np.ones(4)
    res = sstep.solve(A, b, np.zeros(4), sstep.Opts(mode="fixed", fixed_s=2, tol=1e-12, max_iters=50))
    assert res.status in (sstep.BREAKDOWN, sstep.NOT_CONVERGED)


def test_fixed_large_s_loses_accuracy_where_adaptive_does_not():
    """Section 5's observations, on the 32x32 Poisson stand-in at a target
    near classical CG's attainable accuracy: fixed s = 8 (monomial) stagnates
    above the target, adaptive s-step reaches it with far fewer outer loops
    than classical CG's iterations, and at s = 4, where fixed s-step converges,
    adaptive needs at most two more outer loops."""
    A, b, x1, _ = poisson2d_32_system(0)
    tol = 1e-14
    cl = ocg.cg(A, b, x1, tol=tol, max_iters=1000)
    assert cl.status == sstep.OK
    fx8 = sstep.solve(A, b, x1, sstep.Opts(mode="fixed", fixed_s=8, tol=tol, equilibrate=True,
                                           max_iters=600))
    ad8 = sstep.solve(A, b, x1, sstep.Opts(mode="adaptive", s_max=8, tol=tol, equilibrate=True,
                                           max_iters=600))
    assert fx8.status == sstep.NOT_CONVERGED and min(bl.relres_true for bl in fx8.blocks) > 10 * tol
    assert ad8.status == sstep.OK and ad8.relres <= tol
    assert len(ad8.blocks) * 4 < cl.iters
    fx4 = sstep.solve(A, b, x1, sstep.Opts(mode="fixed", fixed_s=4, tol=tol, equilibrate=True))
    ad4 = sstep.solve(A, b, x1, sstep.Opts(mode="adaptive", s_max=4, tol=tol, equilibrate=True))
    assert fx4.status == sstep.OK and ad4.status == sstep.OK
    assert len(ad4.blocks) <= len(fx4.blocks) + 2


def test_plain_arithmetic_within_summation_bounds_and_solves():
    """The plain-FP64 back-end (timing only): every reduction within the
    recursive-summation bound n eps sum|terms| of the correctly rounded one,
    and an adaptive solve with it reaches the tolerance near CR's solution."""
    from oracle.arith import Plain

    rng = np.random.default_rng(2)
    ar, cr = Plain(), CR()
    A = poisson2d(20)
    u = rng.standard_normal(A.n)
    w = rng.standard_normal(A.n)
    eps = 2.0 ** -53
    got = ar.csr_comb(A, u, [(-0.5, w)])
    ref = cr.csr_comb(A, u, [(-0.5, w)])
    mag = np.abs(A.to_scipy()) @ np.abs(u) + 0.5 * np.abs(w)
    assert np.all(np.abs(got - ref) <= 8 * eps * mag)
    cols = [rng.standard_normal(500) * 10.0 ** k for k in range(-2, 3)]
    G, Gc = np.array(ar.gram(cols)), np.array(cr.gram(cols))
    Y = np.abs(np.stack(cols))
    assert np.all(np.abs(G - Gc) <= 500 * eps * (Y @ Y.T))
    A2, b, x1, _ = poisson2d_32_system(0)
    opts = sstep.Opts(mode="adaptive", s_max=8, tol=1e-10, equilibrate=True)
    rp = sstep.solve(A2, b, x1, opts, ar=Plain())
    rc = sstep.solve(A2, b, x1, opts)
    assert rp.status == sstep.OK and rp.relres <= 1e-10
    M = A2.to_scipy().toarray()
    assert np.linalg.norm(rp.x - rc.x) / np.linalg.norm(rc.x) <= np.linalg.cond(M) * 2e-10
    lo, hi = spectral.chebyshev_interval(A2, 30, 0, ar=Plain())
    lo_c, hi_c = spectral.chebyshev_interval(A2, 30, 0)
    assert lo == pytest.approx(lo_c, rel=1e-8) and hi == pytest.approx(hi_c, rel=1e-14)
