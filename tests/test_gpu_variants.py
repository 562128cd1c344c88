"""Method variants on the GPU against the oracle, through the C ABI: the Newton
basis (Section 2; shifts = Leja-ordered Ritz values of a short Lanczos run)
and the theoretical c_{k,j} = 6 N_k j kappa(A) of Section 4.1.

Bars as for the other parity tests: stage outputs (shifts, basis, kappa list,
thresholds, coefficients) agree to the last bit (1e-15 relative allowed for a
near-tie of the double-double sums); whole solves take the oracle's s_k
schedule and iterates within 1e-12 relative.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kappa as okappa  # noqa: E402
from oracle import spectral, sstep  # noqa: E402
from oracle.arith import CR  # noqa: E402
from paper_1701_03989_amd import problems, sscg  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    h = sscg.sscg_create(0)
    yield h
    sscg.sscg_destroy(h)


def dvec(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def assert_bits(got, ref, what, rel=1e-15):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, what
    diff = np.abs(got - ref)
    scale = np.maximum(np.abs(ref), 1e-300)
    worst = float((diff / scale).max()) if diff.size else 0.0
    say(f"{what}: exact {(got == ref).mean() if got.size else 1.0:.6f}, worst rel {worst:.2e}")
    assert worst <= rel, f"{what}: worst relative difference {worst}"


MATRICES = {
    "poisson2d_32": lambda: problems.poisson2d(32),
    "poisson3d_11": lambda: problems.poisson3d(11),
    "laplacian_3001": lambda: problems.graph_laplacian(3001, 7),
}


@pytest.mark.parametrize("name", list(MATRICES))
@pytest.mark.parametrize("m", [1, 5, 8, 16])
def test_newton_shifts_match_oracle(ctx, name, m):
    A = MATRICES[name]()
    say(f"newton shifts {name} m={m}")
    got = sscg.sscg_newton_shifts(ctx, sscg.DeviceCsr.from_host(A, DEV), m, 3)
    ref = spectral.newton_shifts(A, m, 3)
    assert_bits(got, ref, "shifts")
    assert got[0] == max(got, key=abs)


@pytest.mark.parametrize("name", ["poisson2d_32", "laplacian_3001"])
@pytest.mark.parametrize("first", [True, False])
def test_mpk_newton_matches_oracle(ctx, name, first):
    A = MATRICES[name]()
    n, s = A.n, 6
    shifts = spectral.newton_shifts(A, s, 0)
    say(f"mpk newton {name} first={first}")
    p = problems.uniform(n, 21)
    r = problems.uniform(n, 22)
    ar = CR()
    prm = sstep.basis_params("newton", s, ar=ar, shifts=shifts)
    Yo = sstep.krylov_basis(ar, A, p, r, s, first, prm)
    ld = (n + 63) // 64 * 64
    rcol = s + 1
    Y = torch.zeros((2 * s + 1) * ld, dtype=torch.float64, device=DEV)
    Y[:n] = dvec(p)
    if not first:
        Y[rcol * ld: rcol * ld + n] = dvec(r)
    sscg.sscg_mpk_newton(ctx, sscg.DeviceCsr.from_host(A, DEV), s, first, shifts, Y, ld, rcol)
    Yh = host(Y)
    cols = list(range(s + 1)) + ([] if first else list(range(rcol, rcol + s)))
    for a, c in enumerate(cols):
        assert_bits(Yh[c * ld: c * ld + n], Yo[a], f"Y col {a}")


@pytest.mark.parametrize("first", [True, False])
@pytest.mark.parametrize("basis", ["monomial", "chebyshev", "newton"])
def test_small_solve_theory_c_matches_oracle(ctx, first, basis):
    """kappa list, thr with c_{k,s_max}, s~, the eq. check breaks with c_{k,j},
    alpha/beta and coefficients from the same G."""
    A = problems.poisson2d(32)
    s, s_max = (8, 10) if first else (5, 8)
    lmin, lmax = (0.0181, 7.99) if basis == "chebyshev" else (0.0, 1.0)
    shifts = spectral.newton_shifts(A, s_max, 0) if basis == "newton" else None
    ar = CR()
    prm_o = sstep.basis_params(basis, s, lmin, lmax, ar, shifts)
    Yo = sstep.krylov_basis(ar, A, problems.uniform(A.n, 1), problems.uniform(A.n, 2), s, first,
                            prm_o)
    G = ar.gram(Yo)
    d = len(G)
    eps_star = 1e-8 * 30.0
    n_a, kappa_a, norm_a = 5, 440.69, 7.99
    say(f"small solve theory c: first={first} basis={basis} d={d}")
    code = {"monomial": 0, "chebyshev": sscg.BASIS_CHEBYSHEV, "newton": sscg.BASIS_NEWTON}[basis]
    prm = sscg.BlockParams(s=s, first=int(first), adaptive=1, iters=s, inner_check=1, basis=code,
                           lambda_min=lmin, lambda_max=lmax, eps_star=eps_star, c=1.0,
                           c_mode=sscg.C_THEORY, n_a=n_a, s_max=s_max, kappa_a=kappa_a,
                           norm_a=norm_a)
    if shifts is not None:
        for i in range(s_max):
            prm.shifts[i] = shifts[i]
    coef = torch.zeros(3 * d, dtype=torch.float64, device=DEV)
    info_t = torch.zeros(1024, dtype=torch.uint8, device=DEV)
    sscg.sscg_small_solve(ctx, dvec(np.array(G).ravel()), prm, coef, info_t)
    info = sscg.block_info_from(info_t)
    # the oracle's decisions (eqs. condy and check with the theoretical c)
    bnorm = sstep.b_norm_bound(sstep.assemble_B(ar, s, first, prm_o))

    def cfun(j):
        return sstep.c_theory(j, n_a, bnorm, norm_a, kappa_a)

    rnorm = ar.sqrt(G[0][0] if first else G[s + 1][s + 1])
    thr = ar.div(eps_star, (cfun(s_max) * sstep.EPS) * rnorm)
    kap = [okappa.kappa_spd(sstep.principal(G, sstep.sub_indices(s, i, first)))
           for i in range(1, s + 1)]
    assert_bits(list(info.kappa)[:s], kap, "kappa")
    st = 1
    for i in range(1, s + 1):
        if ar.sqrt(kap[i - 1]) <= thr:
            st = i
        else:
            break
    gam = ar.sqrt(kap[st - 1])
    say(f"  ||B|| bound {bnorm:.6g}, c(s_max) {cfun(s_max):.6g}, thr {thr:.4g}, s~ {st}")
    assert info.thr == thr and info.gamma == gam and info.s_tilde == st

    def check(j, rr1):
        return gam >= ar.div(eps_star, (cfun(j) * sstep.EPS) * ar.sqrt(max(rr1, 0.0)))

    idx = sstep.sub_indices(s, st, first)
    Bs = sstep.assemble_B(ar, st, first, sstep.basis_params(basis, st, lmin, lmax, ar, shifts))
    s_k, xc, rc, pc, al, be, rr, status = sstep.inner_loop(ar, sstep.principal(G, idx), Bs, st,
                                                           first, check)
    assert info.s_k == s_k and info.status == status
    assert_bits(list(info.alpha)[:s_k], al, "alpha")
    assert_bits(list(info.beta)[:s_k], be, "beta")
    full = np.zeros((3, d))
    for a, fa in enumerate(idx):
        full[0, fa], full[1, fa], full[2, fa] = xc[a], rc[a], pc[a]
    assert_bits(host(coef), full.ravel(), "coef")


LO32, HI32 = problems.poisson_interval(32, 2)

# (device options, oracle options); shifts "oracle" = spectral.newton_shifts of
# the solve's matrix with m = s_max (the device computes its own when the
# device options carry none)
SOLVES = [
    ("newton s_max 8, device shifts", dict(mode="adaptive", basis="newton", s_max=8, tol=1e-10)),
    ("newton s_max 16, device shifts", dict(mode="adaptive", basis="newton", s_max=16,
                                            tol=1e-10)),
    ("newton s_max 12 tol 1e-13, given shifts",
     dict(mode="adaptive", basis="newton", s_max=12, tol=1e-13, give_shifts=True)),
    ("newton fixed 8", dict(mode="fixed", fixed_s=8, basis="newton", s_max=8, tol=1e-10)),
    ("newton speculative", dict(mode="adaptive", basis="newton", s_max=8, tol=1e-10, s0_bar=1,
                                f=1)),
    ("newton equilibrated", dict(mode="adaptive", basis="newton", s_max=10, tol=1e-12,
                                 equilibrate=True)),
    ("theory monomial", dict(mode="adaptive", s_max=8, tol=1e-10, c_mode="theory",
                             kappa_a=HI32 / LO32, norm_a=HI32)),
    ("theory chebyshev", dict(mode="adaptive", basis="chebyshev", lmin=LO32, lmax=HI32, s_max=8,
                              tol=1e-10, c_mode="theory", kappa_a=HI32 / LO32, norm_a=HI32)),
    ("theory chebyshev speculative",
     dict(mode="adaptive", basis="chebyshev", lmin=LO32, lmax=HI32, s_max=8, tol=1e-10,
          s0_bar=1, f=1, c_mode="theory", kappa_a=HI32 / LO32, norm_a=HI32)),
    ("theory newton speculative",
     dict(mode="adaptive", basis="newton", s_max=8, tol=1e-10, s0_bar=1, f=1, c_mode="theory",
          kappa_a=HI32 / LO32, norm_a=HI32)),
    ("theory chebyshev, estimated interval and kappa",
     dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10, c_mode="theory",
          estimate=True)),
]


@pytest.mark.parametrize("k", range(len(SOLVES)))
def test_variant_solve_matches_oracle_on_poisson_32(ctx, k):
    name, kw = SOLVES[k]
    kw = dict(kw)
    give = kw.pop("give_shifts", False)
    estimate = kw.pop("estimate", False)
    A, b, x1, _ = problems.poisson2d_32_system(0)
    say(f"variant solve: {name}")
    okw = dict(kw)
    Ao = sstep.equilibrate(A)[0] if kw.get("equilibrate") else A
    if kw.get("basis") == "newton":
        okw["shifts"] = spectral.newton_shifts(Ao, kw["s_max"], 0)
        if give:
            kw["shifts"] = okw["shifts"]
    if estimate:
        lo, hi = spectral.chebyshev_interval(A, 30, 0)
        okw.update(lmin=lo, lmax=hi, kappa_a=hi / lo, norm_a=hi)
    ref = sstep.solve(A, b, x1, sstep.Opts(**okw))
    Ad = sscg.DeviceCsr.from_host(A, DEV)
    x = dvec(x1)
    hist = sscg.History(4096, kw["s_max"])
    rc = sscg.sscg_solve(ctx, Ad, dvec(b), x, sscg.make_opts(**kw), hist)
    xh = host(x)
    say(f"  gpu {hist.blocks} blocks {hist.schedule[:24]}  oracle {len(ref.blocks)} blocks, "
        f"spec {hist.res.spec_blocks}/{hist.res.spec_rejected}")
    assert rc == ref.status
    assert hist.schedule == ref.schedule
    for kb, blk in enumerate(ref.blocks):
        assert hist.s_tilde[kb] == blk.s_tilde and hist.s_built[kb] == blk.s_built
        if kw["mode"] == "adaptive" and kb < 64:
            assert hist.thr[kb] == blk.thr, kb
    err = np.linalg.norm(xh - ref.x) / np.linalg.norm(ref.x)
    say(f"  |x - x_oracle| / |x_oracle| = {err:.2e}")
    assert err <= 1e-12
    assert hist.res.relres <= kw["tol"] or rc != sscg.OK


@pytest.mark.parametrize("basis", ["newton", "chebyshev"])
def test_mixed_precision_variants_reach_tolerance(ctx, basis):
    A, b, x1, _ = problems.poisson2d_32_system(0)
    kw = dict(mode="adaptive", basis=basis, s_max=8, tol=1e-10, precision="mixed",
              c_mode="theory")
    say(f"mixed precision {basis}, theoretical c with estimated kappa")
    x = dvec(x1)
    hist = sscg.History(4096, 8)
    rc = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(A, DEV), dvec(b), x,
                         sscg.make_opts(**kw), hist)
    xh = host(x)
    relres = np.linalg.norm(b - A.matvec(xh)) / np.linalg.norm(b)
    say(f"  status {rc} blocks {hist.blocks} iters {hist.res.iters} relres {relres:.2e}")
    assert rc == sscg.OK and relres <= 1e-10


def test_unsupported_variant_combinations_are_rejected(ctx):
    A, b, x1, _ = problems.poisson2d_32_system(0)
    Ad = sscg.DeviceCsr.from_host(A, DEV)
    with pytest.raises(sscg.SscgError) as e:
        sscg.sscg_batch_solve(ctx, [Ad], [dvec(b)], [dvec(x1)],
                              sscg.make_opts(basis="newton", s_max=4))
    assert e.value.code == sscg.ERR_ARG
    with pytest.raises(sscg.SscgError) as e:
        sscg.sscg_server_create(ctx, sscg.make_opts(c_mode="theory"), 4096, 40000, 4)
    assert e.value.code == sscg.ERR_ARG
    # mixed precision is a sscg_solve option: batches and the server refuse it
    with pytest.raises(sscg.SscgError) as e:
        sscg.sscg_batch_solve(ctx, [Ad], [dvec(b)], [dvec(x1)], sscg.make_opts(precision="mixed"))
    assert e.value.code == sscg.ERR_ARG and "SSCG_PREC_MIXED is not supported" in str(e.value)
    with pytest.raises(sscg.SscgError) as e:
        sscg.sscg_server_create(ctx, sscg.make_opts(precision="mixed"), 4096, 40000, 4)
    assert e.value.code == sscg.ERR_ARG and "SSCG_PREC_MIXED is not supported" in str(e.value)
    Y = torch.zeros(8 * 1024, dtype=torch.float64, device=DEV)
    with pytest.raises(sscg.SscgError) as e:  # Newton needs its shifts: sscg_mpk_newton
        sscg.sscg_mpk(ctx, Ad, 3, True, sscg.BASIS_NEWTON, 0.0, 1.0, Y, 1024, 4)
    assert e.value.code == sscg.ERR_ARG
    with pytest.raises(sscg.SscgError) as e:
        sscg.sscg_solve(ctx, Ad, dvec(b), dvec(x1),
                        sscg.make_opts(basis="newton", s_max=4, shifts=[1.0, math.inf, 2.0, 3.0]))
    assert e.value.code == sscg.ERR_ARG


def banded_far(n, D, seed):
    """SPD: tridiagonal plus a coupling at distance D in every row that has one
    (diagonally dominant), CSR with ascending columns."""
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    off1 = -rng.uniform(0.1, 0.5, n - 1)
    offD = -rng.uniform(0.1, 0.5, n - D)
    M = sp.diags([off1, off1, offD, offD], [1, -1, D, -D], shape=(n, n), format="lil")
    M.setdiag(2.5)
    M = M.tocsr()
    M.sort_indices()
    return problems.CSR(M.indptr.astype(np.int32), M.indices.astype(np.int32),
                        M.data.astype(np.float64))


@pytest.mark.parametrize("D", [32700, 32768, 40000])
def test_column_offset_formats(ctx, D):
    """The matrix-powers pass reads 16-bit column offsets from the slice's first
    row when every one fits (D = 32700: at most 32700 + 63), else the 32-bit
    indices (D = 32768, 40000): same bits as the oracle either way."""
    A = banded_far(D + 4000, D, 3)
    n, s = A.n, 5
    lo, hi = 0.5, 4.5  # Gershgorin interval of banded_far
    p = problems.uniform(n, 31)
    r = problems.uniform(n, 32)
    ar = CR()
    Yo = sstep.krylov_basis(ar, A, p, r, s, False, sstep.basis_params("chebyshev", s, lo, hi, ar))
    ld = (n + 63) // 64 * 64
    rcol = s + 1
    Y = torch.zeros((2 * s + 1) * ld, dtype=torch.float64, device=DEV)
    Y[:n] = dvec(p)
    Y[rcol * ld: rcol * ld + n] = dvec(r)
    say(f"column offsets: n={n}, coupling distance {D}")
    sscg.sscg_mpk(ctx, sscg.DeviceCsr.from_host(A, DEV), s, False, sscg.BASIS_CHEBYSHEV, lo, hi, Y,
                  ld, rcol)
    Yh = host(Y)
    cols = list(range(s + 1)) + list(range(rcol, rcol + s))
    for a, c in enumerate(cols):
        assert_bits(Yh[c * ld: c * ld + n], Yo[a], f"Y col {a}")
    # and a whole solve through sscg_solve
    b = problems.uniform(n, 33)
    ref = sstep.solve(A, b, np.zeros(n), sstep.Opts(mode="adaptive", basis="chebyshev", lmin=lo,
                                                     lmax=hi, s_max=6, tol=1e-12))
    x = dvec(np.zeros(n))
    h = sscg.History(512, 6)
    rc = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(A, DEV), dvec(b), x,
                         sscg.make_opts(mode="adaptive", basis="chebyshev", lmin=lo, lmax=hi,
                                        s_max=6, tol=1e-12), h)
    assert rc == ref.status and h.schedule == ref.schedule
    assert np.linalg.norm(host(x) - ref.x) <= 1e-12 * np.linalg.norm(ref.x)
