"""Parity at the full single-solve size: 3-D 7-point Poisson 128^3 (n = 2,097,152,
nnz = 14,581,760), in the launch configuration bench.py times (sscg_solve,
Chebyshev basis, s_max = 10, tol 1e-12).

The oracle cannot run the whole solve in seconds, but it can run the set-up
and the first outer blocks, and each stage on seeded inputs:
  * the Chebyshev interval estimate (30 Lanczos steps): same bits;
  * the first two outer blocks of Algorithm 4 (19 matrix-powers passes, two
    Gram matrices, the kappa lists, s~, the coefficient recurrences and the
    recoveries): same s_k schedule, kappa lists and thresholds, and x within
    1e-12 relative;
  * the Gram matrix and the recovery of 21 seeded columns of 2.1 M rows
    (scaled, nearly parallel and nearly orthogonal columns): same bits.
The whole solve is checked through properties that hold at any size: the
true relative residual recomputed on the host is below the tolerance, and
two runs give the same bits.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import spectral, sstep  # noqa: E402
from oracle.arith import CR  # noqa: E402
from paper_1701_03989_amd import problems, sscg  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"
N = 128
KW = dict(mode="adaptive", basis="chebyshev", s_max=10, tol=1e-12)


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


@pytest.fixture(scope="module")
def system():
    A, b, x1 = problems.poisson3d_128_system(0, N=N)
    return A, b, x1


@pytest.fixture(scope="module")
def interval(system):
    A, _, _ = system
    return spectral.chebyshev_interval(A, 30, 0)


def rel_worst(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float((np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)).max())


def test_fullsize_chebyshev_interval(ctx, system, interval):
    A, _, _ = system
    say(f"128^3 interval: n={A.n} nnz={A.nnz}")
    lo, hi = sscg.sscg_spectral_bounds(ctx, sscg.DeviceCsr.from_host(A, DEV), 30, 0)
    say(f"  device [{lo!r}, {hi!r}]  oracle [{interval[0]!r}, {interval[1]!r}]")
    assert rel_worst([lo, hi], interval) <= 1e-15


def test_fullsize_first_blocks_match_oracle(ctx, system, interval):
    A, b, x1 = system
    lo, hi = interval
    kw = dict(KW, lmin=lo, lmax=hi, max_iters=20)  # two outer blocks of s = 10
    say("128^3 first two blocks: oracle")
    ref = sstep.solve(A, b, x1, sstep.Opts(**kw))
    say("128^3 first two blocks: device")
    x = torch.as_tensor(x1, device=DEV)
    hist = sscg.History(64, KW["s_max"])
    rc = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(A, DEV), torch.as_tensor(b, device=DEV), x,
                         sscg.make_opts(**kw), hist)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    say(f"  device {hist.schedule} oracle {ref.schedule}; status {rc} / {ref.status}")
    assert rc == ref.status
    assert hist.schedule == ref.schedule and len(ref.blocks) == 2
    for kb, blk in enumerate(ref.blocks):
        assert hist.s_tilde[kb] == blk.s_tilde and hist.s_built[kb] == blk.s_built
        gk = hist.kappas(kb)
        assert gk[: len(blk.kappas)] == blk.kappas, kb
        assert hist.thr[kb] == blk.thr, kb
        assert hist.relres_true[kb] == pytest.approx(blk.relres_true, rel=1e-12)
    err = np.linalg.norm(xh - ref.x) / np.linalg.norm(ref.x)
    say(f"  |x - x_oracle| / |x_oracle| = {err:.2e}, equal entries {(xh == ref.x).mean():.6f}")
    assert err <= 1e-12


def test_fullsize_gram_and_recovery_match_oracle(ctx):
    n, s = N ** 3, 10
    d = 2 * s + 1
    rng = np.random.default_rng(11)
    base = rng.uniform(-1.0, 1.0, n)
    cols = []
    for a in range(d):
        if a % 3 == 0:  # nearly parallel to the base vector: large entries, cancellation in G
            v = base + 1e-7 * rng.uniform(-1.0, 1.0, n)
        elif a % 3 == 1:  # an independent vector at another scale
            v = rng.uniform(-1.0, 1.0, n) * 10.0 ** rng.uniform(-4, 4)
        else:  # nearly orthogonal to the base vector: small entries of G
            w = rng.uniform(-1.0, 1.0, n)
            v = w - (w @ base) / (base @ base) * base
        cols.append(np.ascontiguousarray(v))
    ld = n + 64
    rcol = s + 1
    Y = torch.zeros((2 * s + 1) * ld, dtype=torch.float64, device=DEV)
    for a in range(d):
        c = a if a <= s else rcol + (a - s - 1)
        Y[c * ld: c * ld + n] = torch.as_tensor(cols[a], device=DEV)
    G = torch.zeros(d * d, dtype=torch.float64, device=DEV)
    say("128^3-row Gram of 21 seeded columns")
    sscg.sscg_gram(ctx, n, s, False, Y, ld, rcol, G)
    torch.cuda.synchronize()
    Gh = G.cpu().numpy().reshape(d, d)
    Go = np.array(CR().gram(cols))
    say(f"  equal entries {(Gh == Go).mean():.4f}, worst rel {rel_worst(Gh, Go):.1e}")
    assert rel_worst(Gh, Go) <= 1e-15
    # recovery with seeded coefficients (some columns unused)
    coef = rng.standard_normal(3 * d)
    coef[[4, 4 + d, 4 + 2 * d]] = 0.0
    x0 = rng.uniform(-1.0, 1.0, n)
    xd = torch.as_tensor(x0, device=DEV)
    rd = torch.zeros(n, dtype=torch.float64, device=DEV)
    pd = torch.zeros(n, dtype=torch.float64, device=DEV)
    say("128^3-row recovery")
    sscg.sscg_recover(ctx, n, s, False, Y, ld, rcol, torch.as_tensor(coef, device=DEV), xd, rd, pd)
    torch.cuda.synchronize()
    xo, ro, po = sstep.recover(CR(), cols, coef[:d], coef[d:2 * d], coef[2 * d:], x0)
    for got, ref, what in ((xd, xo, "x"), (rd, ro, "r"), (pd, po, "p")):
        gh = got.cpu().numpy()
        say(f"  {what}: equal {(gh == ref).mean():.6f}, worst rel {rel_worst(gh, ref):.1e}")
        assert rel_worst(gh, ref) <= 1e-15


def test_fullsize_solve_properties(ctx, system):
    A, b, x1 = system
    Ad = sscg.DeviceCsr.from_host(A, DEV)
    bd = torch.as_tensor(b, device=DEV)
    xs, hists = [], []
    for run in range(2):
        say(f"128^3 whole solve, run {run}")
        x = torch.as_tensor(x1, device=DEV)
        hist = sscg.History(4096, KW["s_max"])
        rc = sscg.sscg_solve(ctx, Ad, bd, x, sscg.make_opts(**KW), hist)
        torch.cuda.synchronize()
        assert rc == sscg.OK
        xs.append(x.cpu().numpy())
        hists.append(hist)
    relres = np.linalg.norm(b - A.matvec(xs[0])) / np.linalg.norm(b)
    h = hists[0]
    say(f"  blocks {h.blocks}, iterations {h.res.iters}, host relres {relres:.3e} "
        f"(reported {h.res.relres:.3e})")
    assert relres <= KW["tol"]
    assert h.res.relres == pytest.approx(relres, rel=1e-6)
    assert np.array_equal(xs[0], xs[1]) and h.schedule == hists[1].schedule
    assert sum(h.schedule) == h.res.iters
