"""Mixed precision (FP32 basis inside FP64 iterative refinement) through the C
ABI.

Stages: the FP32 matrix-powers pass must equal, bit for bit, its definition in
the oracle (oracle/mixed.py: exact products of FP32 values summed in FP64 in
each row's CSR order, the three-term correction and the division in FP64, one
rounding to FP32); the Gram matrix of FP32 columns must equal the oracle's
(the stated order of the Gram) bit for bit.  Whole solves: the
true relative residual of A x = b (the caller's system, also when
equilibrating) reaches the tolerance, and the error against the FP64 oracle's
solution is stated and bounded by kappa(A) times the tolerance.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mixed, sstep  # noqa: E402
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


def mpk32_ref(A, s, first, basis, lmin, lmax, p0, r0):
    """The FP32 pass by its definition (oracle/mixed.py)."""
    name = "chebyshev" if basis == sscg.BASIS_CHEBYSHEV else "monomial"
    return mixed.mpk32_basis(A, s, first, name, p0, r0, lmin, lmax)


CASES = [("poisson2d", sscg.BASIS_MONOMIAL, True), ("poisson2d", sscg.BASIS_CHEBYSHEV, False),
         ("graph", sscg.BASIS_CHEBYSHEV, False), ("graph", sscg.BASIS_MONOMIAL, False)]


@pytest.mark.parametrize("k", range(len(CASES)))
def test_mpk32_matches_its_definition_bitwise(ctx, k):
    kind, basis, first = CASES[k]
    A = problems.poisson2d(40) if kind == "poisson2d" else problems.graph_laplacian(3001, 3)
    lmin, lmax = (0.01, 8.0) if kind == "poisson2d" else (0.005, 30.0)
    s, n = 6, A.n
    ld = (n + 63) // 64 * 64 + 64
    rcol = s + 1
    p0 = problems.uniform(n, 1).astype(np.float32)
    r0 = problems.uniform(n, 2).astype(np.float32)
    Y = torch.zeros((2 * s + 1) * ld, dtype=torch.float32, device=DEV)
    Y[:n] = torch.as_tensor(p0, device=DEV)
    Y[rcol * ld:rcol * ld + n] = torch.as_tensor(r0, device=DEV)
    sscg.sscg_mpk32(ctx, sscg.DeviceCsr.from_host(A, DEV), s, first, basis, lmin, lmax, Y, ld,
                    rcol)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy()
    P, R = mpk32_ref(A, s, first, basis, lmin, lmax, p0, r0)
    say(f"mpk32 {kind} basis={basis} first={first}")
    for j in range(1, s + 1):
        assert np.array_equal(Yh[j * ld:j * ld + n], P[j]), ("P", j)
    if not first:
        for j in range(1, s):
            got = Yh[(rcol + j) * ld:(rcol + j) * ld + n]
            assert np.array_equal(got, R[j]), ("R", j)


@pytest.mark.parametrize("s", [5, 8, 10, 12])
def test_gram32_matches_the_oracle_bitwise(ctx, s):
    n = 20000
    ld = n + 64
    rcol = s + 1
    rng = np.random.default_rng(5)
    Yh = np.zeros((2 * s + 1) * ld, dtype=np.float32)
    cols = []
    for a in range(2 * s + 1):
        v = (rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 3)).astype(np.float32)
        c = a if a <= s else rcol + (a - s - 1)
        Yh[c * ld:c * ld + n] = v
        cols.append(v.astype(np.float64))
    Y = torch.as_tensor(Yh, device=DEV)
    d = 2 * s + 1
    G = torch.zeros(d * d, dtype=torch.float64, device=DEV)
    sscg.sscg_gram32(ctx, n, s, False, Y, ld, rcol, G)
    torch.cuda.synchronize()
    Gh = G.cpu().numpy().reshape(d, d)
    fcols = [c.astype(np.float32) for c in cols]
    ref = mixed.gram32(fcols)
    say(f"gram32: {int(np.sum(Gh == ref))}/{d * d} entries bit-identical")
    assert np.array_equal(Gh, ref)
    assert np.array_equal(Gh, Gh.T)


SOLVES = [
    ("poisson2d_32", dict(basis="chebyshev", s_max=8, tol=1e-10, lmin=0.0181, lmax=8.0)),
    ("poisson2d_32", dict(basis="monomial", s_max=4, tol=1e-12)),
    ("poisson3d_24", dict(basis="chebyshev", s_max=10, tol=1e-12)),
    ("diffusion_48", dict(basis="chebyshev", s_max=8, tol=1e-10, equilibrate=True)),
]


def system(name):
    if name == "poisson2d_32":
        A, b, x1, _ = problems.poisson2d_32_system(0)
        return A, b, x1
    if name == "poisson3d_24":
        return problems.poisson3d_128_system(0, N=24)
    return problems.diffusion2d_system(48, 0)


@pytest.mark.parametrize("k", range(len(SOLVES)))
def test_mixed_solve_reaches_tolerance_and_matches_fp64_oracle(ctx, k):
    name, kw = SOLVES[k]
    A, b, x1 = system(name)
    say(f"mixed {name} {kw}")
    x = torch.as_tensor(x1, device=DEV)
    hist = sscg.History(4096, kw["s_max"])
    rc = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(A, DEV), torch.as_tensor(b, device=DEV), x,
                         sscg.make_opts(mode="adaptive", precision="mixed", **kw), hist)
    xh = x.cpu().numpy()
    ar = CR()  # correctly rounded residual rows and sums, as on the device
    relres = sstep.relres_of(ar, A, b, xh, ar.sqrt(ar.dot(b, b)))
    okw = dict(kw, tol=1e-14)
    if kw["basis"] == "chebyshev" and "lmin" not in kw:  # the interval the solve estimated
        okw.update(lmin=hist.res.lambda_min, lmax=hist.res.lambda_max)
    ref = sstep.solve(A, b, x1, sstep.Opts(mode="adaptive", **okw))
    err = np.linalg.norm(xh - ref.x) / np.linalg.norm(ref.x)
    if name.startswith("poisson"):  # closed form
        lo, hi = problems.poisson_interval(*((32, 2) if name == "poisson2d_32" else (24, 3)))
        kappa = hi / lo
    else:  # dense spectrum (n = 2304)
        D = np.zeros((A.n, A.n))
        for i in range(A.n):
            D[i, A.col[A.rowptr[i]:A.rowptr[i + 1]]] = A.val[A.rowptr[i]:A.rowptr[i + 1]]
        ev = np.linalg.eigvalsh(D)
        kappa = ev[-1] / ev[0]
    say(f"  status {rc} blocks {hist.blocks} iters {hist.res.iters} relres {relres:.2e} "
        f"(reported {hist.res.relres:.2e}); error vs FP64 oracle {err:.2e}, kappa {kappa:.1e}")
    assert rc == sscg.OK
    # the refinement stops on the caller's system, equilibrated or not
    assert hist.res.relres <= kw["tol"]
    assert relres <= kw["tol"] * (1 + 1e-6)
    assert err <= 10.0 * kappa * (kw["tol"] + 1e-14)
