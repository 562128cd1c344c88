"""GPU parity of the device forms of the matrix.

The matrix-powers pass reads A in one of four forms: the slice-diagonal form
(every 64-row slice couples its rows to at most 8 column distances with at
most 3 distinct values: per-slice distances and values, a 2-bit code per row
and distance), per-slice value tables with one-byte indices and 16-bit column
offsets (no 64-row slice holds more than four distinct values), 16-bit offsets
with the stored values, or 32-bit indices with the stored values.  Each form must give the oracle's row sums
(eq. cg-krylovbasis, every row rounded once), and since a table entry carries
the stored value's bits, the three forms must agree with each other to the last
bit on the same rows.  Block-diagonal matrices put the same block into each
form: a second block with five values in a slice, or with a column 33000 rows
away from its slice, switches the whole matrix to the wider form while the rows
of the first block keep their entries and their order.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sstep  # noqa: E402
from oracle.arith import CR  # noqa: E402
from paper_1701_03989_amd import problems, sscg  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"
FULL = sscg.FMT_COL16 | sscg.FMT_VTAB
SDIA = FULL | sscg.FMT_SDIA
SDP = SDIA | sscg.FMT_SDPAIR
SDV = SDP | sscg.FMT_SDVAL
ALL_FORMS = sscg.FMT_COL16 | sscg.FMT_VTAB | sscg.FMT_SDIA | sscg.FMT_SDPAIR | sscg.FMT_SDVAL


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


def csr_of(n, rows, cols, vals):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return problems.CSR(rowptr.astype(np.int32), cols[order].astype(np.int32),
                        np.asarray(vals, dtype=np.float64)[order])


def slice_valued(n, seed, lens, band, nvals):
    """Row i: lens[i] distinct columns within `band` of i (cyclic), each value
    drawn from the nvals values of row i's 64-row slice."""
    rng = np.random.default_rng(seed)
    tab = rng.standard_normal(((n + 63) // 64, nvals))
    rows, cols, vals = [], [], []
    for i in range(n):
        k = int(lens[i])
        off = rng.choice(2 * band + 1, size=k, replace=False) - band
        rows.append(np.full(k, i))
        cols.append((i + off) % n)
        vals.append(tab[i // 64, rng.integers(0, nvals, size=k)])
    return csr_of(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def ring(n, seed, sigma=0.05):
    """Weighted ring Laplacian + sigma I, edge (i, i+1 mod n) weighted by
    c[i // 64]: every row has three entries and every slice four values."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.5, 2.0, size=(n + 63) // 64)
    i = np.arange(n)
    wr = c[i // 64]
    wl = c[((i - 1) % n) // 64]
    rows = np.concatenate([i, i, i])
    cols = np.concatenate([i, (i + 1) % n, (i - 1) % n])
    vals = np.concatenate([wl + wr + sigma, -wr, -wl])
    return csr_of(n, rows, cols, vals), sigma, 4.0 * c.max() + sigma


def block_diag(A, B):
    n = A.n + B.n
    ra = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    rb = np.repeat(np.arange(B.n), np.diff(B.rowptr)) + A.n
    return csr_of(n, np.concatenate([ra, rb]),
                  np.concatenate([A.col, B.col.astype(np.int64) + A.n]),
                  np.concatenate([A.val, B.val]))


def nine_point(N):
    """2-D 9-point stencil on N x N (Dirichlet): 9 column distances per row."""
    rows, cols, vals = [], [], []
    for y in range(N):
        for x in range(N):
            i = y * N + x
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if 0 <= x + dx < N and 0 <= y + dy < N:
                        rows.append(i)
                        cols.append((y + dy) * N + x + dx)
                        vals.append(8.0 if dx == dy == 0 else -1.0)
    return csr_of(N * N, rows, cols, vals)


def with_duplicate(A):
    """A with row 70's diagonal split into two entries of the same column (the
    CSR sum is unchanged in exact arithmetic; both entries are products)."""
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    k = int(A.rowptr[70]) + int(np.nonzero(A.col[A.rowptr[70]:A.rowptr[71]] == 70)[0][0])
    half = A.val[k] / 2.0
    val = A.val.copy()
    val[k] = half
    rowptr = A.rowptr.copy()
    rowptr[71:] += 1
    col = np.insert(A.col, k + 1, 70)
    val = np.insert(val, k + 1, half)
    del rows
    return problems.CSR(rowptr, col.astype(np.int32), val)


def with_explicit_zero(A, i):
    """A with an explicitly stored 0.0 at (i, i + 2) and (i + 2, i)."""
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr)).tolist() + [i, i + 2]
    cols = A.col.tolist() + [i + 2, i]
    vals = A.val.tolist() + [0.0, 0.0]
    return csr_of(A.n, rows, cols, vals)


def far_ring(n=33000):
    """Cyclic tridiagonal block: row 0 holds column n - 1, beyond 16 bits."""
    A, _, _ = ring(n, 5)
    return A


def mpk(ctx, A, s, p, r, lmin, lmax, basis="chebyshev", first=False):
    n = A.n
    ld = (n + 63) // 64 * 64
    rcol = s + 1
    ncol = s + 1 if first else 2 * s + 1
    Y = torch.zeros(ncol * ld, dtype=torch.float64, device=DEV)
    Y[:n] = dvec(p)
    if not first:
        Y[rcol * ld: rcol * ld + n] = dvec(r)
    code = sscg.BASIS_CHEBYSHEV if basis == "chebyshev" else sscg.BASIS_MONOMIAL
    sscg.sscg_mpk(ctx, sscg.DeviceCsr.from_host(A, DEV), s, first, code, lmin, lmax, Y, ld, rcol)
    Yh = host(Y)
    return [Yh[c * ld: c * ld + n] for c in range(ncol)]


def oracle_basis(A, s, p, r, lmin, lmax, basis="chebyshev", first=False):
    ar = CR()
    prm = sstep.basis_params(basis, s, lmin, lmax, ar)
    return sstep.krylov_basis(ar, A, p, r, s, first, prm)


def slice_tables(A):
    """Per 64-row slice: its sorted column distances and the sorted bit
    patterns of its stored values (the slice-diagonal form's tables)."""
    out = []
    for t in range((A.n + 63) // 64):
        ds, vs = set(), set()
        for i in range(64 * t, min(A.n, 64 * t + 64)):
            for k in range(int(A.rowptr[i]), int(A.rowptr[i + 1])):
                ds.add(int(A.col[k]) - i)
                vs.add(np.float64(A.val[k]).tobytes())
        out.append((tuple(sorted(ds)), tuple(sorted(vs))))
    return out


def pairs_agree(A):
    """Whether slices 2t and 2t + 1 have the same tables for every t (the
    condition of the paired pass)."""
    t = slice_tables(A)
    return all(t[2 * i] == t[2 * i + 1] for i in range(len(t) // 2))


def values_per_distance(A):
    """(uniform, pairs): whether in every slice all rows with an entry at one
    distance have the same value there (the condition of the pass that keeps
    each distance's value in scalar registers), and whether slices 2t and
    2t + 1 then agree on those values (needed to take them in pairs)."""
    per = []
    for t in range((A.n + 63) // 64):
        m = {}
        for i in range(64 * t, min(A.n, 64 * t + 64)):
            for k in range(int(A.rowptr[i]), int(A.rowptr[i + 1])):
                m.setdefault(int(A.col[k]) - i, set()).add(np.float64(A.val[k]).tobytes())
        if any(len(v) > 1 for v in m.values()):
            return False, False
        per.append(m)
    return True, all(per[2 * i] == per[2 * i + 1] for i in range(len(per) // 2))


def expected_sd_format(A):
    """The slice-diagonal format bits the library must choose for A (which
    has the slice-diagonal form), from the host's own reading of A."""
    uniform, vpairs = values_per_distance(A)
    paired = pairs_agree(A) and (not uniform or vpairs)
    return SDIA | (sscg.FMT_SDPAIR if paired else 0) | (sscg.FMT_SDVAL if uniform else 0)


def laplace1d(n):
    return problems._stencil_csr((n,), 2.0)


def laplace1d_alternating(n):
    """Tridiagonal with diagonal 2 on even rows and 2.5 on odd ones: every
    pair of slices agrees, but distance 0 has two values in each slice."""
    i = np.arange(n)
    lo, hi = i > 0, i < n - 1
    rows = np.concatenate([i, i[lo], i[hi]])
    cols = np.concatenate([i, i[lo] - 1, i[hi] + 1])
    vals = np.concatenate([2.0 + 0.5 * (i % 2), np.full(lo.sum(), -1.0), np.full(hi.sum(), -1.0)])
    return csr_of(n, rows, cols, vals)


def pair_weighted(n, seed):
    """Tridiagonal, row i scaled by c[i // 128] (+ 0.1 on the diagonal):
    values change from one pair of slices to the next and agree within it."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.5, 2.0, size=(n + 127) // 128)
    i = np.arange(n)
    ci = c[i // 128]
    lo, hi = i > 0, i < n - 1
    rows = np.concatenate([i, i[lo], i[hi]])
    cols = np.concatenate([i, i[lo] - 1, i[hi] + 1])
    vals = np.concatenate([2.0 * ci + 0.1, -ci[lo], -ci[hi]])
    return csr_of(n, rows, cols, vals)


def check_against_oracle(got, A, s, p, r, lmin, lmax, what, basis="chebyshev", first=False):
    ref = oracle_basis(A, s, p, r, lmin, lmax, basis, first)
    worst, exact = 0.0, 0
    for g, o in zip(got, ref):
        worst = max(worst, float((np.abs(g - o) / np.maximum(np.abs(o), 1e-300)).max()))
        exact += int(np.array_equal(g, o))
    say(f"{what}: {exact}/{len(ref)} columns bit-identical, worst rel {worst:.2e}")
    assert worst <= 1e-15, what


S, LMIN, LMAX = 5, 0.5, 4.0


def vecs(n, seed):
    return problems.uniform(n, seed), problems.uniform(n, seed + 1)


def test_forms_chosen_as_documented(ctx):
    n = 64 * 8
    cases = [
        ("4 values per slice, no padding", slice_valued(n, 1, np.full(n, 6), 40, 4), FULL),
        ("3 values + padding, ragged n",
         slice_valued(64 * 7 + 17, 2, np.random.default_rng(2).integers(2, 8, 64 * 7 + 17), 40, 3),
         FULL),
        ("5 values in a slice", slice_valued(n, 3, np.full(n, 6), 40, 5), sscg.FMT_COL16),
        ("column 32999 rows away", far_ring(), 0),
        ("ring, per-slice weights", ring(64 * 8, 4)[0], FULL),
        ("3-D Poisson", problems.poisson3d(12), SDIA | sscg.FMT_SDVAL),
        ("3-D Poisson, planes of 4 slices", problems.poisson3d(16), SDV),
        ("2-D Poisson, ragged n", problems.poisson2d(25, 41), SDV),
        ("1-D Laplacian, ragged last pair", laplace1d(64 * 7 + 17), SDV),
        ("1-D Laplacian, odd slice count", laplace1d(64 * 8 + 5), SDV),
        ("1-D Laplacian, one-row last slice", laplace1d(64 * 9 + 1), SDIA | sscg.FMT_SDVAL),
        ("1-D, two diagonal values per slice", laplace1d_alternating(64 * 6 + 9), SDP),
        ("weights changing from pair to pair", pair_weighted(64 * 6 + 9, 83), SDV),
        ("9-point stencil: 9 distances", nine_point(20), FULL),
        ("a repeated column in a row", with_duplicate(problems.poisson2d(16)), FULL),
        ("graph Laplacian", problems.graph_laplacian(3001, 7), sscg.FMT_COL16),
    ]
    for what, A, want in cases:
        f, stored = sscg.sscg_matrix_format(ctx, sscg.DeviceCsr.from_host(A, DEV))
        lens = np.diff(A.rowptr)
        nsl = (A.n + 63) // 64
        pad = np.zeros(nsl * 64, dtype=np.int64)
        pad[:A.n] = lens
        want_stored = int(pad.reshape(nsl, 64).max(axis=1).sum()) * 64
        say(f"{what}: n={A.n} format {f} stored {stored}")
        if want & sscg.FMT_SDIA:  # the case's premise, from the host's reading of A
            assert want == expected_sd_format(A), what
        assert f == want, what
        assert stored == want_stored, what


def test_table_form_matches_oracle_and_wider_forms_bitwise(ctx):
    A = slice_valued(64 * 48, 11, np.full(64 * 48, 6), 60, 4)
    B = slice_valued(64 * 4, 12, np.full(64 * 4, 6), 20, 5)
    D1 = block_diag(A, B)
    D2 = block_diag(A, far_ring())
    fmts = [sscg.sscg_matrix_format(ctx, sscg.DeviceCsr.from_host(M, DEV))[0] for M in (A, D1, D2)]
    assert fmts == [FULL, sscg.FMT_COL16, 0]
    p, r = vecs(A.n, 21)
    ya = mpk(ctx, A, S, p, r, LMIN, LMAX)
    check_against_oracle(ya, A, S, p, r, LMIN, LMAX, "value tables")
    for D, what in [(D1, "16-bit offsets, stored values"), (D2, "32-bit indices")]:
        pe, re_ = vecs(D.n, 31)
        pe[:A.n], re_[:A.n] = p, r
        yd = mpk(ctx, D, S, pe, re_, LMIN, LMAX)
        for c in range(2 * S + 1):
            assert np.array_equal(yd[c][:A.n], ya[c]), (what, c)
        say(f"{what}: first {A.n} rows bit-identical to the table form")
        check_against_oracle(yd, D, S, pe, re_, LMIN, LMAX, what)


def test_ragged_table_form_with_padding_matches_oracle(ctx):
    n = 64 * 37 + 29
    A = slice_valued(n, 41, np.random.default_rng(41).integers(1, 10, n), 80, 3)
    assert sscg.sscg_matrix_format(ctx, sscg.DeviceCsr.from_host(A, DEV))[0] == FULL
    p, r = vecs(n, 43)
    check_against_oracle(mpk(ctx, A, S, p, r, LMIN, LMAX), A, S, p, r, LMIN, LMAX,
                         "ragged value tables")


@pytest.mark.parametrize("basis", ["monomial", "chebyshev"])
def test_solve_on_per_slice_coefficients_matches_oracle(ctx, basis):
    """Whole adaptive solve (Algorithm 4) on a matrix read through value tables
    whose values differ from slice to slice: same s_k schedule, iterates
    within 1e-12."""
    A, lmin, lmax = ring(64 * 40, 51)
    assert sscg.sscg_matrix_format(ctx, sscg.DeviceCsr.from_host(A, DEV))[0] == FULL
    b = problems.uniform(A.n, 52)
    x1 = np.zeros(A.n)
    kw = dict(mode="adaptive", s_max=8, tol=1e-11, basis=basis)
    if basis == "chebyshev":
        kw.update(lmin=lmin, lmax=lmax)
    ref = sstep.solve(A, b, x1, sstep.Opts(**kw))
    x = dvec(x1)
    hist = sscg.History(4096, kw["s_max"])
    rc = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(A, DEV), dvec(b), x, sscg.make_opts(**kw),
                         hist)
    xh = host(x)
    say(f"ring {basis}: gpu {hist.blocks} blocks {hist.schedule[:12]}, oracle {len(ref.blocks)}")
    assert rc == ref.status == sscg.OK
    assert hist.schedule == ref.schedule
    assert np.linalg.norm(xh - ref.x) <= 1e-12 * np.linalg.norm(ref.x)


def test_fp32_pass_table_form_matches_wider_forms_bitwise(ctx):
    """The FP32 matrix-powers pass of the mixed-precision solve reads the same
    three forms (its values rounded from the FP64 tables or from the stored
    values): the rows of the first block agree to the last bit."""
    A = slice_valued(64 * 48, 11, np.full(64 * 48, 6), 60, 4)
    B = slice_valued(64 * 4, 12, np.full(64 * 4, 6), 20, 5)
    pa, ra = vecs(A.n, 21)
    outs = []
    for M in (A, block_diag(A, B), block_diag(A, far_ring())):
        n = M.n
        ld = (n + 63) // 64 * 64
        rcol = S + 1
        p, r = vecs(n, 31)
        p[:A.n], r[:A.n] = pa, ra
        Y = torch.zeros((2 * S + 1) * ld, dtype=torch.float32, device=DEV)
        Y[:n] = torch.as_tensor(p.astype(np.float32), device=DEV)
        Y[rcol * ld: rcol * ld + n] = torch.as_tensor(r.astype(np.float32), device=DEV)
        sscg.sscg_mpk32(ctx, sscg.DeviceCsr.from_host(M, DEV), S, False, sscg.BASIS_CHEBYSHEV,
                        LMIN, LMAX, Y, ld, rcol)
        Yh = host(Y)
        outs.append([Yh[c * ld: c * ld + A.n] for c in range(2 * S + 1)])
    assert all(np.isfinite(c).all() for c in outs[0])
    for k, other in enumerate(outs[1:]):
        for c in range(2 * S + 1):
            assert np.array_equal(other[c], outs[0][c]), (k, c)
    say("FP32 pass: table, 16-bit and 32-bit forms bit-identical on the first block")


SD_CASES = {
    "poisson3d_12": lambda: problems.poisson3d(12),
    "poisson2d_25x41": lambda: problems.poisson2d(25, 41),
    "poisson2d_explicit_zero": lambda: with_explicit_zero(problems.poisson2d(24), 100),
    "poisson3d_9": lambda: problems.poisson3d(9),
    "poisson3d_20": lambda: problems.poisson3d(20),
    "poisson2d_256x9": lambda: problems.poisson2d(256, 9),
    "poisson3d_16": lambda: problems.poisson3d(16),
    "poisson2d_128x9": lambda: problems.poisson2d(128, 9),
    "laplace1d_465": lambda: laplace1d(64 * 7 + 17),
    "laplace1d_517": lambda: laplace1d(64 * 8 + 5),
    "pair_weighted_1400": lambda: pair_weighted(1400, 81),
    "pair_weighted_2": lambda: pair_weighted(2, 82),
    "laplace1d_alternating_1289": lambda: laplace1d_alternating(64 * 20 + 9),
}


@pytest.mark.parametrize("name", list(SD_CASES))
def test_slice_diagonal_form_matches_oracle_and_other_forms_bitwise(ctx, name):
    """The slice-diagonal form, taken one slice or (where consecutive slices
    agree) two slices per wavefront, against the oracle's row sums and
    against the value-table, 16-bit and 32-bit forms of the same matrix
    (sscg_set_forms), bit for bit: two-sequence Chebyshev passes, ragged last
    slice, a stored explicit zero among three values; distances of 400 rows
    (20^3) and 256 rows (256 x 9); for the paired pass an odd slice count, a
    ragged last pair, boundary pairs whose neighbours leave [0, n), values
    that change from pair to pair, and n = 2."""
    A = SD_CASES[name]()
    p, r = vecs(A.n, 61)
    uniform, vpairs = values_per_distance(A)
    paired_any = pairs_agree(A)  # pairs taken when the values are decoded per row
    outs = {}
    try:
        for forms in (ALL_FORMS, ALL_FORMS & ~sscg.FMT_SDVAL, ALL_FORMS & ~sscg.FMT_SDPAIR,
                      ALL_FORMS & ~(sscg.FMT_SDVAL | sscg.FMT_SDPAIR),
                      sscg.FMT_COL16 | sscg.FMT_VTAB, sscg.FMT_COL16, 0):
            sscg.sscg_set_forms(ctx, forms)
            f, _ = sscg.sscg_matrix_format(ctx, sscg.DeviceCsr.from_host(A, DEV))
            outs[f] = mpk(ctx, A, S, p, r, LMIN, LMAX)
    finally:
        sscg.sscg_set_forms(ctx, ALL_FORMS)
    # ALL, ALL without per-distance values, ALL without pairs, neither; the plain forms
    want = {expected_sd_format(A), SDP if paired_any else SDIA,
            SDIA | (sscg.FMT_SDVAL if uniform else 0), SDIA, FULL, sscg.FMT_COL16, 0}
    want = sorted(want)
    assert sorted(outs) == want or (
        name == "poisson2d_explicit_zero" and sorted(outs) == [f for f in want if f != FULL]), \
        sorted(outs)
    check_against_oracle(outs[SDIA], A, S, p, r, LMIN, LMAX, f"slice-diagonal {name}")
    for f, y in outs.items():
        for c in range(2 * S + 1):
            assert np.array_equal(y[c], outs[SDIA][c]), (name, f, c)
    say(f"{name}: slice-diagonal form bit-identical to forms {sorted(outs)}")


@pytest.mark.parametrize("basis,first", [("monomial", False), ("monomial", True),
                                         ("chebyshev", True)])
@pytest.mark.parametrize("name", ["poisson3d_16", "laplace1d_517", "pair_weighted_1400",
                                  "laplace1d_alternating_1289"])
def test_paired_pass_other_bases_match_oracle_and_single_slices(ctx, name, basis, first):
    """The paired pass's monomial and one-sequence (first block) forms, with
    per-row and per-distance values: the oracle's basis, and the
    one-slice-per-wavefront pass bit for bit."""
    A = SD_CASES[name]()
    assert pairs_agree(A)
    uniform, vpairs = values_per_distance(A)
    assert not uniform or vpairs
    p, r = vecs(A.n, 67)
    outs = {}
    try:
        for forms in (ALL_FORMS, ALL_FORMS & ~sscg.FMT_SDVAL, ALL_FORMS & ~sscg.FMT_SDPAIR):
            sscg.sscg_set_forms(ctx, forms)
            f, _ = sscg.sscg_matrix_format(ctx, sscg.DeviceCsr.from_host(A, DEV))
            outs[f] = mpk(ctx, A, S, p, r, LMIN, LMAX, basis, first)
    finally:
        sscg.sscg_set_forms(ctx, ALL_FORMS)
    assert sorted(outs) == sorted({SDP, SDV if uniform else SDP, SDIA | (sscg.FMT_SDVAL if uniform else 0)})
    check_against_oracle(outs[SDP], A, S, p, r, LMIN, LMAX, f"paired {name} {basis} first={first}",
                         basis, first)
    for f, y in outs.items():
        for a, b in zip(y, outs[SDP]):
            assert np.array_equal(a, b), (name, f)


@pytest.mark.parametrize("N", [14, 16])
def test_slice_diagonal_whole_solve_with_fused_residual(ctx, N):
    """Whole adaptive solves (the first pass of every block also forms the
    true residual through the form) with and without the slice-diagonal
    form, and with and without pairs of slices (16^3: planes of four
    slices): same schedule, same bits, and the oracle's iterates."""
    A = problems.poisson3d(N)
    b = problems.uniform(A.n, 71)
    x1 = np.zeros(A.n)
    kw = dict(mode="adaptive", s_max=10, tol=1e-12, basis="chebyshev", lmin=0.05, lmax=12.0)
    ref = sstep.solve(A, b, x1, sstep.Opts(**kw))
    xs = []
    try:
        for forms in (ALL_FORMS, ALL_FORMS & ~sscg.FMT_SDVAL, ALL_FORMS & ~sscg.FMT_SDPAIR,
                      sscg.FMT_COL16 | sscg.FMT_VTAB):
            sscg.sscg_set_forms(ctx, forms)
            x = dvec(x1)
            hist = sscg.History(4096, 10)
            rc = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(A, DEV), dvec(b), x,
                                 sscg.make_opts(**kw), hist)
            assert rc == ref.status == sscg.OK and hist.schedule == ref.schedule
            xs.append(host(x))
    finally:
        sscg.sscg_set_forms(ctx, ALL_FORMS)
    assert all(np.array_equal(xs[0], x) for x in xs[1:])
    assert np.linalg.norm(xs[0] - ref.x) <= 1e-12 * np.linalg.norm(ref.x)


def test_set_forms_rejects_unknown_bits(ctx):
    with pytest.raises(sscg.SscgError):
        sscg.sscg_set_forms(ctx, 32)
