"""Batched solves (sscg_batch_solve) against the CPU oracle and against the
single-system path, through the C ABI.

Every system of a batch must give what the oracle gives for it alone (same
s_k schedule, iterates within 1e-12 relative, same status), and the same bits
as sscg_solve on that system alone and as a batch of one: a system's result
does not depend on the rest of the batch.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sstep  # noqa: E402
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


def run_batch(ctx, systems, x1s=None, tols=None, cap=512, **kw):
    devA = [sscg.DeviceCsr.from_host(s.A, DEV) for s in systems]
    bs = [dvec(s.b) for s in systems]
    xs = [dvec(np.zeros(s.A.n) if x1s is None else x1s[i]) for i, s in enumerate(systems)]
    hist = sscg.BatchHistory(len(systems), cap)
    cheb = kw.get("basis") == "chebyshev"
    rc = sscg.sscg_batch_solve(ctx, devA, bs, xs, sscg.make_opts(**kw), tol=tols,
                               lambda_min=[s.lmin for s in systems] if cheb else None,
                               lambda_max=[s.lmax for s in systems] if cheb else None, hist=hist)
    torch.cuda.synchronize()
    return rc, [x.cpu().numpy() for x in xs], hist


def oracle_opts(kw, s, tol=None):
    o = dict(kw)
    if o.get("basis") == "chebyshev":
        o["lmin"], o["lmax"] = s.lmin, s.lmax
    if tol is not None:
        o["tol"] = tol
    return sstep.Opts(**o)


CASES = [
    dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10),
    dict(mode="adaptive", s_max=6, tol=1e-10, s0_bar=2, f=1),
    dict(mode="fixed", fixed_s=4, s_max=8, tol=1e-10),
    dict(mode="adaptive", s_max=8, tol=1e-10, inner_check=False, c=10.0),
    dict(mode="adaptive", basis="chebyshev", s_max=16, tol=1e-10),  # 33 x 33 sub-Gram matrices
    # growing blocks s = 2, 5, 8, 11, 12: Gram widths 5, 11, 17, 23, 25 (one column
    # block, the split blocking, two full column blocks in one batched launch)
    dict(mode="adaptive", basis="chebyshev", s_max=12, tol=1e-10, s0_bar=2, f=3),
]


@pytest.mark.parametrize("k", range(len(CASES)))
def test_batch_matches_oracle_and_single_path(ctx, k):
    kw = CASES[k]
    systems = problems.batch_systems(6, seed=1 + k, nlo=100, nhi=3000)
    say(f"batch {kw}: {[s.kind for s in systems]}")
    rc, xs, hist = run_batch(ctx, systems, **kw)
    say(f"  status {hist.status.tolist()} blocks {hist.blocks.tolist()} "
        f"replays {hist.res.graph_launches} rows {hist.res.rows}")
    for i, s in enumerate(systems):
        ref = sstep.solve(s.A, s.b, np.zeros(s.A.n), oracle_opts(kw, s))
        sched = hist.schedule(i)
        assert int(hist.status[i]) == ref.status, (i, hist.status[i], ref.status)
        assert sched == ref.schedule, (i, sched[:12], ref.schedule[:12])
        err = np.linalg.norm(xs[i] - ref.x) / np.linalg.norm(ref.x)
        assert err <= 1e-12, (i, err)
        # the single-system path: the same bits
        single_kw = dict(kw)
        if kw.get("basis") == "chebyshev":
            single_kw.update(lmin=s.lmin, lmax=s.lmax)
        x = dvec(np.zeros(s.A.n))
        h1 = sscg.History(512, kw.get("s_max", 8))
        rc1 = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(s.A, DEV), dvec(s.b), x,
                              sscg.make_opts(**single_kw), h1)
        assert rc1 == int(hist.status[i]) and h1.schedule == sched
        assert np.array_equal(x.cpu().numpy(), xs[i]), i
    assert rc == max(int(v) for v in hist.status)


def test_batch_result_independent_of_the_mix(ctx):
    """Each system alone (a batch of one) and in the mix: identical bits."""
    kw = dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10)
    systems = problems.batch_systems(5, seed=11, nlo=200, nhi=2000)
    say("mix vs alone")
    _, xs, hist = run_batch(ctx, systems, **kw)
    for i, s in enumerate(systems):
        _, x1, h1 = run_batch(ctx, [s], **kw)
        assert h1.schedule(0) == hist.schedule(i)
        assert np.array_equal(x1[0], xs[i]), i


def test_batch_per_system_tolerances_and_degenerate_systems(ctx):
    kw = dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10)
    systems = problems.batch_systems(4, seed=21, nlo=200, nhi=1500)
    tols = [1e-6, 1e-8, 1e-10, 1e-12]
    x1s = [np.zeros(s.A.n) for s in systems]
    # system 1: zero right-hand side; system 2: x_1 already solves it exactly
    systems[1].b = np.zeros(systems[1].A.n)
    xt = problems.uniform(systems[2].A.n, 5)
    x1s[2] = xt
    systems[2].b = systems[2].A.matvec(xt)
    say("tolerances / degenerate")
    rc, xs, hist = run_batch(ctx, systems, x1s=x1s, tols=tols, **kw)
    assert rc == sscg.OK and all(int(v) == sscg.OK for v in hist.status)
    assert np.all(xs[1] == 0.0) and hist.blocks[1] == 0
    for i in (0, 3):
        s = systems[i]
        ref = sstep.solve(s.A, s.b, np.zeros(s.A.n), oracle_opts(kw, s, tol=tols[i]))
        assert hist.schedule(i) == ref.schedule
        assert np.linalg.norm(xs[i] - ref.x) <= 1e-12 * np.linalg.norm(ref.x)
        assert hist.relres[i] <= tols[i]
    ref = sstep.solve(systems[2].A, systems[2].b, xt, oracle_opts(kw, systems[2], tol=tols[2]))
    assert hist.blocks[2] == len(ref.blocks) and np.array_equal(xs[2], ref.x)


def test_batch_iteration_cap(ctx):
    kw = dict(mode="adaptive", basis="chebyshev", s_max=4, tol=1e-14, max_iters=9)
    systems = problems.batch_systems(3, seed=31, nlo=500, nhi=2000)
    rc, xs, hist = run_batch(ctx, systems, **kw)
    for i, s in enumerate(systems):
        ref = sstep.solve(s.A, s.b, np.zeros(s.A.n), oracle_opts(kw, s))
        assert int(hist.status[i]) == ref.status == sscg.NOT_CONVERGED
        assert hist.schedule(i) == ref.schedule and int(hist.iters[i]) == sum(ref.schedule)
        assert np.linalg.norm(xs[i] - ref.x) <= 1e-12 * np.linalg.norm(ref.x)


def test_batch_argument_errors(ctx):
    systems = problems.batch_systems(2, seed=41, nlo=100, nhi=300)
    with pytest.raises(sscg.SscgError):
        run_batch(ctx, systems, mode="schedule", schedule=[2])
    with pytest.raises(sscg.SscgError):
        run_batch(ctx, systems, equilibrate=True)
    devA = [sscg.DeviceCsr.from_host(s.A, DEV) for s in systems]
    with pytest.raises(sscg.SscgError):  # Chebyshev without intervals
        sscg.sscg_batch_solve(ctx, devA, [dvec(s.b) for s in systems],
                              [dvec(np.zeros(s.A.n)) for s in systems],
                              sscg.make_opts(basis="chebyshev"))


def _arrow_system(n, seed):
    """SPD arrow matrix: diagonal 4 + U[0,1], first row and column U[-1,1]/sqrt(n),
    so that one row holds n entries and every other row two (rows of very uneven
    length: the batch sorts them within windows)."""
    rng = np.random.default_rng(seed)
    d = 4.0 + rng.uniform(0.0, 1.0, n)
    w = rng.uniform(-1.0, 1.0, n - 1) / np.sqrt(n)
    rows, cols, vals = [0], [0], [d[0]]
    rows += [0] * (n - 1)
    cols += list(range(1, n))
    vals += list(w)
    for i in range(1, n):
        rows += [i, i]
        cols += [0, i]
        vals += [w[i - 1], d[i]]
    rows, cols, vals = np.array(rows), np.array(cols), np.array(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    A = problems.CSR(np.cumsum(rowptr).astype(np.int32), cols.astype(np.int32), vals)
    dense = A.to_scipy().toarray()
    ev = np.linalg.eigvalsh(dense)
    b = rng.uniform(-1.0, 1.0, n)
    return problems.BatchSystem(A, b, 0.9 * ev[0], 1.1 * ev[-1], f"arrow_{n}")


def test_batch_uneven_rows_match_single_path_and_oracle(ctx):
    """Row order and paired gathers: a batch mixing an arrow matrix (one row of
    n entries), a graph Laplacian (scattered columns, uneven degrees) and a
    stencil gives each system the bits sscg_solve gives it in natural order."""
    kw = dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10)
    systems = [_arrow_system(1500, 3)] + problems.batch_systems(4, seed=11, nlo=500, nhi=4000)
    say(f"batch {[s.kind for s in systems]}")
    rc, xs, hist = run_batch(ctx, systems, **kw)
    for i, s in enumerate(systems):
        x = dvec(np.zeros(s.A.n))
        h1 = sscg.History(512, 8)
        rc1 = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(s.A, DEV), dvec(s.b), x,
                              sscg.make_opts(lmin=s.lmin, lmax=s.lmax, **kw), h1)
        say(f"  {s.kind}: status {int(hist.status[i])}/{rc1}, blocks {int(hist.blocks[i])}/{h1.blocks}")
        assert rc1 == int(hist.status[i]) and h1.schedule == hist.schedule(i)
        assert np.array_equal(x.cpu().numpy(), xs[i]), s.kind
        ref = sstep.solve(s.A, s.b, np.zeros(s.A.n), oracle_opts(kw, s))
        err = np.linalg.norm(xs[i] - ref.x) / np.linalg.norm(ref.x)
        assert hist.schedule(i) == ref.schedule and err <= 1e-12, (s.kind, err)


def test_batch_launch_shapes_give_the_same_bits_and_the_tuner_picks_the_fastest(ctx):
    """Every launch shape the batch tuner chooses from (threads per kappa
    problem, wavefronts per Gram workgroup) gives the same bits; the tuner
    times all of them on the live batch, keeps the fastest, and a second
    batch of the same shape reuses that choice without timing again."""
    systems = problems.batch_systems(8, seed=77, nlo=500, nhi=6000)
    kw = CASES[0]

    def bits(rc, xs, hist):
        return (rc, [x.tobytes() for x in xs], hist.blocks.tolist(), hist.status.tolist())

    ref = None
    try:
        shapes = [(kbt, gw, 4) for kbt in (64, 128, 192, 256) for gw in (1, 2, 4)]
        shapes += [(128, 4, 2), (128, 4, 8), (64, 1, 8)]
        for kbt, gw, mch in shapes:
            sscg.sscg_set_batch_tuning(ctx, 0, kbt, gw, mch)
            got = bits(*run_batch(ctx, systems, **kw))
            t = sscg.sscg_batch_tuning(ctx)
            assert (t["kappa_threads"], t["gram_waves"], t["mpk_chunk"]) == (kbt, gw, mch)
            assert np.all(np.isnan(t["kappa_us"])) and np.all(np.isnan(t["gram_us"]))
            if ref is None:
                ref = got
                say(f"  blocks {got[2]}")
            assert got == ref, (kbt, gw, mch)
        sscg.sscg_set_batch_tuning(ctx, 1)
        got = bits(*run_batch(ctx, systems, **kw))
        t = sscg.sscg_batch_tuning(ctx)
        say(f"  tuned: {t}")
        assert got == ref
        assert all(v > 0 for v in t["kappa_us"] + t["gram_us"] + t["mpk_us"])
        assert t["kappa_threads"] == (64, 128, 192, 256)[int(np.argmin(t["kappa_us"]))]
        assert t["gram_waves"] == (1, 2, 4)[int(np.argmin(t["gram_us"]))]
        assert t["mpk_chunk"] == (2, 4, 8)[int(np.argmin(t["mpk_us"]))]
        got2 = bits(*run_batch(ctx, systems, **kw))
        t2 = sscg.sscg_batch_tuning(ctx)
        assert got2 == ref
        assert (t2["kappa_threads"], t2["gram_waves"], t2["mpk_chunk"]) == \
            (t["kappa_threads"], t["gram_waves"], t["mpk_chunk"])
        assert np.all(np.isnan(t2["kappa_us"]))
        for bad in ((2, 0, 0, 0), (0, 100, 4, 4), (0, 128, 3, 4), (0, 128, 4, 3)):
            with pytest.raises(sscg.SscgError):
                sscg.sscg_set_batch_tuning(ctx, *bad)
    finally:
        sscg.sscg_set_batch_tuning(ctx, 1)


def test_batch_variable_precision_matches_oracle_and_each_system_alone(ctx):
    """SSCG_PREC_VARIABLE (reading R17: an FP32 basis in the blocks the
    rearranged eq. fb admits): every system has the oracle's s_k schedule,
    s~_k and per-block precision, x within 1e-12, and the same bits alone in
    a batch of one as in the mix; some blocks are FP32."""
    systems = problems.batch_systems(6, seed=21, nlo=300, nhi=4000)
    tols = [1e-6, 1e-8, 1e-10, 1e-12, 1e-10, 1e-8]
    kw = dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10, precision="variable")
    rc, xs, hist = run_batch(ctx, systems, tols=tols, **kw)
    n32 = 0
    for i, s in enumerate(systems):
        ref = sstep.solve(s.A, s.b, np.zeros(s.A.n), oracle_opts(kw, s, tols[i]))
        prec = hist.precisions(i)
        err = np.linalg.norm(xs[i] - ref.x) / np.linalg.norm(ref.x)
        say(f"  {s.kind} n={s.A.n} tol {tols[i]:g}: precisions {prec}; error vs oracle {err:.1e}")
        assert hist.status[i] == ref.status
        assert hist.schedule(i) == ref.schedule
        assert prec == [int(blk.fp32) for blk in ref.blocks]
        assert err <= 1e-12
        n32 += sum(prec)
        rc1, xs1, h1 = run_batch(ctx, [s], tols=[tols[i]], **kw)
        assert np.array_equal(xs1[0], xs[i]) and h1.precisions(0) == prec
    assert n32 > 0


def test_single_solve_variable_precision_is_the_batch_of_one(ctx):
    """sscg_solve with SSCG_PREC_VARIABLE runs as a batch of one: the same bits,
    schedule and per-block precisions as sscg_batch_solve on that system with
    the same interval; with the interval estimated on the device it reaches
    the tolerance; unsupported combinations are refused."""
    s = problems.batch_systems(1, seed=3, nlo=2000, nhi=4000)[0]
    kw = dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10, precision="variable")
    x = dvec(np.zeros(s.A.n))
    h = sscg.History(1024, 8)
    rc = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(s.A, DEV), dvec(s.b), x,
                         sscg.make_opts(**dict(kw, lmin=s.lmin, lmax=s.lmax)), h)
    rcb, xs, hist = run_batch(ctx, [s], **kw)
    say(f"  {s.kind} n={s.A.n}: precisions {h.fp32[:h.blocks].tolist()}")
    assert rc == rcb and h.blocks == int(hist.blocks[0])
    assert np.array_equal(x.cpu().numpy(), xs[0])
    assert h.schedule == hist.schedule(0)
    assert h.fp32[:h.blocks].tolist() == hist.precisions(0) and sum(hist.precisions(0)) > 0
    h2 = sscg.History(1024, 8)
    x.zero_()
    rc2 = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(s.A, DEV), dvec(s.b), x,
                          sscg.make_opts(**kw), h2)
    xh = x.cpu().numpy()
    assert rc2 == sscg.OK and h2.res.lambda_max > h2.res.lambda_min > 0
    assert np.linalg.norm(s.b - s.A.matvec(xh)) <= 1e-10 * np.linalg.norm(s.b) * (1 + 1e-6)
    with pytest.raises(sscg.SscgError):  # needs the adaptive mode
        run_batch(ctx, [s], mode="fixed", fixed_s=4, s_max=8, tol=1e-10, precision="variable")
    with pytest.raises(sscg.SscgError):  # no equilibration
        sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(s.A, DEV), dvec(s.b), x,
                        sscg.make_opts(**dict(kw, lmin=s.lmin, lmax=s.lmax, equilibrate=True)))
