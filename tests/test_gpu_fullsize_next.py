"""Parity at the full sizes of the batch, precision and serving workloads.

* 256 uneven systems (rows log-uniform in [1e3, 2e5], 11.6 M rows in all,
  generated exactly as bench.py's batch workload): every true relative
  residual below 1e-10 (recomputed on the host), sampled systems bit for bit
  equal to sscg_solve alone, the two smallest against the oracle's full solves.
* Variable-coefficient diffusion 2048^2 (n = 4,194,304), equilibrated: the
  interval estimate and the first two FP64 outer blocks against the oracle;
  the FP32 matrix-powers pass against its definition, bit for bit, over all
  4.2 M rows; the mixed-precision solve reaches its tolerance.
* Serving, operators of 1e4 to 4e6 rows: each request's result equals
  sscg_solve alone, bit for bit, and meets its tolerance.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mixed, spectral, sstep  # noqa: E402
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


def relres(A, b, x):
    """||b - A x|| / ||b|| with every row of the residual and both sums
    correctly rounded (the oracle's arithmetic)."""
    ar = CR()
    return float(sstep.relres_of(ar, A, np.asarray(b, float), np.asarray(x, float),
                                 ar.sqrt(ar.dot(np.asarray(b, float), np.asarray(b, float)))))


def single(ctx, s, **kw):
    x = dvec(np.zeros(s.A.n))
    h = sscg.History(4096, kw.get("s_max", 8))
    rc = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(s.A, DEV), dvec(s.b), x,
                         sscg.make_opts(**kw), h)
    torch.cuda.synchronize()
    return rc, x.cpu().numpy(), h


def test_batch256_fullsize(ctx):
    kw = dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10)
    systems = problems.batch_systems(256, seed=0)
    say(f"batch of {len(systems)} systems, {sum(s.A.n for s in systems)} rows")
    devA = [sscg.DeviceCsr.from_host(s.A, DEV) for s in systems]
    bs = [dvec(s.b) for s in systems]
    xs = [dvec(np.zeros(s.A.n)) for s in systems]
    hist = sscg.BatchHistory(len(systems), 4096)
    rc = sscg.sscg_batch_solve(ctx, devA, bs, xs, sscg.make_opts(**kw),
                               lambda_min=[s.lmin for s in systems],
                               lambda_max=[s.lmax for s in systems], hist=hist)
    torch.cuda.synchronize()
    assert rc == sscg.OK
    xh = [x.cpu().numpy() for x in xs]
    worst = max(relres(s.A, s.b, x) for s, x in zip(systems, xh))
    say(f"  worst host relres {worst:.3e}, replays {hist.res.graph_launches}")
    assert worst <= kw["tol"]
    sizes = [s.A.n for s in systems]
    order = np.argsort(sizes)
    rng = np.random.default_rng(5)
    sample = sorted({int(order[0]), int(order[1]), int(order[-1])}
                    | set(int(v) for v in rng.choice(len(systems), 4, replace=False)))
    for i in sample:
        s = systems[i]
        rc1, x1, h1 = single(ctx, s, lmin=s.lmin, lmax=s.lmax, **kw)
        say(f"  system {i} ({s.kind}, n={s.A.n}): {h1.blocks} blocks alone, "
            f"{int(hist.blocks[i])} in the batch")
        assert rc1 == int(hist.status[i]) and h1.schedule == hist.schedule(i)
        assert np.array_equal(x1, xh[i]), i
    for i in (int(order[0]), int(order[1])):
        s = systems[i]
        ref = sstep.solve(s.A, s.b, np.zeros(s.A.n), sstep.Opts(lmin=s.lmin, lmax=s.lmax, **kw))
        err = np.linalg.norm(xh[i] - ref.x) / np.linalg.norm(ref.x)
        say(f"  system {i} vs the oracle: schedule equal {hist.schedule(i) == ref.schedule}, "
            f"error {err:.1e}")
        assert hist.schedule(i) == ref.schedule and err <= 1e-12


@pytest.fixture(scope="module")
def diffusion():
    return problems.diffusion2d_system(2048, 0)


def test_diffusion2048_fp64_first_blocks(ctx, diffusion):
    A, b, x1 = diffusion
    kw = dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10, equilibrate=True)
    As, _ = sstep.equilibrate(A)
    say(f"diffusion 2048^2: n={A.n} nnz={A.nnz}; oracle interval of the scaled matrix")
    lo, hi = spectral.chebyshev_interval(As, 30, 0)
    # the device's own estimate (what an unspecified interval uses): the same bits
    x = dvec(x1)
    h0 = sscg.History(16, 8)
    sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(A, DEV), dvec(b), x,
                    sscg.make_opts(max_iters=1, **kw), h0)
    say(f"  device [{h0.res.lambda_min!r}, {h0.res.lambda_max!r}] oracle [{lo!r}, {hi!r}]")
    assert h0.res.lambda_min == lo and h0.res.lambda_max == hi
    kb = dict(kw, lmin=lo, lmax=hi, max_iters=16)
    say("  first two blocks: oracle")
    ref = sstep.solve(A, b, x1, sstep.Opts(**kb))
    say("  first two blocks: device")
    x = dvec(x1)
    h = sscg.History(16, 8)
    rc = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(A, DEV), dvec(b), x, sscg.make_opts(**kb),
                         h)
    xh = x.cpu().numpy()
    say(f"  device {h.schedule} oracle {ref.schedule}")
    assert rc == ref.status and h.schedule == ref.schedule
    for k, blk in enumerate(ref.blocks):
        assert h.kappas(k)[: len(blk.kappas)] == blk.kappas and h.thr[k] == blk.thr
    err = np.linalg.norm(xh - ref.x) / np.linalg.norm(ref.x)
    say(f"  |x - x_oracle| / |x_oracle| = {err:.2e}")
    assert err <= 1e-12


def test_diffusion2048_fp32_pass_and_mixed_solve(ctx, diffusion):
    A, b, x1 = diffusion
    n, s = A.n, 8
    lmin, lmax = 1e-3, float(np.max(np.abs(A.val)) * 5)
    ld = (n + 63) // 64 * 64
    rcol = s + 1
    p0 = problems.uniform(n, 3).astype(np.float32)
    r0 = problems.uniform(n, 4).astype(np.float32)
    Y = torch.zeros((2 * s + 1) * ld, dtype=torch.float32, device=DEV)
    Y[:n] = torch.as_tensor(p0, device=DEV)
    Y[rcol * ld:rcol * ld + n] = torch.as_tensor(r0, device=DEV)
    say("diffusion 2048^2: FP32 matrix-powers pass over all rows")
    sscg.sscg_mpk32(ctx, sscg.DeviceCsr.from_host(A, DEV), s, False, sscg.BASIS_CHEBYSHEV, lmin,
                    lmax, Y, ld, rcol)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy()
    P, R = mixed.mpk32_basis(A, s, False, "chebyshev", p0, r0, lmin, lmax)
    for j in range(1, s + 1):
        assert np.array_equal(Yh[j * ld:j * ld + n], P[j]), ("P", j)
    for j in range(1, s):
        assert np.array_equal(Yh[(rcol + j) * ld:(rcol + j) * ld + n], R[j]), ("R", j)
    say("  mixed-precision solve")
    kw = dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10, equilibrate=True,
              precision="mixed")
    x = dvec(x1)
    h = sscg.History(1 << 14, 8)
    rc = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(A, DEV), dvec(b), x, sscg.make_opts(**kw),
                         h)
    xh = x.cpu().numpy()
    dmax = np.maximum.reduceat(np.abs(A.val), A.rowptr[:-1])  # D_i = max_j |a_ij| (no empty rows)
    rel = relres(A, b, xh)
    say(f"  status {rc}, blocks {h.blocks}, iterations {h.res.iters}, host relres {rel:.2e} "
        f"(device {h.res.relres:.2e}, max D / min D = {dmax.max() / dmax.min():.2e})")
    # the refinement stops on A x = b itself: relres <= tol on the caller's system
    assert rc == sscg.OK and h.res.relres <= kw["tol"]
    assert rel <= kw["tol"] * (1 + 1e-6)


def test_serving_fullsize_operators(ctx):
    ops = problems.batch_systems(6, seed=100, nlo=1e4, nhi=4e6)
    tols = [1e-6, 1e-8, 1e-10, 1e-12]
    rng = np.random.default_rng(7)
    reqs = [(int(rng.integers(0, len(ops))), tols[int(rng.integers(0, 4))]) for _ in range(8)]
    say(f"serving: operators {[s.A.n for s in ops]}, requests {reqs}")
    kw = dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10)
    srv = sscg.sscg_server_create(ctx, sscg.make_opts(**kw), 24 << 20, 160 << 20, 64)
    try:
        live = []
        devA = [sscg.DeviceCsr.from_host(s.A, DEV) for s in ops]
        for k, (w, tol) in enumerate(reqs):
            s = ops[w]
            b, x = dvec(s.b), dvec(np.zeros(s.A.n))
            rid = sscg.sscg_server_submit(ctx, srv, devA[w], b, x, tol, s.lmin, s.lmax)
            live.append((rid, w, tol, b, x))
            for _ in range(3):  # staggered arrivals: a few blocks between requests
                sscg.sscg_server_step(ctx, srv)
        for _ in range(200000):
            run, q, _ = sscg.sscg_server_step(ctx, srv)
            if run == 0 and q == 0:
                break
        for rid, w, tol, b, x in live:
            p = sscg.sscg_server_poll(ctx, srv, rid)
            s = ops[w]
            rc1, x1, h1 = single(ctx, s, lmin=s.lmin, lmax=s.lmax, **dict(kw, tol=tol))
            xh = x.cpu().numpy()
            say(f"  request {rid}: n={s.A.n} tol={tol:g} status {p['status']} blocks "
                f"{p['blocks']} (alone {h1.blocks})")
            assert p["state"] == 2 and p["status"] == rc1 == sscg.OK and p["blocks"] == h1.blocks
            assert np.array_equal(xh, x1)
            assert relres(s.A, s.b, xh) <= tol
    finally:
        sscg.sscg_server_destroy(srv)
