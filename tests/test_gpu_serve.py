"""The solve server (continuous batching) through the C ABI: every request's
result must be the one sscg_solve gives for that system alone (same bits,
schedule length and status), whatever else shares the device with it, however
requests arrive, and however tight the pools are; and, against the CPU oracle
(Algorithm 4 in FP64), the same s_k schedule and iterates within 1e-12."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sstep  # noqa: E402
from paper_1701_03989_amd import problems, sscg  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"
KW = dict(mode="adaptive", basis="chebyshev", s_max=8, tol=1e-10)


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


def alone(ctx, s, tol):
    x = dvec(np.zeros(s.A.n))
    h = sscg.History(1024, 8)
    kw = dict(KW, tol=tol, lmin=s.lmin, lmax=s.lmax)
    rc = sscg.sscg_solve(ctx, sscg.DeviceCsr.from_host(s.A, DEV), dvec(s.b), x,
                         sscg.make_opts(**kw), h)
    return rc, x.cpu().numpy(), h.blocks


class Client:
    """Keeps every request's device buffers alive until it is checked."""

    def __init__(self, ctx, srv):
        self.ctx, self.srv, self.live = ctx, srv, {}

    def submit(self, s, tol):
        A = sscg.DeviceCsr.from_host(s.A, DEV)
        b, x = dvec(s.b), dvec(np.zeros(s.A.n))
        rid = sscg.sscg_server_submit(self.ctx, self.srv, A, b, x, tol, s.lmin, s.lmax)
        self.live[rid] = (s, tol, A, b, x)
        return rid

    def step(self):
        return sscg.sscg_server_step(self.ctx, self.srv)

    def drain(self, limit=5000):
        for _ in range(limit):
            run, q, _ = self.step()
            if run == 0 and q == 0:
                return
        raise AssertionError("server did not drain")

    def check_all(self):
        for rid, (s, tol, _, _, x) in self.live.items():
            p = sscg.sscg_server_poll(self.ctx, self.srv, rid)
            assert p["state"] == 2, (rid, p)
            rc, xa, blocks = alone(self.ctx, s, tol)
            assert p["status"] == rc and p["blocks"] == blocks, (rid, p, rc, blocks)
            assert np.array_equal(x.cpu().numpy(), xa), (rid, s.kind)

    def check_oracle(self):
        """Each served request against the oracle's Algorithm 4 with the same
        tolerance and interval: status, s_k schedule, s~_k, and x within 1e-12."""
        for rid, (s, tol, _, _, x) in self.live.items():
            p = sscg.sscg_server_poll(self.ctx, self.srv, rid)
            h = sscg.sscg_server_history(self.ctx, self.srv, rid)
            ref = sstep.solve(s.A, s.b, np.zeros(s.A.n),
                              sstep.Opts(**dict(KW, tol=tol, lmin=s.lmin, lmax=s.lmax)))
            xh = x.cpu().numpy()
            err = np.linalg.norm(xh - ref.x) / np.linalg.norm(ref.x)
            say(f"  request {rid} ({s.kind}, n={s.A.n}, tol {tol:g}): {len(h['s_k'])} blocks, "
                f"oracle {len(ref.blocks)}; error vs oracle {err:.1e}")
            assert p["status"] == ref.status
            assert h["s_k"] == ref.schedule
            assert h["s_tilde"] == [blk.s_tilde for blk in ref.blocks]
            assert err <= 1e-12


def make_server(ctx, rows=1 << 16, nnz=1 << 20, slots=64):
    return sscg.sscg_server_create(ctx, sscg.make_opts(**KW), rows, nnz, slots)


def test_server_results_equal_alone(ctx):
    systems = problems.batch_systems(6, seed=51, nlo=200, nhi=4000)
    srv = make_server(ctx)
    try:
        cl = Client(ctx, srv)
        for s in systems:
            cl.submit(s, 1e-10)
        say("server: all at once", [s.kind for s in systems])
        cl.drain()
        cl.check_all()
        st = sscg.sscg_server_stats(ctx, srv)
        # every replay ran some admitted rows, at most the pool's
        assert st["replays"] >= 1
        assert 0 < st["rows_active"] <= st["replays"] * (1 << 16)
    finally:
        sscg.sscg_server_destroy(srv)


def test_server_staggered_arrivals_and_tolerances(ctx):
    systems = problems.batch_systems(7, seed=61, nlo=200, nhi=4000)
    tols = [1e-6, 1e-8, 1e-10, 1e-12, 1e-8, 1e-10, 1e-6]
    srv = make_server(ctx)
    try:
        cl = Client(ctx, srv)
        say("server: staggered")
        order = iter(range(len(systems)))
        for burst, steps in ((2, 3), (2, 2), (3, 1)):
            for _ in range(burst):
                i = next(order)
                cl.submit(systems[i], tols[i])
            for _ in range(steps):
                cl.step()
        cl.drain()
        cl.check_all()
        for rid, (s, tol, *_r) in cl.live.items():
            assert sscg.sscg_server_poll(ctx, srv, rid)["relres"] <= tol
        cl.check_oracle()
    finally:
        sscg.sscg_server_destroy(srv)


def test_server_admission_waits_for_room(ctx):
    """Pools that hold about one request at a time and two slots: requests
    wait for room, all finish, results unchanged."""
    systems = problems.batch_systems(5, seed=71, nlo=1500, nhi=3000)
    npad = max((s.A.n + 1023) // 1024 * 1024 for s in systems)
    srv = make_server(ctx, rows=npad + 1024, nnz=64 * max(s.A.nnz for s in systems), slots=2)
    try:
        cl = Client(ctx, srv)
        for s in systems:
            cl.submit(s, 1e-10)
        say("server: tight pools")
        seen_queue = False
        for _ in range(5000):
            run, q, _ = cl.step()
            seen_queue |= q > 0 and run > 0
            if run == 0 and q == 0:
                break
        assert seen_queue
        cl.check_all()
    finally:
        sscg.sscg_server_destroy(srv)


def test_server_history_requires_a_finished_request(ctx):
    s = problems.batch_systems(1, seed=91, nlo=300, nhi=400)[0]
    srv = make_server(ctx)
    try:
        cl = Client(ctx, srv)
        rid = cl.submit(s, 1e-10)
        with pytest.raises(sscg.SscgError):
            sscg.sscg_server_history(ctx, srv, rid)
        with pytest.raises(sscg.SscgError):
            sscg.sscg_server_history(ctx, srv, rid + 1000)
        cl.drain()
        h = sscg.sscg_server_history(ctx, srv, rid)
        assert len(h["s_k"]) == sscg.sscg_server_poll(ctx, srv, rid)["blocks"] >= 1
        assert h["relres_true"][-1] <= 1e-10
        cl.check_oracle()
    finally:
        sscg.sscg_server_destroy(srv)


def test_server_refuses_what_never_fits(ctx):
    s = problems.batch_systems(1, seed=81, nlo=5000, nhi=6000)[0]
    srv = make_server(ctx, rows=2048, nnz=1 << 16, slots=4)
    try:
        with pytest.raises(sscg.SscgError):
            Client(ctx, srv).submit(s, 1e-10)
    finally:
        sscg.sscg_server_destroy(srv)


def test_server_variable_precision_matches_oracle_and_batch_of_one(ctx):
    """A SSCG_PREC_VARIABLE server: each request has the oracle's schedule,
    s~_k and per-block basis precision (reading R17), x within 1e-12, and the
    bits a batch of that one system gives, however the requests arrive."""
    systems = problems.batch_systems(6, seed=71, nlo=300, nhi=4000)
    tols = [1e-6, 1e-10, 1e-8, 1e-12, 1e-10, 1e-6]
    kwv = dict(KW, precision="variable")
    srv = sscg.sscg_server_create(ctx, sscg.make_opts(**kwv), 1 << 16, 1 << 20, 64)
    try:
        cl = Client(ctx, srv)
        order = iter(range(len(systems)))
        for burst, steps in ((2, 3), (3, 2), (1, 1)):
            for _ in range(burst):
                i = next(order)
                cl.submit(systems[i], tols[i])
            for _ in range(steps):
                cl.step()
        cl.drain()
        n32 = 0
        for rid, (s, tol, _, _, x) in cl.live.items():
            p = sscg.sscg_server_poll(ctx, srv, rid)
            h = sscg.sscg_server_history(ctx, srv, rid)
            ref = sstep.solve(s.A, s.b, np.zeros(s.A.n),
                              sstep.Opts(**dict(kwv, tol=tol, lmin=s.lmin, lmax=s.lmax)))
            xh = x.cpu().numpy()
            err = np.linalg.norm(xh - ref.x) / np.linalg.norm(ref.x)
            say(f"  request {rid} ({s.kind}, n={s.A.n}, tol {tol:g}): precisions {h['fp32']}; "
                f"error vs oracle {err:.1e}")
            assert p["status"] == ref.status
            assert h["s_k"] == ref.schedule
            assert h["s_tilde"] == [blk.s_tilde for blk in ref.blocks]
            assert h["fp32"] == [int(blk.fp32) for blk in ref.blocks]
            assert err <= 1e-12
            n32 += sum(h["fp32"])
            # the same system as a batch of one
            x1 = dvec(np.zeros(s.A.n))
            hist = sscg.BatchHistory(1, 1024)
            rc = sscg.sscg_batch_solve(ctx, [sscg.DeviceCsr.from_host(s.A, DEV)], [dvec(s.b)],
                                       [x1], sscg.make_opts(**dict(kwv, tol=tol)),
                                       lambda_min=[s.lmin], lambda_max=[s.lmax], hist=hist)
            assert rc == p["status"]
            assert np.array_equal(x1.cpu().numpy(), xh)
        assert n32 > 0
    finally:
        sscg.sscg_server_destroy(srv)
