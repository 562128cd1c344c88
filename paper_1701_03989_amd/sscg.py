"""ctypes binding of libsscg (include/sscg.h): argument marshalling only.

Every function of the C ABI has a Python function of the same name here,
taking torch CUDA tensors (device memory) where the C call takes device
pointers.  All numerical work happens in the HIP kernels of libsscg.so; this
module raises if the library has not been built or no GPU is present.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsscg.so")

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
ERR_ARG, ERR_HIP, ERR_OOM = -1, -2, -3
MODE_ADAPTIVE, MODE_FIXED, MODE_SCHEDULE = 0, 1, 2
BASIS_MONOMIAL, BASIS_CHEBYSHEV, BASIS_NEWTON = 0, 1, 2
FMT_COL16, FMT_VTAB, FMT_SDIA, FMT_SDPAIR, FMT_SDVAL = 1, 2, 4, 8, 16
C_CONST, C_THEORY = 0, 1
PREC_FP64, PREC_MIXED, PREC_VARIABLE = 0, 1, 2
S_LIMIT = 16
FAMILIES = {"mpk": 0, "gram": 1, "recover": 2, "small": 3}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class SscgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sscg error {code}: {msg}")
        self.code = code


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("basis", ctypes.c_int32), ("tol", ctypes.c_double),
                ("s_max", ctypes.c_int32), ("s0_bar", ctypes.c_int32), ("f", ctypes.c_int32),
                ("fixed_s", ctypes.c_int32), ("schedule", _ip), ("schedule_len", ctypes.c_int32),
                ("c", ctypes.c_double), ("lambda_min", ctypes.c_double),
                ("lambda_max", ctypes.c_double), ("lanczos_steps", ctypes.c_int32),
                ("lanczos_seed", ctypes.c_uint64), ("equilibrate", ctypes.c_int32),
                ("inner_check", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("c_mode", ctypes.c_int32), ("kappa_a", ctypes.c_double),
                ("norm_a", ctypes.c_double), ("shifts", _dp),
                ("precision", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("inner_tol", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int32), ("blocks", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("status", ctypes.c_int32), ("relres0", ctypes.c_double),
                ("relres", ctypes.c_double), ("lambda_min", ctypes.c_double),
                ("lambda_max", ctypes.c_double), ("basis_vectors", ctypes.c_int64),
                ("wasted_vectors", ctypes.c_int64), ("s_bar", _ip), ("s_built", _ip),
                ("s_tilde", _ip), ("s_k", _ip), ("gamma", _dp), ("thr", _dp),
                ("res_updated", _dp), ("relres_true", _dp), ("kappa", _dp),
                ("spec_blocks", ctypes.c_int32), ("spec_rejected", ctypes.c_int32),
                ("fp32", _ip)]


class Batch(ctypes.Structure):
    _fields_ = [("nsys", ctypes.c_int32), ("A", ctypes.POINTER(Csr)),
                ("b", ctypes.POINTER(ctypes.c_void_p)), ("x", ctypes.POINTER(ctypes.c_void_p)),
                ("tol", _dp), ("lambda_min", _dp), ("lambda_max", _dp)]


class BatchResult(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int32), ("status", _ip), ("blocks", _ip), ("iters", _ip),
                ("relres", _dp), ("s_k", _ip), ("s_tilde", _ip), ("relres_true", _dp),
                ("graph_launches", ctypes.c_int32), ("rows", ctypes.c_int32), ("fp32", _ip)]


class BlockInfo(ctypes.Structure):
    _fields_ = [("s_tilde", ctypes.c_int32), ("s_k", ctypes.c_int32), ("status", ctypes.c_int32),
                ("d", ctypes.c_int32), ("gamma", ctypes.c_double), ("thr", ctypes.c_double),
                ("rnorm", ctypes.c_double), ("rr", ctypes.c_double),
                ("kappa", ctypes.c_double * S_LIMIT), ("alpha", ctypes.c_double * S_LIMIT),
                ("beta", ctypes.c_double * S_LIMIT), ("rr_trace", ctypes.c_double * S_LIMIT),
                ("relres_in", ctypes.c_double), ("spec", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class BlockParams(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int32), ("first", ctypes.c_int32), ("adaptive", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("inner_check", ctypes.c_int32),
                ("basis", ctypes.c_int32), ("lambda_min", ctypes.c_double),
                ("lambda_max", ctypes.c_double), ("eps_star", ctypes.c_double),
                ("c", ctypes.c_double), ("unit_roundoff", ctypes.c_double),
                ("c_mode", ctypes.c_int32), ("n_a", ctypes.c_int32), ("s_max", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("kappa_a", ctypes.c_double),
                ("norm_a", ctypes.c_double), ("shifts", ctypes.c_double * S_LIMIT)]


_lib = None

EXPORTS = {
    "sscg_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p]),
    "sscg_destroy": (None, [ctypes.c_void_p]),
    "sscg_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "sscg_opts_default": (None, [ctypes.POINTER(Opts)]),
    "sscg_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Csr), ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.POINTER(Opts), ctypes.POINTER(Result)]),
    "sscg_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Csr), ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sscg_spectral_bounds": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Csr), ctypes.c_int,
                                            ctypes.c_uint64, _dp, _dp]),
    "sscg_newton_shifts": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Csr), ctypes.c_int,
                                          ctypes.c_uint64, _dp]),
    "sscg_matrix_format": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Csr),
                                          ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int64)]),
    "sscg_set_forms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sscg_mpk_newton": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Csr), ctypes.c_int,
                                       ctypes.c_int, _dp, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_int]),
    "sscg_mpk": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Csr), ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                ctypes.c_int64, ctypes.c_int]),
    "sscg_gram": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]),
    "sscg_gram_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_int, ctypes.c_void_p]),
    "sscg_small_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(BlockParams), ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "sscg_recover": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sscg_mpk32": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Csr), ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]),
    "sscg_gram32": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                   ctypes.c_void_p]),
    "sscg_batch_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Batch),
                                        ctypes.POINTER(Opts), ctypes.POINTER(BatchResult)]),
    "sscg_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Opts), ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "sscg_server_destroy": (None, [ctypes.c_void_p]),
    "sscg_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Csr), ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]),
    "sscg_server_step": (ctypes.c_int, [ctypes.c_void_p, _ip, _ip, _ip]),
    "sscg_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _ip, _ip, _ip, _ip,
                                        _dp]),
    "sscg_server_history": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, _ip,
                                           _ip, _dp, _ip, _ip]),
    "sscg_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64)]),
    "sscg_set_batch_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int]),
    "sscg_batch_tuning": (ctypes.c_int, [ctypes.c_void_p, _ip, _ip, _ip, _dp, _dp, _dp]),
    "sscg_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sscg_kernel_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int64), _dp, _dp]),
}


def lib():
    """Load libsscg.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(t) -> int:
    if t is None:
        return 0
    import torch

    assert isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous(), "need contiguous CUDA tensors"
    return t.data_ptr()


def _f64(t):
    import torch

    assert t.dtype == torch.float64, "FP64 tensors expected"
    return _ptr(t)


@dataclass
class DeviceCsr:
    """CSR matrix in device memory (torch tensors: int32, int32, float64)."""
    rowptr: object
    col: object
    val: object

    @property
    def n(self):
        return int(self.rowptr.numel() - 1)

    @property
    def nnz(self):
        return int(self.col.numel())

    @classmethod
    def from_host(cls, A, device="cuda"):
        import torch

        return cls(torch.as_tensor(np.asarray(A.rowptr, dtype=np.int32)).to(device),
                   torch.as_tensor(np.asarray(A.col, dtype=np.int32)).to(device),
                   torch.as_tensor(np.asarray(A.val, dtype=np.float64)).to(device))

    def cstruct(self) -> Csr:
        return Csr(self.n, self.nnz, _ptr(self.rowptr), _ptr(self.col) if self.nnz else 0,
                   _ptr(self.val) if self.nnz else 0)


def _check(ctx_handle, rc):
    if rc < 0:
        msg = lib().sscg_last_error(ctx_handle)
        raise SscgError(rc, msg.decode() if msg else "")
    return rc


# ------------------------------------------------------------- C-ABI names

def sscg_create(device: int = 0, stream=None) -> int:
    """Context handle on `device`, enqueueing on `stream` (a torch stream, a raw
    hipStream_t int, or None for torch's current stream)."""
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("sscg needs a HIP GPU")
    if stream is None:
        stream = torch.cuda.current_stream(device)
    raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    h = ctypes.c_void_p()
    rc = lib().sscg_create(ctypes.byref(h), device, ctypes.c_void_p(raw))
    _check(None, rc)
    return h.value


def sscg_destroy(ctx: int) -> None:
    lib().sscg_destroy(ctx)


def sscg_last_error(ctx) -> str:
    msg = lib().sscg_last_error(ctx)
    return msg.decode() if msg else ""


def sscg_opts_default() -> Opts:
    o = Opts()
    lib().sscg_opts_default(ctypes.byref(o))
    return o


class History:
    """Host arrays receiving the per-block history of a solve."""

    def __init__(self, cap: int, s_max: int):
        self.cap = cap
        self.s_max = s_max
        self.s_bar = np.zeros(cap, np.int32)
        self.s_built = np.zeros(cap, np.int32)
        self.s_tilde = np.zeros(cap, np.int32)
        self.s_k = np.zeros(cap, np.int32)
        self.gamma = np.full(cap, np.nan)
        self.thr = np.full(cap, np.nan)
        self.res_updated = np.full(cap, np.nan)
        self.relres_true = np.full(cap, np.nan)
        self.kappa = np.full(cap * s_max, np.nan)
        self.fp32 = np.zeros(cap, np.int32)
        self.res = Result()
        r = self.res
        r.cap = cap
        r.s_bar = self.s_bar.ctypes.data_as(_ip)
        r.s_built = self.s_built.ctypes.data_as(_ip)
        r.s_tilde = self.s_tilde.ctypes.data_as(_ip)
        r.s_k = self.s_k.ctypes.data_as(_ip)
        r.gamma = self.gamma.ctypes.data_as(_dp)
        r.thr = self.thr.ctypes.data_as(_dp)
        r.res_updated = self.res_updated.ctypes.data_as(_dp)
        r.relres_true = self.relres_true.ctypes.data_as(_dp)
        r.kappa = self.kappa.ctypes.data_as(_dp)
        r.fp32 = self.fp32.ctypes.data_as(_ip)

    @property
    def blocks(self):
        return int(self.res.blocks)

    @property
    def schedule(self):
        return self.s_k[: min(self.blocks, self.cap)].tolist()

    def kappas(self, k):
        row = self.kappa[k * self.s_max:(k + 1) * self.s_max]
        return row[~np.isnan(row)].tolist()


def sscg_solve(ctx: int, A: DeviceCsr, b, x, opts: Opts, hist: History | None = None) -> int:
    """Run the solver; x (CUDA float64 tensor) holds x_1 on entry, x on return.
    Waits for the device; returns the status code."""
    import torch

    torch.cuda.current_stream().synchronize()
    c = A.cstruct()
    rc = lib().sscg_solve(ctx, ctypes.byref(c), _f64(b), _f64(x), ctypes.byref(opts),
                          ctypes.byref(hist.res) if hist is not None else None)
    return _check(ctx, rc)


class BatchHistory:
    """Host arrays receiving the per-system outputs of a batched solve."""

    def __init__(self, nsys: int, cap: int):
        self.nsys, self.cap = nsys, cap
        self.status = np.zeros(nsys, np.int32)
        self.blocks = np.zeros(nsys, np.int32)
        self.iters = np.zeros(nsys, np.int32)
        self.relres = np.full(nsys, np.nan)
        self.s_k = np.zeros(nsys * cap, np.int32)
        self.s_tilde = np.zeros(nsys * cap, np.int32)
        self.relres_true = np.full(nsys * cap, np.nan)
        self.fp32 = np.zeros(nsys * cap, np.int32)
        r = self.res = BatchResult()
        r.cap = cap
        r.status = self.status.ctypes.data_as(_ip)
        r.blocks = self.blocks.ctypes.data_as(_ip)
        r.iters = self.iters.ctypes.data_as(_ip)
        r.relres = self.relres.ctypes.data_as(_dp)
        r.s_k = self.s_k.ctypes.data_as(_ip)
        r.s_tilde = self.s_tilde.ctypes.data_as(_ip)
        r.relres_true = self.relres_true.ctypes.data_as(_dp)
        r.fp32 = self.fp32.ctypes.data_as(_ip)

    def schedule(self, i: int):
        return self.s_k[i * self.cap:i * self.cap + min(int(self.blocks[i]), self.cap)].tolist()

    def precisions(self, i: int):
        """1 per block whose basis was FP32 (SSCG_PREC_VARIABLE), else 0."""
        return self.fp32[i * self.cap:i * self.cap + min(int(self.blocks[i]), self.cap)].tolist()


def sscg_batch_solve(ctx: int, systems, bs, xs, opts: Opts, tol=None, lambda_min=None,
                     lambda_max=None, hist: BatchHistory | None = None) -> int:
    """Solve the systems (DeviceCsr list) with right-hand sides bs and iterates
    xs (CUDA float64 tensors; x_1 in, solution out) side by side.  tol and the
    Chebyshev intervals are optional per-system sequences.  Waits for the
    device; returns the worst per-system status."""
    import torch

    torch.cuda.current_stream().synchronize()
    n = len(systems)
    A = (Csr * n)(*[S.cstruct() for S in systems])
    b = (ctypes.c_void_p * n)(*[_f64(t) for t in bs])
    x = (ctypes.c_void_p * n)(*[_f64(t) for t in xs])
    keep = []

    def darr(v):
        if v is None:
            return None
        a = np.ascontiguousarray(v, dtype=np.float64)
        assert a.size == n
        keep.append(a)
        return a.ctypes.data_as(_dp)

    B = Batch(n, A, b, x, darr(tol), darr(lambda_min), darr(lambda_max))
    rc = lib().sscg_batch_solve(ctx, ctypes.byref(B), ctypes.byref(opts),
                                ctypes.byref(hist.res) if hist is not None else None)
    return _check(ctx, rc)


def sscg_server_create(ctx: int, opts: Opts, pool_rows: int, pool_nnz: int, slots: int) -> int:
    h = ctypes.c_void_p()
    _check(ctx, lib().sscg_server_create(ctx, ctypes.byref(opts), pool_rows, pool_nnz, slots,
                                         ctypes.byref(h)))
    return h.value


def sscg_server_destroy(server: int) -> None:
    lib().sscg_server_destroy(server)


def sscg_server_submit(ctx: int, server: int, A: DeviceCsr, b, x, tol: float = 0.0,
                       lambda_min: float = 0.0, lambda_max: float = 1.0) -> int:
    """Queue a request (b, x: CUDA float64 tensors kept alive by the caller
    until it is done); returns its id.  Errors are reported through ctx."""
    import torch

    torch.cuda.current_stream().synchronize()
    c = A.cstruct()
    rid = ctypes.c_int64()
    _check(ctx, lib().sscg_server_submit(server, ctypes.byref(c), _f64(b), _f64(x), tol,
                                         lambda_min, lambda_max, ctypes.byref(rid)))
    return rid.value


def sscg_server_step(ctx: int, server: int) -> tuple[int, int, int]:
    """One outer block for all admitted systems; returns (running, queued, retired)."""
    run, q, ret = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, lib().sscg_server_step(server, ctypes.byref(run), ctypes.byref(q),
                                       ctypes.byref(ret)))
    return run.value, q.value, ret.value


def sscg_server_poll(ctx: int, server: int, rid: int) -> dict:
    st, status, blocks, iters = (ctypes.c_int32() for _ in range(4))
    rel = ctypes.c_double()
    _check(ctx, lib().sscg_server_poll(server, rid, ctypes.byref(st), ctypes.byref(status),
                                       ctypes.byref(blocks), ctypes.byref(iters),
                                       ctypes.byref(rel)))
    return dict(state=st.value, status=status.value, blocks=blocks.value, iters=iters.value,
                relres=rel.value)


def sscg_server_history(ctx: int, server: int, rid: int, cap: int = 4096) -> dict:
    """Per-block s_k, s~_k, true relative residual and basis precision (1: FP32)
    of a finished request."""
    sk = np.zeros(cap, np.int32)
    st = np.zeros(cap, np.int32)
    rel = np.full(cap, np.nan)
    f32 = np.zeros(cap, np.int32)
    rows = ctypes.c_int32()
    _check(ctx, lib().sscg_server_history(server, rid, cap, sk.ctypes.data_as(_ip),
                                          st.ctypes.data_as(_ip), rel.ctypes.data_as(_dp),
                                          f32.ctypes.data_as(_ip), ctypes.byref(rows)))
    k = rows.value
    return dict(s_k=sk[:k].tolist(), s_tilde=st[:k].tolist(), relres_true=rel[:k].tolist(),
                fp32=f32[:k].tolist())


def sscg_set_batch_tuning(ctx: int, mode: int, kappa_threads: int = 0, gram_waves: int = 0,
                          mpk_chunk: int = 0) -> int:
    return _check(ctx, lib().sscg_set_batch_tuning(ctx, mode, kappa_threads, gram_waves,
                                                   mpk_chunk))


def sscg_batch_tuning(ctx: int) -> dict:
    """Launch shapes of the last batch and the candidates' timings (us)."""
    kt, gw, mc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ku, gu, mu = np.zeros(4), np.zeros(3), np.zeros(3)
    _check(ctx, lib().sscg_batch_tuning(ctx, ctypes.byref(kt), ctypes.byref(gw), ctypes.byref(mc),
                                        ku.ctypes.data_as(_dp), gu.ctypes.data_as(_dp),
                                        mu.ctypes.data_as(_dp)))
    return dict(kappa_threads=kt.value, gram_waves=gw.value, mpk_chunk=mc.value,
                kappa_us=ku.tolist(), gram_us=gu.tolist(), mpk_us=mu.tolist())


def sscg_server_stats(ctx: int, server: int) -> dict:
    """Replays launched and the sum over them of the admitted rows."""
    v = [ctypes.c_int64() for _ in range(2)]
    _check(ctx, lib().sscg_server_stats(server, *[ctypes.byref(x) for x in v]))
    return dict(replays=v[0].value, rows_active=v[1].value)


def sscg_residual(ctx: int, A: DeviceCsr, b, x, r, out2) -> int:
    c = A.cstruct()
    return _check(ctx, lib().sscg_residual(ctx, ctypes.byref(c), _f64(b), _f64(x),
                                           _f64(r) if r is not None else None, _f64(out2)))


def sscg_spectral_bounds(ctx: int, A: DeviceCsr, steps: int = 30, seed: int = 0):
    c = A.cstruct()
    lo = ctypes.c_double()
    hi = ctypes.c_double()
    _check(ctx, lib().sscg_spectral_bounds(ctx, ctypes.byref(c), steps, seed, ctypes.byref(lo),
                                           ctypes.byref(hi)))
    return lo.value, hi.value


def sscg_mpk(ctx: int, A: DeviceCsr, s: int, first: bool, basis: int, lmin: float, lmax: float,
             Y, ldy: int, rcol: int) -> int:
    c = A.cstruct()
    return _check(ctx, lib().sscg_mpk(ctx, ctypes.byref(c), s, int(first), basis, lmin, lmax,
                                      _f64(Y), ldy, rcol))


def sscg_matrix_format(ctx: int, A: DeviceCsr):
    """(format bits FMT_COL16 | FMT_VTAB | FMT_SDIA | FMT_SDPAIR | FMT_SDVAL,
    padded SELL-64 entry count)."""
    c = A.cstruct()
    f = ctypes.c_int()
    st = ctypes.c_int64()
    _check(ctx, lib().sscg_matrix_format(ctx, ctypes.byref(c), ctypes.byref(f), ctypes.byref(st)))
    return f.value, st.value


def sscg_set_forms(ctx: int, forms: int) -> int:
    """Allowed compact forms of A (FMT_COL16 | FMT_VTAB | FMT_SDIA | FMT_SDPAIR |
    FMT_SDVAL bits)."""
    return _check(ctx, lib().sscg_set_forms(ctx, forms))


def sscg_newton_shifts(ctx: int, A: DeviceCsr, m: int, seed: int = 0) -> list:
    c = A.cstruct()
    out = (ctypes.c_double * m)()
    _check(ctx, lib().sscg_newton_shifts(ctx, ctypes.byref(c), m, seed, out))
    return list(out)


def sscg_mpk_newton(ctx: int, A: DeviceCsr, s: int, first: bool, shifts, Y, ldy: int,
                    rcol: int) -> int:
    c = A.cstruct()
    th = (ctypes.c_double * s)(*[float(t) for t in shifts[:s]])
    return _check(ctx, lib().sscg_mpk_newton(ctx, ctypes.byref(c), s, int(first), th, _f64(Y), ldy,
                                             rcol))


def sscg_gram(ctx: int, n: int, s: int, first: bool, Y, ldy: int, rcol: int, G) -> int:
    return _check(ctx, lib().sscg_gram(ctx, n, s, int(first), _f64(Y), ldy, rcol, _f64(G)))


def sscg_gram_noalloc(ctx: int, n: int, s: int, first: bool, Y, ldy: int, rcol: int, G) -> int:
    return _check(ctx, lib().sscg_gram_noalloc(ctx, n, s, int(first), _f64(Y), ldy, rcol,
                                               _f64(G)))


def sscg_small_solve(ctx: int, G, prm: BlockParams, coef, info) -> int:
    """info: a CUDA uint8 tensor of at least ctypes.sizeof(BlockInfo) bytes."""
    return _check(ctx, lib().sscg_small_solve(ctx, _f64(G), ctypes.byref(prm), _f64(coef),
                                              _ptr(info)))


def sscg_recover(ctx: int, n: int, s: int, first: bool, Y, ldy: int, rcol: int, coef, x, r, p):
    return _check(ctx, lib().sscg_recover(ctx, n, s, int(first), _f64(Y), ldy, rcol, _f64(coef),
                                          _f64(x), _ptr(r), _ptr(p)))


TIME_ALL = 0xF


def sscg_mpk32(ctx: int, A: DeviceCsr, s: int, first: bool, basis: int, lmin: float, lmax: float,
               Y, ldy: int, rcol: int) -> int:
    import torch

    assert Y.dtype == torch.float32
    c = A.cstruct()
    return _check(ctx, lib().sscg_mpk32(ctx, ctypes.byref(c), s, int(first), basis, lmin, lmax,
                                        _ptr(Y), ldy, rcol))


def sscg_gram32(ctx: int, n: int, s: int, first: bool, Y, ldy: int, rcol: int, G) -> int:
    import torch

    assert Y.dtype == torch.float32
    return _check(ctx, lib().sscg_gram32(ctx, n, s, int(first), _ptr(Y), ldy, rcol, _f64(G)))


def sscg_set_timing(ctx: int, on) -> int:
    """on: True (every family), False (off), or an iterable of family names."""
    if isinstance(on, bool):
        mask = TIME_ALL if on else 0
    else:
        mask = 0
        for f in on:
            mask |= 1 << (FAMILIES[f] if isinstance(f, str) else int(f))
    return _check(ctx, lib().sscg_set_timing(ctx, mask))


def sscg_kernel_stats(ctx: int, family) -> tuple[int, float, float]:
    fam = FAMILIES[family] if isinstance(family, str) else int(family)
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(ctx, lib().sscg_kernel_stats(ctx, fam, ctypes.byref(n), ctypes.byref(ms),
                                        ctypes.byref(by)))
    return n.value, ms.value, by.value


def block_info_from(t) -> BlockInfo:
    """Decode a BlockInfo from a device byte tensor."""
    raw = bytes(t.cpu().numpy().tobytes()[: ctypes.sizeof(BlockInfo)])
    return BlockInfo.from_buffer_copy(raw)


def make_opts(mode="adaptive", basis="monomial", tol=1e-10, s_max=8, s0_bar=0, f=0, fixed_s=4,
              schedule=None, c=1.0, lmin=math.nan, lmax=math.nan, lanczos_steps=30,
              lanczos_seed=0, equilibrate=False, inner_check=True, max_iters=100000,
              precision="fp64", max_outer=30, inner_tol=1e-5, c_mode="const",
              kappa_a=math.nan, norm_a=math.nan, shifts=None) -> Opts:
    o = sscg_opts_default()
    o.mode = {"adaptive": MODE_ADAPTIVE, "fixed": MODE_FIXED, "schedule": MODE_SCHEDULE}[mode]
    o.basis = {"monomial": BASIS_MONOMIAL, "chebyshev": BASIS_CHEBYSHEV,
               "newton": BASIS_NEWTON}[basis]
    o.c_mode = {"const": C_CONST, "theory": C_THEORY}[c_mode]
    o.kappa_a = kappa_a
    o.norm_a = norm_a
    if shifts is not None:
        arr = np.ascontiguousarray(shifts, dtype=np.float64)
        o._shifts_keep = arr  # keep alive with the struct
        o.shifts = arr.ctypes.data_as(_dp)
    o.tol = tol
    o.s_max = s_max
    o.s0_bar = s0_bar
    o.f = f
    o.fixed_s = fixed_s
    if schedule is not None:
        arr = np.ascontiguousarray(schedule, dtype=np.int32)
        o._sched_keep = arr  # keep alive with the struct
        o.schedule = arr.ctypes.data_as(_ip)
        o.schedule_len = arr.size
    o.c = c
    o.lambda_min = lmin
    o.lambda_max = lmax
    o.lanczos_steps = lanczos_steps
    o.lanczos_seed = lanczos_seed
    o.equilibrate = int(equilibrate)
    o.inner_check = int(inner_check)
    o.max_iters = max_iters
    o.precision = {"fp64": PREC_FP64, "mixed": PREC_MIXED, "variable": PREC_VARIABLE}[precision]
    o.max_outer = max_outer
    o.inner_tol = inner_tol
    return o
