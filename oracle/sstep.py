"""s-step CG in its three forms (test infrastructure only).

  * fixed s        -- Algorithm 2 (s-step conjugate gradient),
  * given schedule -- Algorithm 3 (variable s-step CG),
  * adaptive       -- Algorithm 4 (adaptive s-step CG), with s_k chosen by the
                      condition-number rule (eq. condy) and the in-loop check
                      (eq. check) of Section 4.2.

Written once against ``oracle.arith`` so that the same code runs in FP64 with
correctly rounded reductions and in exact rational arithmetic.

Readings taken where the paper is silent (each is also listed in the design
notes of the repository):
  R1  unit round-off eps = 2^-53 (Section 5 runs in double precision).
  R2  eps* = tol * ||b||_2: the target is a relative residual.
  R3  after each outer block the true residual ||b - A x|| / ||b|| is formed
      and the solve stops when it is <= tol (the tables count outer loops until
      the true residual reaches the target); a cap on total inner iterations.
  R4  block 0 builds only the P block [rho_0(A) p .. rho_s(A) p]: with
      p_1 = r_1 the R block would repeat column P_0, the Gram matrix would be
      singular and the rule could never pick s_0 > 1, yet the experiments
      report s_0 = 6 and s_0 = 2.  The space is the same (K_{s+1}(A, r_1)); the
      coordinates start as p' = r' = e_0.
  R5  rank guard: by eq. reqsubspaces the i-step basis of block k >= 1 lies in
      K_{m+i+1}(A, r_1), so it is rank deficient when i > m.  Only i <= m is
      considered and only min(s_bar, m) steps of the basis are built.  This
      changes nothing in exact arithmetic.
  R6  kappa(G_i) from ``oracle.kappa`` (Jacobi), +inf if not positive definite.
  R7  s~ is the end of the longest prefix i = 1, 2, .. that satisfies eq.
      condy (accept on equality); none -> s~ = 1 (Section 4.2's default).  The
      in-loop check breaks on '>=' after the updates of that iteration.
  R8  ||r_{m+1}|| in eq. condy is sqrt(G[R_0, R_0]) (sqrt(G[P_0,P_0]) in block 0).
  R9  reductions are order independent (correctly rounded), except the Gram
      matrix G = Y^T Y, whose entries are fma chains over 1024-row groups in row
      order with the group partials added pairwise (``oracle.arith``);
      quadratic forms: v^T G v = RN(v . RN(G v)); p'^T G B p' = RN(p' . RN(G RN(B p'))).
  R10 breakdown: if p'^T G B p' is not positive and finite, or alpha is not
      finite, the block ends after the previous iteration (status BREAKDOWN if
      that leaves no iteration).
  R11 Chebyshev parameters on [lmin, lmax]: c0 = (lmax+lmin)/2, h = (lmax-lmin)/2,
      theta_j = c0, gamma_0 = h, gamma_j = h/2 (j >= 1), sigma_j = h/2, so that
      rho_j(z) = T_j((z - c0)/h).
  R12 B (eq. AVVB) in the paper's column order [P_0..P_s, R_0..R_{s-1}]: within
      each block, column j (not the last) has B[j+1,j] = gamma_j,
      B[j,j] = theta_j, B[j-1,j] = sigma_{j-1}; the last column of each block is
      zero because those columns of Y are zeroed in the underlined Y.
  R13 optional equilibration A <- D^{-1/2} A D^{-1/2}, D_i = max_j |a_ij|
      (Section 5); with s_i = 1/sqrt(D_i): a~_ij = (a_ij s_i) s_j, b~ = s b,
      x~_1 = x_1 / s, x = s x~ at the end.  Tolerance and eps* refer to the
      scaled system.
  R17 variable precision (Section 6's closing remark, which rearranges eq. fb
      into a bound eps_k <= eps* / (c kappa(Y_k) max ||r^||) on the unit
      round-off of outer loop k and leaves the method as future work): with
      precision='variable' (adaptive mode, constant c), block k >= 1 stores its
      basis in FP32 when ((2^-24 c) gamma_{k-1}) sqrt(max(rr_{k-1}, 0)) <= eps*
      (``fp32_block_allowed``): the previous block's gamma stands in for
      kappa(Y_k), which is not built yet, and the residual norm the block
      starts from for the maximum over the block.  In such a block every basis
      column, P_0 = RN32(p) and R_0 = RN32(r) included, is the FP64 block's
      column computed from the stored columns and rounded once to FP32; the
      Gram matrix, kappa, the coefficient recurrence and the recovery are the
      FP64 block's operations on these columns, and eqs. condy and check use
      eps = 2^-24.  Block 0 is FP64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .arith import CR, ieee_div, ieee_sqrt
from .kappa import kappa_spd

EPS = 2.0 ** -53  # R1
EPS32 = 2.0 ** -24  # R1 for an FP32 basis (R17)

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


@dataclass
class Opts:
    mode: str = "adaptive"  # 'adaptive' | 'fixed' | 'schedule'
    basis: str = "monomial"  # 'monomial' | 'chebyshev'
    tol: float = 1e-10
    s_max: int = 8
    s0_bar: Optional[int] = None  # default s_max (Section 5)
    f: Optional[int] = None  # default s_max (Section 5)
    fixed_s: Optional[int] = None
    schedule: Optional[list] = None
    c: float = 1.0  # constant c_{k,j} (Section 5 uses 1, 10, sqrt(kappa(A)))
    lmin: Optional[float] = None
    lmax: Optional[float] = None
    equilibrate: bool = False
    max_iters: int = 100000
    inner_check: bool = True
    shifts: Optional[list] = None  # Newton basis: shifts theta_0, theta_1, ... (R15)
    c_mode: str = "const"  # 'const': c_{k,j} = c; 'theory': 6 N_k j kappa(A) (R16)
    kappa_a: Optional[float] = None  # theory mode: kappa(A)
    norm_a: Optional[float] = None  # theory mode: ||A||_2
    n_a: Optional[int] = None  # theory mode: max nonzeros per row (None: from A)
    precision: str = "fp64"  # 'fp64' | 'variable': FP32 basis in the blocks R17 allows


@dataclass
class Block:
    k: int
    m: int  # iterations done before this block
    s_bar: int  # s_bar_k of Alg. 4 (or s of Alg. 2/3)
    s_built: int  # basis steps actually built (R5)
    s_tilde: int
    s_k: int
    gamma: float  # estimate of kappa(Y_{k, s~})
    thr: float  # right-hand side of eq. condy
    rnorm: float  # ||r_{m+1}|| from the Gram matrix (R8)
    kappas: list  # kappa(G_{k,i}), i = 1..imax
    alphas: list
    betas: list
    res_updated: float  # sqrt(r'^T G r') after the last inner iteration
    relres_true: float  # ||b - A x|| / ||b|| after the block
    status: int = OK
    rr_trace: list = field(default_factory=list)  # r'^T G r' after inner iteration j = 1..s_k
    fp32: bool = False  # basis stored in FP32, eqs. condy and check with 2^-24 (R17)


@dataclass
class Result:
    x: object
    status: int
    blocks: list = field(default_factory=list)
    iters: int = 0
    relres0: float = 1.0

    @property
    def schedule(self):
        return [b.s_k for b in self.blocks]

    @property
    def relres(self):
        return self.blocks[-1].relres_true if self.blocks else self.relres0


# --------------------------------------------------------------------------
# polynomial basis (eqs. cg-krylovbasis, polybasiscg) and B (eq. AVVB)


def basis_params(basis: str, s: int, lmin=None, lmax=None, ar=None, shifts=None):
    """(theta, gamma, sigma), lists of length s+1, of the three-term recurrence."""
    one = ar.scalar(1) if ar is not None else 1.0
    zero = one - one
    if basis == "monomial":
        return [zero] * (s + 1), [one] * (s + 1), [zero] * (s + 1)
    if basis == "newton":  # rho_j(z) = (z - theta_{j-1}) rho_{j-1}(z): gamma = 1, sigma = 0
        if shifts is None or len(shifts) < s:
            raise ValueError("the Newton basis needs s shifts")
        theta = [ar.scalar(t) if ar is not None else t for t in shifts[:s]] + [zero]
        return theta, [one] * (s + 1), [zero] * (s + 1)
    if basis == "chebyshev":
        half = one / 2
        c0 = (lmax + lmin) * half
        h = (lmax - lmin) * half
        h2 = h * half
        theta = [c0] * (s + 1)
        gamma = [h] + [h2] * s
        sigma = [h2] * (s + 1)
        return theta, gamma, sigma
    raise ValueError(basis)


def poly_next(ar, A, u, w, j, prm):
    """rho_j(A)v from rho_{j-1}(A)v = u and rho_{j-2}(A)v = w (eq. polybasiscg):
    RN(A u - theta_{j-1} u - sigma_{j-2} w) / gamma_{j-1}."""
    theta, gamma, sigma = prm
    extra = [(-theta[j - 1], u)]
    if j >= 2:
        extra.append((-sigma[j - 2], w))
    num = ar.csr_comb(A, u, extra)
    return ar.vdiv(num, gamma[j - 1])


def round32(v) -> np.ndarray:
    """Every entry rounded once to FP32 (IEEE round to nearest even), kept as
    FP64 values."""
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def krylov_basis(ar, A, p, r, s: int, first: bool, prm, fp32: bool = False):
    """Columns of Y_{k,s} = [P_{k,s}, R_{k,s}] in the paper's order
    [P_0..P_s, R_0..R_{s-1}] (eq. cg-krylovbasis); block 0: P only (R4).
    fp32 (R17): p, r and every new column are rounded to FP32 as soon as they
    are formed, so each column is computed from the stored (rounded) ones."""
    rnd = round32 if fp32 else (lambda v: v)
    P = [rnd(p)]
    for j in range(1, s + 1):
        P.append(rnd(poly_next(ar, A, P[j - 1], P[j - 2] if j >= 2 else None, j, prm)))
    if first:
        return P
    R = [rnd(r)]
    for j in range(1, s):
        R.append(rnd(poly_next(ar, A, R[j - 1], R[j - 2] if j >= 2 else None, j, prm)))
    return P + R


def fp32_block_allowed(c_smax: float, gamma_prev: float, rr_prev: float,
                       eps_star: float) -> bool:
    """R17: Section 6 rearranges eq. fb into a bound on the unit round-off an
    outer loop may use, eps_k <= eps* / (c kappa(Y_k) max ||r^||).  Block k takes
    an FP32 basis when that bound admits 2^-24 with the previous block's
    estimate gamma_{k-1} of kappa(Y) standing in for the basis not yet built
    and the updated residual norm the block starts from,
    sqrt(max(r'^T G r', 0)) of block k-1:
        ((2^-24 c_{k,s_max}) gamma_{k-1}) sqrt(max(rr_{k-1}, 0)) <= eps*,
    each operation one IEEE rounding in this order."""
    lhs = ((EPS32 * c_smax) * gamma_prev) * ieee_sqrt(max(rr_prev, 0.0))
    return lhs <= eps_star


def assemble_B(ar, s: int, first: bool, prm):
    """(2s+1)^2 (block 0: (s+1)^2) matrix with A Y_underline = Y B (R12)."""
    theta, gamma, sigma = prm
    zero = ar.scalar(0)
    d = s + 1 if first else 2 * s + 1
    B = [[zero] * d for _ in range(d)]

    def block(off, size):
        for j in range(size - 1):  # last column stays zero
            B[off + j + 1][off + j] = gamma[j]
            B[off + j][off + j] = theta[j]
            if j >= 1:
                B[off + j - 1][off + j] = sigma[j - 1]

    block(0, s + 1)
    if not first:
        block(s + 1, s)
    return B


def sub_indices(s_bar: int, i: int, first: bool):
    """Columns of Y_{k,i} inside Y_{k,s_bar}: [1:i+1, i_s:i_s+i-1] (1-based,
    i_s = s_bar + 2) of Section 4.2, here 0-based."""
    if first:
        return list(range(i + 1))
    return list(range(i + 1)) + list(range(s_bar + 1, s_bar + 1 + i))


def principal(M, idx):
    return [[M[a][b] for b in idx] for a in idx]


# --------------------------------------------------------------------------
# the coordinate recurrence (inner loop of Algs. 2-4)


def quad(ar, G, v):
    """v^T G v = RN(v . RN(G v)) (R9)."""
    return ar.sdot(v, ar.smatvec(G, v))


def inner_loop(ar, G, B, s: int, first: bool, check=None, iters=None, trace=None):
    """Run up to s iterations (or `iters` <= s) of the coordinate recurrence
    in the s-step basis (dimension 2s+1; s+1 in block 0).

    check: None (Algs. 2/3) or a function (j, rr1) -> bool that is True when
    the in-loop test of Alg. 4 (eq. check) says to break after iteration j.
    trace: optional list; r'^T G r' after each iteration is appended to it.
    Returns (s_k, x', r', p', alphas, betas, rr, status)."""
    d = len(G)
    zero = ar.scalar(0)
    one = ar.scalar(1)
    p = [zero] * d
    r = [zero] * d
    xc = [zero] * d
    p[0] = one
    r[0 if first else s + 1] = one
    rr = quad(ar, G, r)
    alphas, betas = [], []
    s_k = 0
    status = OK
    for j in range(1, (s if iters is None else iters) + 1):
        Bp = ar.smatvec(B, p)
        den = ar.sdot(p, ar.smatvec(G, Bp))
        if den == 0 or (not ar.exact and (not (den > 0.0) or not math.isfinite(den))):
            status = BREAKDOWN if j == 1 else OK
            break
        alpha = ar.div(rr, den)
        if not ar.isfinite(alpha):
            status = BREAKDOWN if j == 1 else OK
            break
        s_k = j
        q = [alpha * v for v in p]
        xc = [a + b for a, b in zip(xc, q)]
        Bq = ar.smatvec(B, q)
        r = [a - b for a, b in zip(r, Bq)]
        rr1 = quad(ar, G, r)
        beta = ar.div(rr1, rr)
        p = [a + beta * b for a, b in zip(r, p)]
        alphas.append(alpha)
        betas.append(beta)
        if trace is not None:
            trace.append(rr1)
        rr = rr1
        if check is not None and check(j, rr1):
            break
    return s_k, xc, r, p, alphas, betas, rr, status


def recover(ar, cols, xc, rc, pc, x):
    """x <- Y x' + x, r <- Y r', p <- Y p' (eq. coords)."""
    return ar.rows_comb(cols, xc, x), ar.rows_comb(cols, rc), ar.rows_comb(cols, pc)


# --------------------------------------------------------------------------


def true_residual(ar, A, b, x):
    """b - A x, one rounding per row."""
    neg_one = ar.scalar(-1)
    return ar.neg(ar.csr_comb(A, x, [(neg_one, b)]))


def relres_of(ar, A, b, x, nb):
    res = true_residual(ar, A, b, x)
    return ar.div(ar.sqrt(ar.dot(res, res)), nb)


class _Scaled:
    def __init__(self, rowptr, col, val):
        self.rowptr, self.col, self.val = rowptr, col, val
        self.n = len(rowptr) - 1


def equilibrate(A):
    """(scaled matrix, s) with s_i = 1/sqrt(max_j |a_ij|) (R13)."""
    rowptr = np.asarray(A.rowptr)
    col = np.asarray(A.col)
    val = np.asarray(A.val, dtype=np.float64)
    n = rowptr.size - 1
    D = np.zeros(n)
    for i in range(n):
        seg = np.abs(val[rowptr[i]:rowptr[i + 1]])
        D[i] = seg.max() if seg.size else 0.0
    s = 1.0 / np.sqrt(D)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    vs = (val * s[rows]) * s[col]
    return _Scaled(rowptr, col, vs), s


def b_norm_bound(B) -> float:
    """sqrt(||B||_1 ||B||_inf) >= ||B||_2 for the tridiagonal-block B of R12:
    column sums |B[j-1][j]| + |B[j][j]| + |B[j+1][j]| and row sums
    |B[i][i-1]| + |B[i][i]| + |B[i][i+1]|, each added in that order (R16)."""
    d = len(B)
    n1 = 0.0
    ni = 0.0
    for j in range(d):
        c = 0.0
        for i in (j - 1, j, j + 1):
            if 0 <= i < d:
                c = c + abs(float(B[i][j]))
        n1 = max(n1, c)
        r = 0.0
        for i in (j - 1, j, j + 1):
            if 0 <= i < d:
                r = r + abs(float(B[j][i]))
        ni = max(ni, r)
    return math.sqrt(n1 * ni)


def c_theory(j: int, n_a: int, bnorm: float, norm_a: float, kappa_a: float) -> float:
    """c_{k,j} = 6 N_k j kappa(A), N_k = 7 + 2 N_A + 14 ||B_k|| / ||A|| (Section 4.1,
    the bound behind eq. fb), evaluated in this order in FP64 (R16)."""
    tau = bnorm / norm_a
    nk = (7.0 + 2.0 * n_a) + 14.0 * tau
    return ((6.0 * nk) * j) * kappa_a


def condy_accepts(kappa_i: float, thr: float) -> bool:
    """eq. condy for one sub-basis: sqrt(kappa(G_{k,i})) <= thr, accepted on
    equality (R7)."""
    return ieee_sqrt(kappa_i) <= thr


def check_breaks(gam: float, eps_star: float, c_j: float, rr1: float, eps: float = EPS) -> bool:
    """eq. check after inner iteration j: break when
    gamma >= eps* / (c_{k,j} eps (r'^T G r')^(1/2)), with r' the coordinates
    after iteration j's update and its quadratic form clamped at 0 (R7, R10);
    eps = the unit round-off of the block's basis (R1, R17)."""
    rhs = ieee_div(eps_star, (c_j * eps) * ieee_sqrt(max(rr1, 0.0)))
    return gam >= rhs


def max_row_nnz(A) -> int:
    return int(np.max(np.diff(np.asarray(A.rowptr)))) if len(A.rowptr) > 1 else 0


def next_s(opts: Opts, k: int, s_prev: int, m: int):
    """(s_bar_k, steps to build) for block k."""
    if opts.mode == "fixed":
        return opts.fixed_s, opts.fixed_s
    if opts.mode == "schedule":
        sch = opts.schedule
        s = sch[k] if k < len(sch) else sch[-1]
        return s, s
    s0 = opts.s0_bar if opts.s0_bar is not None else opts.s_max
    f = opts.f if opts.f is not None else opts.s_max
    s_bar = s0 if k == 0 else min(s_prev + f, opts.s_max)
    s_built = s_bar if k == 0 else min(s_bar, max(m, 1))  # R5
    return s_bar, s_built


def solve(A, b, x1, opts: Opts, ar=None, diag=None) -> Result:
    """Algorithms 2, 3 or 4 (opts.mode) for A x = b from x_1.

    diag: optional list; if given, every inner iteration appends the
    materialised iterates (x^, r^) used by the residual-gap test."""
    ar = ar if ar is not None else CR()
    scale = None
    if opts.equilibrate:
        if ar.exact:
            raise ValueError("equilibration takes square roots")
        A, scale = equilibrate(A)
        b = np.asarray(b, dtype=np.float64) * scale
        x = np.asarray(x1, dtype=np.float64) / scale
    else:
        b = ar.vec(b)
        x = ar.vec(x1)
    nb2 = ar.dot(b, b)
    if nb2 == 0:
        x = ar.zeros(len(b))
        return Result(x=(x if scale is None else x * scale), status=OK, relres0=0.0)
    nb = ar.sqrt(nb2) if not ar.exact else None
    eps_star = opts.tol * nb if not ar.exact else None  # R2

    if opts.basis == "chebyshev":
        if opts.lmin is None or opts.lmax is None:
            raise ValueError("the Chebyshev basis needs lmin and lmax")
    if opts.c_mode == "theory":
        if opts.kappa_a is None or opts.norm_a is None:
            raise ValueError("the theoretical c_{k,j} needs kappa_a and norm_a")
        n_a = opts.n_a if opts.n_a is not None else max_row_nnz(A)
    r = true_residual(ar, A, b, x)
    p = r
    res = Result(x=x, status=NOT_CONVERGED)
    if not ar.exact:
        res.relres0 = ar.div(ar.sqrt(ar.dot(r, r)), nb)
        if res.relres0 <= opts.tol:
            res.status = OK
            res.x = x if scale is None else x * scale
            return res
    if opts.precision not in ("fp64", "variable"):
        raise ValueError(opts.precision)
    if opts.precision == "variable" and (opts.mode != "adaptive" or opts.c_mode != "const"
                                         or ar.exact):
        raise ValueError("variable precision: adaptive mode, constant c, FP64 arithmetic")
    m = 0
    s_prev = 0
    k = 0
    gam_prev = rr_prev = math.nan
    while True:
        first = k == 0
        s_bar, s_built = next_s(opts, k, s_prev, m)
        prm = basis_params(opts.basis, s_built, opts.lmin, opts.lmax, ar, opts.shifts)
        fp32 = (opts.precision == "variable" and not first
                and fp32_block_allowed(opts.c, gam_prev, rr_prev, eps_star))
        ueps = EPS32 if fp32 else EPS
        cols = krylov_basis(ar, A, p, r, s_built, first, prm, fp32)
        G = ar.gram(cols)
        kappas = []
        gam = math.nan
        thr = math.nan
        rnorm = math.nan
        check = None
        if opts.mode == "adaptive":
            rnorm = ar.sqrt(G[0][0] if first else G[s_built + 1][s_built + 1])  # R8
            if opts.c_mode == "theory":  # R16: B of the block's built basis
                bnorm = b_norm_bound(assemble_B(ar, s_built, first, prm))

                def cfun(j, _b=bnorm):
                    return c_theory(j, n_a, _b, opts.norm_a, opts.kappa_a)
            else:
                def cfun(j):
                    return opts.c
            c_smax = cfun(opts.s_max)
            thr = ar.div(eps_star, (c_smax * ueps) * rnorm)  # eq. condy
            imax = s_built
            s_tilde = 1
            for i in range(1, imax + 1):  # R7
                kap = kappa_spd(principal(G, sub_indices(s_built, i, first)))
                kappas.append(kap)
                if condy_accepts(kap, thr):
                    s_tilde = i
                else:
                    break
            gam = ar.sqrt(kappas[s_tilde - 1])
            if opts.inner_check:
                def check(j, rr1, _gam=gam, _c=cfun, _e=ueps):
                    return check_breaks(_gam, eps_star, _c(j), rr1, _e)
        else:
            s_tilde = s_built
        idx = sub_indices(s_built, s_tilde, first)
        Gs = principal(G, idx)
        Bs = assemble_B(ar, s_tilde, first,
                        basis_params(opts.basis, s_tilde, opts.lmin, opts.lmax, ar, opts.shifts))
        ys = [cols[a] for a in idx]
        rr_trace = []
        s_k, xc, rc, pc, alphas, betas, rr, st = inner_loop(ar, Gs, Bs, s_tilde, first, check,
                                                            trace=rr_trace)
        if diag is not None:
            _diag_block(ar, diag, ys, Gs, Bs, s_tilde, first, x, check, k, m)
        if s_k == 0:
            # exact arithmetic: r = 0 exactly means the solve has terminated
            res.status = OK if (ar.exact and quad(ar, Gs, rc) == 0) else BREAKDOWN
            break
        x, r, p = recover(ar, ys, xc, rc, pc, x)
        m += s_k
        s_prev = s_k
        blk = Block(k=k, m=m - s_k, s_bar=s_bar, s_built=s_built, s_tilde=s_tilde, s_k=s_k,
                    gamma=gam, thr=thr, rnorm=rnorm, kappas=kappas, alphas=alphas, betas=betas,
                    res_updated=(ar.sqrt(max(rr, 0.0)) if not ar.exact else rr),
                    relres_true=(relres_of(ar, A, b, x, nb) if not ar.exact else math.nan),
                    status=st, rr_trace=rr_trace, fp32=fp32)
        res.blocks.append(blk)
        gam_prev, rr_prev = gam, rr
        k += 1
        if not ar.exact and blk.relres_true <= opts.tol:
            res.status = OK
            break
        if not ar.exact and not math.isfinite(blk.relres_true):
            res.status = BREAKDOWN
            break
        if m >= opts.max_iters:
            res.status = NOT_CONVERGED
            break
    res.iters = m
    res.x = x if scale is None else x * scale
    return res


def _diag_block(ar, diag, ys, Gs, Bs, s, first, x_start, check, k, m):
    """Re-run the block's inner loop, materialising after every iteration j
    x^_{m+j+1} = Y x' + x^_{m+1} and r^_{m+j+1} = Y r' (eqs. x, r)."""
    for j in range(1, s + 1):
        s_k, xc, rc, pc, *_ = inner_loop(ar, Gs, Bs, s, first, None, iters=j)
        if s_k < j:
            break
        xj = ar.rows_comb(ys, xc, x_start)
        rj = ar.rows_comb(ys, rc)
        diag.append(dict(k=k, m=m, j=j, x=xj, r=rj, Y=ys, xc=xc, rc=rc))
        if check is not None:
            rr1 = quad(ar, Gs, rc)
            if check(j, rr1):
                break
