"""Classical conjugate gradient, Algorithm 1 (test infrastructure only).

Written literally: alpha_i = r_i^T r_i / p_i^T A p_i, q_i = alpha_i p_i,
x_{i+1} = x_i + q_i, r_{i+1} = r_i - A q_i, beta_i = r_{i+1}^T r_{i+1} / r_i^T r_i,
p_{i+1} = r_{i+1} + beta_i p_i.  Runs in FP64 with correctly rounded
reductions or in exact rational arithmetic (``oracle.arith``).  In FP64 the
solve stops when the true relative residual ||b - A x|| / ||b|| reaches tol,
checked after every iteration (the experiments count classical CG's
iterations that way).
"""
from __future__ import annotations

from dataclasses import dataclass, field

from .arith import CR
from .sstep import OK, NOT_CONVERGED, BREAKDOWN, relres_of, true_residual


@dataclass
class CGResult:
    x: object
    status: int
    iters: int = 0
    alphas: list = field(default_factory=list)
    betas: list = field(default_factory=list)
    xs: list = field(default_factory=list)  # x_{i+1} after every iteration (if kept)
    relres: list = field(default_factory=list)  # true relres after every iteration


def cg(A, b, x1, tol: float = 1e-10, max_iters: int = 100000, ar=None, keep_iterates=False):
    ar = ar if ar is not None else CR()
    b = ar.vec(b)
    x = ar.vec(x1)
    nb = None if ar.exact else ar.sqrt(ar.dot(b, b))
    r = true_residual(ar, A, b, x)
    p = r
    rr = ar.dot(r, r)
    out = CGResult(x=x, status=NOT_CONVERGED)
    if rr == 0:
        out.status = OK
        return out
    for i in range(max_iters):
        w = ar.csr_comb(A, p)
        den = ar.dot(p, w)
        if den == 0 or (not ar.exact and not den > 0.0):
            out.status = BREAKDOWN
            break
        alpha = ar.div(rr, den)
        q = ar.scale(alpha, p)
        x = ar.axpy(ar.scalar(1), q, x)
        r = ar.sub(r, ar.csr_comb(A, q))
        rr1 = ar.dot(r, r)
        beta = ar.div(rr1, rr)
        p = ar.axpy(beta, p, r)
        rr = rr1
        out.alphas.append(alpha)
        out.betas.append(beta)
        out.iters = i + 1
        if keep_iterates:
            out.xs.append(x)
        if ar.exact:
            if rr == 0:
                out.status = OK
                break
            continue
        rel = relres_of(ar, A, b, x, nb)
        out.relres.append(rel)
        if rel <= tol:
            out.status = OK
            break
    out.x = x
    return out
