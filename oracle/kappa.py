"""Condition numbers of the leading sub-Gram matrices (test infrastructure only).

Section 4.2 chooses the block size from kappa(Y_{k,i}) = sqrt(kappa(G_{k,i})),
the 2-norm condition number, for each candidate i (eq. condy), and notes that
the estimate need not be very accurate.  This oracle takes kappa(G) as the
ratio of the largest to the smallest eigenvalue of the symmetric matrix G,
with kappa = +inf when the smallest computed eigenvalue is not positive.

Eigenvalues come from the two-sided cyclic Jacobi method (Golub & Van Loan,
Matrix Computations, Sec. 8.5: the symmetric 2x2 Schur decomposition and the
parallel round-robin ordering).  Jacobi is chosen because it resolves small
eigenvalues of graded positive definite matrices to high relative accuracy
(Demmel & Veselic 1992), which matters for Gram matrices of unnormalised Krylov
bases.  The procedure is spelled out operation by operation so that the device
implementation, written separately, performs the same IEEE operations:

  * ordering: for m = k (k even) or k+1 (k odd, index k a dummy), step t of a
    sweep pairs positions (pos(i), pos(m-1-i)), i < m/2, where pos(0) = 0 and
    pos(i) = 1 + ((i - 1 + t) mod (m - 1)); a pair is stored as (p, q), p < q;
  * skip rule: a pair rotates only if |a_pq| > eps * (sqrt|a_pp| * sqrt|a_qq|);
  * rotation (from the values at the start of the step):
        tau = (a_qq - a_pp) / (2 a_pq)
        t   = sgn(tau) / (|tau| + sqrt(1 + tau*tau))   (sgn(0) = 1),
              or t = 0.5 / tau when |tau| > 1e150
        c   = 1 / sqrt(1 + t*t),  s = t*c;
    with self/partner weights (c, -s) for p and (c, s) for q;
  * all rotations of a step are applied at once: B = A J by columns
    (new_i = w_self*old_i + w_other*old_partner), then C = J^T B by rows, then
    the strict lower triangle is copied from the upper one, then for every
    rotated pair a_pp <- a_pp - t a_pq, a_qq <- a_qq + t a_pq, a_pq = a_qp = 0
    (start-of-step values);
  * a sweep is m-1 steps; stop after a sweep without rotations or 40 sweeps.
"""
from __future__ import annotations

import math

import numpy as np

EPS = 2.0 ** -53
MAX_SWEEPS = 40


def round_robin_pairs(k: int, t: int):
    m = k if k % 2 == 0 else k + 1
    pos = [0] + [1 + ((i - 1 + t) % (m - 1)) for i in range(1, m)]
    pairs = []
    for i in range(m // 2):
        a, b = pos[i], pos[m - 1 - i]
        p, q = min(a, b), max(a, b)
        if q < k:
            pairs.append((p, q))
    return pairs


def _rotation(app: float, aqq: float, apq: float):
    thr = EPS * (math.sqrt(abs(app)) * math.sqrt(abs(aqq)))
    if not (abs(apq) > thr):
        return None
    tau = (aqq - app) / (2.0 * apq)
    if abs(tau) > 1e150:
        t = 0.5 / tau
    else:
        sg = 1.0 if tau >= 0.0 else -1.0
        t = sg / (abs(tau) + math.sqrt(1.0 + tau * tau))
    c = 1.0 / math.sqrt(1.0 + t * t)
    s = t * c
    return c, s, t


def jacobi_eigenvalues(G) -> tuple[np.ndarray, int]:
    """Eigenvalues of the symmetric matrix G (diagonal after convergence) and
    the number of sweeps used."""
    A = np.array(G, dtype=np.float64)
    k = A.shape[0]
    if k == 1:
        return A.diagonal().copy(), 0
    m = k if k % 2 == 0 else k + 1
    sweeps = 0
    for sweep in range(MAX_SWEEPS):
        sweeps = sweep + 1
        rotated = 0
        for t in range(m - 1):
            rots = []
            for p, q in round_robin_pairs(k, t):
                r = _rotation(A[p, p], A[q, q], A[p, q])
                if r is not None:
                    rots.append((p, q) + r)
            if not rots:
                continue
            rotated += len(rots)
            idx = []
            other = []
            wself = []
            wother = []
            for p, q, c, s, _t in rots:
                idx += [p, q]
                other += [q, p]
                wself += [c, c]
                wother += [-s, s]
            idx = np.array(idx)
            other = np.array(other)
            wself = np.array(wself)
            wother = np.array(wother)
            B = A.copy()
            B[:, idx] = wself[None, :] * A[:, idx] + wother[None, :] * A[:, other]
            C = B.copy()
            C[idx, :] = wself[:, None] * B[idx, :] + wother[:, None] * B[other, :]
            low = np.tril_indices(k, -1)
            C[low] = C.T[low]
            for p, q, c, s, t_ in rots:
                app, aqq, apq = A[p, p], A[q, q], A[p, q]
                C[p, p] = app - t_ * apq
                C[q, q] = aqq + t_ * apq
                C[p, q] = 0.0
                C[q, p] = 0.0
            A = C
        if rotated == 0:
            break
    return A.diagonal().copy(), sweeps


def kappa_spd(G) -> float:
    """lambda_max / lambda_min of G, +inf unless lambda_min > 0 (finite)."""
    ev, _ = jacobi_eigenvalues(G)
    lmin = float(ev.min())
    lmax = float(ev.max())
    if not (lmin > 0.0) or not math.isfinite(lmax):
        return math.inf
    return lmax / lmin
