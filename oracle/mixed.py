"""The FP32 stages of the mixed-precision solve (test infrastructure only).

The mixed-precision form iterates classical FP64 iterative refinement
x_{j+1} = x_j + d_j around inner solves A d_j ~= r_j whose Krylov basis is
stored in FP32.  The paper's closing section (Section 6) notes that eq. fb
could equally fix s and choose the precision of each outer loop; the split
below is this oracle's own reading of such a mixed-precision method, and it
fixes what the inner stages compute:

  * matrix powers in FP32 (``mpk32_basis``): the matrix values are rounded to
    FP32 entry by entry; each new basis entry is
        RN32( (RN64(... RN64(RN64(a_1 u_1) + a_2 u_2) ...) - theta u - sigma w) / gamma )
    i.e. the products of FP32 values are exact in FP64 and are added in FP64
    in the row's CSR order, the three-term correction and the division by
    gamma are single FP64 operations, and the result is rounded once to FP32
    (eq. polybasiscg with FP32 storage);
  * the Gram matrix of the FP32 basis (``gram32``): G = Y^T Y of the FP32
    columns widened to FP64, in the stated order of the FP64 Gram (fma chains
    over 1024-row groups, group partials added pairwise; the products of FP32
    values are exact in FP64, so each fma is one rounding of a sum).

Everything else of the inner solve (kappa, eqs. condy and check with the FP32
unit round-off 2^-24, the coefficient recurrence, d_j) is the FP64 algorithm of
``oracle.sstep`` applied to these quantities.
"""
from __future__ import annotations

import numpy as np

from .arith import CR

EPS32 = 2.0 ** -24  # unit round-off of the FP32 basis (R1 for FP32)


def to_f32(v) -> np.ndarray:
    """Round FP64 values to FP32 (IEEE round to nearest even)."""
    return np.asarray(v, dtype=np.float64).astype(np.float32)


def mpk32_step(A, val32, u, w, j: int, basis: str, lmin=None, lmax=None) -> np.ndarray:
    """rho_j(A) v in FP32 from u = rho_{j-1}(A) v and w = rho_{j-2}(A) v (FP32
    vectors), as defined in the module docstring.  val32: A's values rounded to
    FP32.  Monomial: theta = sigma = 0, gamma = 1; Chebyshev on [lmin, lmax]:
    theta = (lmax + lmin) / 2, gamma_0 = h, gamma_j = h / 2, sigma = h / 2 with
    h = (lmax - lmin) / 2 (the same parameters as the FP64 oracle)."""
    n = len(A.rowptr) - 1
    a = np.asarray(val32, dtype=np.float32).astype(np.float64)
    uu = np.asarray(u, dtype=np.float32).astype(np.float64)
    rowptr = np.asarray(A.rowptr)
    col = np.asarray(A.col)
    lens = np.diff(rowptr)
    acc = np.zeros(n)
    # term t of every row at once: acc = RN64(acc + a_t u_t), in CSR order
    for t in range(int(lens.max()) if n else 0):
        m = t < lens
        k = rowptr[:-1][m] + t
        acc[m] = acc[m] + a[k] * uu[col[k]]
    if basis == "monomial":
        return acc.astype(np.float32)
    if basis != "chebyshev":
        raise ValueError(basis)
    c0 = (lmax + lmin) * 0.5
    h = (lmax - lmin) * 0.5
    h2 = h * 0.5
    num = acc - c0 * uu
    if j >= 2:
        num = num - h2 * np.asarray(w, dtype=np.float32).astype(np.float64)
    return (num / (h if j == 1 else h2)).astype(np.float32)


def mpk32_basis(A, s: int, first: bool, basis: str, p0, r0, lmin=None, lmax=None):
    """P_0..P_s and (unless first) R_0..R_{s-1} in FP32 (lists of arrays)."""
    val32 = to_f32(A.val)
    P = [to_f32(p0)]
    for j in range(1, s + 1):
        P.append(mpk32_step(A, val32, P[j - 1], P[j - 2] if j >= 2 else None, j, basis, lmin,
                            lmax))
    if first:
        return P, []
    R = [to_f32(r0)]
    for j in range(1, s):
        R.append(mpk32_step(A, val32, R[j - 1], R[j - 2] if j >= 2 else None, j, basis, lmin,
                            lmax))
    return P, R


def gram32(cols) -> np.ndarray:
    """Gram matrix of FP32 columns (FP64 result), in the stated order."""
    return np.array(CR().gram([np.asarray(c, dtype=np.float32).astype(np.float64)
                               for c in cols]))


def gram32_tolerance(cols) -> np.ndarray:
    """n eps64 sum_i |y_ia y_ib|: how far any FP64 summation order of the exact
    products may lie from the exact Gram (standard bound for recursive
    summation)."""
    Y = np.abs(np.stack([np.asarray(c, dtype=np.float32).astype(np.float64) for c in cols]))
    n = Y.shape[1]
    return n * 2.0 ** -53 * (Y @ Y.T)
