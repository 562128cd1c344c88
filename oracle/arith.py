"""Arithmetic back-ends for the oracle (test infrastructure only).

The method's algorithms in ``oracle/sstep.py`` and ``oracle/cg.py`` are
written once against the small interface below, so the same code runs

* in FP64 with correctly rounded reductions (``CR``), the reading this oracle
  takes of the paper's plain double-precision arithmetic (Section 5): every row
  sum, inner product and row-wise linear combination is the double nearest to
  its exact value, except the Gram matrix, whose entries are plain FP64 fused
  multiply-add chains in a stated order (fma over the rows of each 1024-row
  group in order, then pairwise summation of the group partials); every other
  operation is a single IEEE operation; and
* in exact rational arithmetic (``Exact``), which pins the algorithms to their
  exact-arithmetic identities (s-step CG and CG produce the same iterates,
  Section 2; CG terminates in at most n steps); and
* in plain FP64 (``Plain``): every reduction is an ordinary FP64 library sum
  (numpy / scipy, order unspecified), as in the paper's MATLAB runs.  Used to
  time the oracle (no correctly rounded sums), never as a parity reference.

Vectors of length n are numpy arrays (CR) or lists of Fractions (Exact);
small coordinate vectors and matrices are Python lists in both.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import native


def ieee_div(a: float, b: float) -> float:
    """a / b with IEEE-754 semantics (Python raises on division by zero)."""
    if b == 0.0:
        if a == 0.0 or a != a:
            return math.nan
        return math.copysign(math.inf, a) * math.copysign(1.0, b)
    return a / b


def ieee_sqrt(a: float) -> float:
    if a != a or a < 0.0:
        return math.nan
    return math.sqrt(a)


class CR:
    """FP64, correctly rounded reductions (order independent)."""

    exact = False
    name = "cr"

    # -- long vectors ------------------------------------------------------
    def vec(self, x):
        return np.array(x, dtype=np.float64)

    def zeros(self, n):
        return np.zeros(n, dtype=np.float64)

    def csr_comb(self, A, u, extra=()):
        """RN(A u + sum_e c_e v_e), row by row."""
        return native.cr_csr_rowsum(A.rowptr, A.col, A.val, u, extra)

    def vdiv(self, v, g: float):
        if g == 1.0:
            return v.copy()
        return v / g

    def axpy(self, alpha, x, y):
        """y + alpha*x elementwise, two roundings (no fused multiply-add)."""
        return y + alpha * x

    def scale(self, alpha, x):
        return alpha * x

    def sub(self, x, y):
        return x - y

    def neg(self, x):
        return -x

    def dot(self, x, y) -> float:
        return native.cr_dot(x, y)

    def gram(self, cols):
        """G = Y^T Y with the stated order of R9 for Gram matrices: IEEE fma
        chains over groups of 1024 rows, group partials added pairwise (the
        reduction a device's FP64 matrix instructions reproduce)."""
        return native.ord_gram(cols).tolist()

    def rows_comb(self, cols, coef, base=None):
        return native.cr_rows_comb(cols, coef, base)

    # -- scalars and small vectors ----------------------------------------
    def scalar(self, v):
        return float(v)

    def div(self, a, b):
        return ieee_div(a, b)

    def sqrt(self, a):
        return ieee_sqrt(a)

    def sdot(self, a, b) -> float:
        return native.cr_dot(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64))

    def smatvec(self, M, v):
        vv = np.asarray(v, dtype=np.float64)
        return [native.cr_dot(np.asarray(row, dtype=np.float64), vv) for row in M]

    def isfinite(self, a) -> bool:
        return math.isfinite(a)


class Exact:
    """Exact rational arithmetic (fractions.Fraction)."""

    exact = True
    name = "exact"

    def vec(self, x):
        return [Fraction(v) for v in x]

    def zeros(self, n):
        return [Fraction(0)] * n

    def csr_comb(self, A, u, extra=()):
        n = len(A.rowptr) - 1
        out = []
        for i in range(n):
            s = Fraction(0)
            for k in range(int(A.rowptr[i]), int(A.rowptr[i + 1])):
                s += Fraction(A.val[k]) * u[int(A.col[k])]
            for c, v in extra:
                s += Fraction(c) * v[i]
            out.append(s)
        return out

    def vdiv(self, v, g):
        g = Fraction(g)
        return [x / g for x in v]

    def axpy(self, alpha, x, y):
        return [yi + alpha * xi for xi, yi in zip(x, y)]

    def scale(self, alpha, x):
        return [alpha * xi for xi in x]

    def sub(self, x, y):
        return [a - b for a, b in zip(x, y)]

    def neg(self, x):
        return [-a for a in x]

    def dot(self, x, y):
        return sum((a * b for a, b in zip(x, y)), Fraction(0))

    def gram(self, cols):
        d = len(cols)
        return [[self.dot(cols[a], cols[b]) for b in range(d)] for a in range(d)]

    def rows_comb(self, cols, coef, base=None):
        n = len(cols[0])
        out = []
        for i in range(n):
            s = base[i] if base is not None else Fraction(0)
            for a, c in enumerate(coef):
                s += cols[a][i] * c
            out.append(s)
        return out

    def scalar(self, v):
        return Fraction(v)

    def div(self, a, b):
        return Fraction(a) / Fraction(b)

    def sqrt(self, a):
        raise TypeError("square roots are not rational; the exact back-end runs Alg. 1-3 only")

    def sdot(self, a, b):
        return sum((x * y for x, y in zip(a, b)), Fraction(0))

    def smatvec(self, M, v):
        return [self.sdot(row, v) for row in M]

    def isfinite(self, a) -> bool:
        return True


class Plain(CR):
    """FP64 with plain library reductions (numpy / scipy sparse): the same
    algorithms and operation sequence as CR, but sums are not correctly
    rounded.  For timing the CPU oracle only."""

    name = "plain"

    def __init__(self):
        self._csr = {}

    def _mat(self, A):
        import scipy.sparse as sp

        key = id(A)
        hit = self._csr.get(key)
        if hit is None or hit[0] is not A:
            n = len(A.rowptr) - 1
            m = sp.csr_matrix((np.asarray(A.val, dtype=np.float64), np.asarray(A.col),
                               np.asarray(A.rowptr)), shape=(n, n))
            hit = (A, m)
            self._csr[key] = hit
        return hit[1]

    def csr_comb(self, A, u, extra=()):
        out = self._mat(A) @ np.asarray(u, dtype=np.float64)
        for c, v in extra:
            out = out + c * v
        return out

    def dot(self, x, y) -> float:
        return float(np.dot(x, y))

    def gram(self, cols):
        Y = np.stack(cols, axis=1)
        return (Y.T @ Y).tolist()

    def rows_comb(self, cols, coef, base=None):
        out = np.stack(cols, axis=1) @ np.asarray(coef, dtype=np.float64)
        return out if base is None else base + out

    def sdot(self, a, b) -> float:
        return float(np.dot(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)))

    def smatvec(self, M, v):
        return (np.asarray(M, dtype=np.float64) @ np.asarray(v, dtype=np.float64)).tolist()
