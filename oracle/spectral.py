"""Spectral interval for the Chebyshev basis (test infrastructure only).

The paper names the Chebyshev basis as a better-conditioned alternative to
the monomial one (Sections 2 and 5) without fixing its parameters.  This
oracle takes the interval [lambda_min, lambda_max] as
  * lambda_max: the Gershgorin bound max_i sum_j |a_ij|, and
  * lambda_min: the smallest Ritz value of an m-step Lanczos run (no
    re-orthogonalisation) started from a SplitMix64 vector,
and the tridiagonal Ritz problem is solved with the oracle's Jacobi method.
"""
from __future__ import annotations

import numpy as np

from .arith import CR
from .kappa import jacobi_eigenvalues

_M64 = (1 << 64) - 1


def splitmix64(seed: int, i: int) -> int:
    """Output i of SplitMix64 (Steele, Lea & Flood 2014) seeded with `seed`:
    state_i = seed + (i+1)*0x9E3779B97F4A7C15, then the published mixer."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def start_vector(n: int, seed: int) -> np.ndarray:
    """u_i = (splitmix64(seed, i) >> 11) * 2^-52 - 1, uniform on [-1, 1)."""
    z = (np.arange(1, n + 1, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
         + np.uint64(seed & _M64))
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0


def gershgorin_max(A, ar=None) -> float:
    """max_i sum_j |a_ij| (each row sum correctly rounded with CR)."""
    ar = ar if ar is not None else CR()
    absval = np.abs(np.asarray(A.val, dtype=np.float64))

    class _Abs:
        rowptr, col, val = A.rowptr, A.col, absval

    ones = np.ones(len(A.rowptr) - 1)
    return float(np.max(ar.csr_comb(_Abs, ones)))


def lanczos_tridiag(A, m: int, seed: int, ar=None):
    """m Lanczos steps on A from start_vector(n, seed); returns (alphas, betas).

    v_1 = u/||u||;  w = A v_j - beta_{j-1} v_{j-1} (one rounding per row);
    alpha_j = w.v_j;  w = w - alpha_j v_j;  beta_j = ||w||;  v_{j+1} = w / beta_j.
    Stops early if beta_j = 0 (invariant subspace)."""
    ar = ar if ar is not None else CR()
    n = len(A.rowptr) - 1
    u = start_vector(n, seed)
    nu = ar.sqrt(ar.dot(u, u))
    v = u / nu
    v_prev = None
    beta_prev = 0.0
    alphas, betas = [], []
    for j in range(m):
        extra = [(-beta_prev, v_prev)] if v_prev is not None else []
        w = ar.csr_comb(A, v, extra)
        alpha = ar.dot(w, v)
        w = w - alpha * v
        beta = ar.sqrt(ar.dot(w, w))
        alphas.append(alpha)
        if j == m - 1 or beta == 0.0:
            break
        betas.append(beta)
        v_prev = v
        v = w / beta
        beta_prev = beta
    return alphas, betas


def ritz_values(alphas, betas) -> np.ndarray:
    k = len(alphas)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = alphas[i]
    for i in range(k - 1):
        T[i, i + 1] = betas[i]
        T[i + 1, i] = betas[i]
    ev, _ = jacobi_eigenvalues(T)
    return np.sort(ev)


def chebyshev_interval(A, m: int = 30, seed: int = 0, ar=None) -> tuple[float, float]:
    a, b = lanczos_tridiag(A, m, seed, ar)
    rv = ritz_values(a, b)
    return float(rv[0]), gershgorin_max(A, ar)


def leja_order(points) -> list:
    """Leja ordering of real points: first the one of largest modulus, then
    repeatedly the one maximising prod_i |z - z_i| over the points already
    chosen (the product taken left to right in the order of choice, plain FP64);
    ties go to the earliest point of the given order.  Used as the shifts of the
    Newton basis, the ordering the Newton-basis references cited in Section 2 use
    for stability."""
    pts = [float(z) for z in points]
    left = list(range(len(pts)))
    order = []
    best = max(left, key=lambda i: (abs(pts[i]), -i))
    order.append(best)
    left.remove(best)
    while left:
        def score(i):
            prod = 1.0
            for c in order:
                prod = prod * abs(pts[i] - pts[c])
            return prod
        best = left[0]
        bs = score(best)
        for i in left[1:]:
            sc = score(i)
            if sc > bs:
                best, bs = i, sc
        order.append(best)
        left.remove(best)
    return [pts[i] for i in order]


def newton_shifts(A, m: int, seed: int = 0) -> list:
    """m shifts of the Newton basis: the Ritz values of an m-step Lanczos run
    from start_vector(n, seed) (Jacobi eigenvalues of the tridiagonal matrix,
    ascending), Leja ordered; repeated cyclically if the run stopped early."""
    a, b = lanczos_tridiag(A, m, seed)
    z = leja_order(ritz_values(a, b))
    return [z[i % len(z)] for i in range(m)]
