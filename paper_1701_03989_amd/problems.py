"""Seeded synthetic inputs (no arithmetic of the method lives here).

The paper's experiments use five small matrices of a public sparse-matrix
collection (Section 5, Table 1), which are not available here.  These
generators stand in for them with SPD systems of the shapes the workloads name:

  * Dirichlet Poisson matrices (5-point 2-D, 7-point 3-D), rows in
    lexicographic order with x fastest, T = tridiag(-1, 2, -1) per dimension;
  * a variable-coefficient 2-D finite-volume diffusion matrix with a
    log-normal coefficient field;
  * random weighted graph Laplacians plus a diagonal shift.

Every random draw comes from ``numpy.random.default_rng(seed)`` (PCG64).
CSR arrays: rowptr int32[n+1], col int32[nnz] (ascending within a row),
val float64[nnz].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def n(self) -> int:
        return int(self.rowptr.size - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.size)

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """Plain FP64 product (input generation only, e.g. b = A x_true)."""
        return self.to_scipy() @ x


def _stencil_csr(dims: tuple[int, ...], diag: float) -> CSR:
    """Dirichlet Laplacian on a grid, lexicographic order (first dim fastest)."""
    n = int(np.prod(dims))
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for d in dims:
        coords.append(rem % d)
        rem //= d
    # offsets in ascending column order: -stride_last .. -1, 0, +1 .. +stride_last
    offs = []
    for ax in reversed(range(len(dims))):
        offs.append((ax, -1))
    offs.append((None, 0))
    for ax in range(len(dims)):
        offs.append((ax, +1))
    cols = []
    vals = []
    masks = []
    for ax, sgn in offs:
        if ax is None:
            m = np.ones(n, dtype=bool)
            c = idx
            v = np.full(n, diag)
        else:
            if sgn < 0:
                m = coords[ax] > 0
            else:
                m = coords[ax] < dims[ax] - 1
            c = idx + sgn * strides[ax]
            v = np.full(n, -1.0)
        masks.append(m)
        cols.append(c)
        vals.append(v)
    M = np.stack(masks, axis=1)
    C = np.stack(cols, axis=1)
    V = np.stack(vals, axis=1)
    counts = M.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = C[M].astype(np.int32)
    val = V[M].astype(np.float64)
    return CSR(rowptr.astype(np.int32), col, val)


def poisson2d(N: int, Ny: int | None = None) -> CSR:
    """5-point Dirichlet Poisson on an N x Ny grid (diagonal 4)."""
    return _stencil_csr((N, Ny if Ny else N), 4.0)


def poisson3d(N: int) -> CSR:
    """7-point Dirichlet Poisson on an N^3 grid (diagonal 6)."""
    return _stencil_csr((N, N, N), 6.0)


def uniform(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)


def from_dense(M: np.ndarray) -> CSR:
    """CSR of the nonzero pattern of a dense matrix (tests only)."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    rowptr = [0]
    col = []
    val = []
    for i in range(n):
        for j in range(n):
            if M[i, j] != 0.0:
                col.append(j)
                val.append(M[i, j])
        rowptr.append(len(col))
    return CSR(np.array(rowptr, dtype=np.int32), np.array(col, dtype=np.int32),
               np.array(val, dtype=np.float64))


def random_spd_integer(n: int, seed: int, density: float = 0.5, maxval: int = 3) -> np.ndarray:
    """Small dense SPD matrix with integer entries: symmetric random off-diagonal
    integers and a strictly dominant integer diagonal."""
    rng = np.random.default_rng(seed)
    M = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < density:
                v = float(rng.integers(-maxval, maxval + 1))
                M[i, j] = M[j, i] = v
    for i in range(n):
        M[i, i] = float(np.abs(M[i]).sum() + rng.integers(1, 4))
    return M


def graph_laplacian(n: int, seed: int, avg_degree: int = 8, wlo: float = 0.1,
                    whi: float = 1.0, shift_frac: float = 1e-3) -> CSR:
    """Weighted Laplacian of a random graph with about avg_degree*n/2 distinct
    edges (weights U[wlo, whi]) plus shift_frac * (max weighted degree) * I."""
    rng = np.random.default_rng(seed)
    m = avg_degree * n // 2
    i = rng.integers(0, n, size=2 * m)
    j = rng.integers(0, n, size=2 * m)
    keep = i != j
    i, j = i[keep], j[keep]
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    key = np.unique(lo.astype(np.int64) * n + hi)
    key = np.sort(rng.permutation(key)[:m])  # m distinct edges, uniformly among the drawn
    lo = key // n
    hi = key % n
    w = rng.uniform(wlo, whi, size=key.size)
    rows = np.concatenate([lo, hi])
    cols = np.concatenate([hi, lo])
    ws = np.concatenate([w, w])
    deg = np.bincount(rows, weights=ws, minlength=n)
    shift = shift_frac * deg.max()
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([cols, np.arange(n)])
    vals = np.concatenate([-ws, deg + shift])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return CSR(rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


# ---------------------------------------------------------------- workloads

def poisson2d_32_system(seed: int = 0):
    """2-D 5-point Poisson on 32x32 (n = 1024): x_true ~ U[-1,1], b = A x_true,
    x_1 = 0.  The small parity workload."""
    A = poisson2d(32)
    x_true = uniform(A.n, seed)
    b = A.matvec(x_true)
    return A, b, np.zeros(A.n), x_true


def poisson3d_128_system(seed: int = 0, N: int = 128):
    """3-D 7-point Poisson on N^3 (128^3: n = 2,097,152), b ~ U[-1,1], x_1 = 0.
    The single-solve throughput workload."""
    A = poisson3d(N)
    b = uniform(A.n, seed)
    return A, b, np.zeros(A.n)


@dataclass
class BatchSystem:
    """One system of a batch: A x = b from x_1 = 0, with a Chebyshev interval
    [lmin, lmax] that contains the spectrum of A."""
    A: CSR
    b: np.ndarray
    lmin: float
    lmax: float
    kind: str


def poisson_interval(N: int, dim: int) -> tuple[float, float]:
    """Extreme eigenvalues of the Dirichlet Poisson matrix on N^dim points (a
    sum of dim copies of tridiag(-1, 2, -1), whose eigenvalues are
    4 sin^2(k pi / (2(N+1)))): 4*dim*sin^2(pi / (2(N+1))) and
    4*dim*cos^2(pi / (2(N+1)))."""
    t = np.pi / (2 * (N + 1))
    return 4 * dim * np.sin(t) ** 2, 4 * dim * np.cos(t) ** 2


def batch_systems(count: int, seed: int = 0, nlo: float = 1e3, nhi: float = 2e5):
    """A batch of uneven SPD systems: sizes n_i = round(exp(U[ln nlo, ln nhi]));
    even i: Dirichlet Poisson, alternating 2-D (N = round(sqrt n_i)) and 3-D
    (N = round(cbrt n_i)), interval in closed form; odd i: graph Laplacian of
    n_i nodes with 4 n_i distinct edges (average degree 8), weights U[0.1, 1],
    plus delta*I with delta = 1e-3 * (max weighted degree), interval
    [delta, Gershgorin bound 2 * max degree + delta].  b ~ U[-1, 1] with seed
    seed + 1000 + i; the graph of system i uses seed + i."""
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(np.log(nlo), np.log(nhi), size=count))).astype(np.int64)
    out = []
    for i, ni in enumerate(sizes):
        if i % 2 == 0:
            if (i // 2) % 2 == 0:
                N = max(2, int(round(np.sqrt(ni))))
                A, (lo, hi), kind = poisson2d(N), poisson_interval(N, 2), f"poisson2d_{N}"
            else:
                N = max(2, int(round(np.cbrt(ni))))
                A, (lo, hi), kind = poisson3d(N), poisson_interval(N, 3), f"poisson3d_{N}"
        else:
            A = graph_laplacian(int(ni), seed + i)
            rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
            on = rows == A.col
            diag = np.zeros(A.n)
            diag[rows[on]] = A.val[on]
            deg = np.bincount(rows[~on], weights=np.abs(A.val[~on]), minlength=A.n)
            # L + delta I: spectrum in [delta, max_i (2 deg_i + delta)] (Gershgorin)
            lo, hi, kind = float(np.min(diag - deg)), float(np.max(diag + deg)), f"graph_{A.n}"
        out.append(BatchSystem(A, uniform(A.n, seed + 1000 + i), float(lo), float(hi), kind))
    return out


def lognormal_field(N: int, seed: int, sigma: float = 2.0, corr: float = 16.0) -> np.ndarray:
    """k = exp(sigma * g) on N x N cells, g a unit-variance Gaussian random field
    with covariance exp(-r^2 / (2 corr^2)) (r in cells), sampled by circulant
    embedding: white noise filtered with the square root of the covariance's
    spectrum on a periodic 2N x 2N grid, the N x N corner kept and scaled to
    unit sample variance."""
    M = 2 * N
    rng = np.random.default_rng(seed)
    d = np.minimum(np.arange(M), M - np.arange(M)).astype(np.float64)
    cov = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2.0 * corr * corr))
    spec = np.sqrt(np.maximum(np.fft.rfft2(cov).real, 0.0))
    noise = rng.standard_normal((M, M))
    g = np.fft.irfft2(np.fft.rfft2(noise) * spec, s=(M, M))[:N, :N]
    g = (g - g.mean()) / g.std()
    return np.exp(sigma * g)


def diffusion2d(k: np.ndarray) -> CSR:
    """Cell-centred finite volumes for -div(k grad u) on the unit-spaced N x N
    grid (rows in lexicographic order, x fastest), Dirichlet boundary: face
    transmissibility 2 k_i k_j / (k_i + k_j) between cells, 2 k_i on a
    boundary face; A = sum of transmissibilities on the diagonal, minus each
    on its neighbour's column.  Symmetric positive definite."""
    N = k.shape[0]
    kk = k.astype(np.float64)
    tx = 2.0 * kk[:, :-1] * kk[:, 1:] / (kk[:, :-1] + kk[:, 1:])  # faces between (i, j), (i, j+1)
    ty = 2.0 * kk[:-1, :] * kk[1:, :] / (kk[:-1, :] + kk[1:, :])  # faces between (i, j), (i+1, j)
    diag = np.zeros((N, N))
    diag[:, :-1] += tx
    diag[:, 1:] += tx
    diag[:-1, :] += ty
    diag[1:, :] += ty
    diag[:, 0] += 2.0 * kk[:, 0]
    diag[:, -1] += 2.0 * kk[:, -1]
    diag[0, :] += 2.0 * kk[0, :]
    diag[-1, :] += 2.0 * kk[-1, :]
    idx = np.arange(N * N).reshape(N, N)
    rows = [idx.ravel(), idx[:, :-1].ravel(), idx[:, 1:].ravel(), idx[:-1, :].ravel(),
            idx[1:, :].ravel()]
    cols = [idx.ravel(), idx[:, 1:].ravel(), idx[:, :-1].ravel(), idx[1:, :].ravel(),
            idx[:-1, :].ravel()]
    vals = [diag.ravel(), -tx.ravel(), -tx.ravel(), -ty.ravel(), -ty.ravel()]
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(N * N + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=N * N), out=rowptr[1:])
    return CSR(rowptr.astype(np.int32), c.astype(np.int32), v)


def diffusion2d_system(N: int = 2048, seed: int = 0, sigma: float = 2.0, corr: float = 16.0):
    """Variable-coefficient diffusion on N x N (2048^2: n = 4,194,304) with a
    log-normal coefficient field (seed), b ~ U[-1, 1] (seed + 1), x_1 = 0."""
    A = diffusion2d(lognormal_field(N, seed, sigma, corr))
    return A, uniform(A.n, seed + 1), np.zeros(A.n)
