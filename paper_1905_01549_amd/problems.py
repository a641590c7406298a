"""Seeded synthetic problem generators (inputs only).

Every solver input used by the tests, the benchmark and the smoke check comes
from here: sparse symmetric positive definite matrices in CSR form (int32
``row_ptr``/``col_idx``, float64 ``values``, columns sorted within each row)
plus right-hand sides.  This module defines problems; it contains none of the
conjugate-gradient arithmetic, and both the CPU oracle and the GPU library
consume the identical arrays it returns.

Right-hand sides of the form ``b = A x*`` are formed with ``scipy.sparse``
(a library product used only to synthesise inputs).

The problem families follow the solver's workloads:

* 2D 5-point and 3D 7-point constant-coefficient Poisson matrices with
  Dirichlet boundaries eliminated;
* 2D anisotropic 5-point matrices (diagonal ``2*eps + 2``);
* a cell-centred 3D 27-point variable-coefficient diffusion matrix;
* a 3D 7-point finite-volume matrix with random face coefficients;
* the Strakos model spectrum of the paper's numerical section (eq. model),
  either as a diagonal matrix or rotated by a Haar-random orthogonal matrix;
* small test matrices (k distinct eigenvalues, random sparse SPD with ragged
  rows, arrowhead matrices with one long row, tiny integer SPD matrices).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    """A square sparse matrix in CSR form (int32 indices, float64 values)."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col_idx: np.ndarray  # int32[nnz]
    values: np.ndarray  # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.values, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        return self.scipy().toarray()

    def diagonal(self) -> np.ndarray:
        return self.scipy().diagonal().copy()


@dataclass
class Problem:
    """A matrix, a right-hand side and the run settings of one workload."""

    name: str
    A: CSR
    b: np.ndarray
    xstar: Optional[np.ndarray] = None
    precond: str = "none"  # "none" | "jacobi"
    tol: float = 1e-10
    maxit: int = 10000
    extra: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# CSR assembly for structured grids
# ----------------------------------------------------------------------------

def _grid_csr(shape, offsets, offdiag_value, diag_value) -> CSR:
    """Assemble a stencil matrix on a lexicographic grid.

    ``shape`` is (nz, ny, nx) with x fastest.  ``offsets`` is a list of
    (dz, dy, dx) including (0, 0, 0), sorted by linear offset so that the
    columns of each row come out sorted.  ``offdiag_value(j, valid)`` returns
    the float64[n] entries of offset j (only entries where ``valid`` is true
    are kept); ``diag_value()`` returns the diagonal.
    """
    nz, ny, nx = shape
    n = nz * ny * nx
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    k = len(offsets)
    cols = np.empty((n, k), dtype=np.int32)
    mask = np.empty((n, k), dtype=bool)
    vals = np.empty((n, k), dtype=np.float64)
    for j, (dz, dy, dx) in enumerate(offsets):
        valid = ((x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny)
                 & (z + dz >= 0) & (z + dz < nz))
        cols[:, j] = (idx + dz * nx * ny + dy * nx + dx).astype(np.int32, copy=False) * valid
        mask[:, j] = valid
        if (dz, dy, dx) == (0, 0, 0):
            vals[:, j] = diag_value()
        else:
            vals[:, j] = offdiag_value(j, valid)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds the int32 CSR limit")
    return CSR(n, row_ptr.astype(np.int32), cols[mask], vals[mask])


def _sorted_offsets(radius_set, dims):
    offs = []
    for dz in ([-1, 0, 1] if dims == 3 else [0]):
        for dy in [-1, 0, 1]:
            for dx in [-1, 0, 1]:
                if (dz * dz + dy * dy + dx * dx) in radius_set:
                    offs.append((dz, dy, dx))
    return offs  # lexicographic (dz, dy, dx) order == increasing linear offset


def poisson2d(nx: int, ny: Optional[int] = None) -> CSR:
    """5-point Laplacian on an nx-by-ny grid, Dirichlet boundary (diag 4, off -1)."""
    ny = nx if ny is None else ny
    offs = _sorted_offsets({0, 1}, 2)
    n = nx * ny
    return _grid_csr((1, ny, nx), offs, lambda j, v: np.full(n, -1.0), lambda: np.full(n, 4.0))


def poisson3d(nx: int, ny: Optional[int] = None, nz: Optional[int] = None) -> CSR:
    """7-point Laplacian on an nx-by-ny-by-nz grid, Dirichlet boundary (diag 6, off -1)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    offs = _sorted_offsets({0, 1}, 3)
    n = nx * ny * nz
    return _grid_csr((nz, ny, nx), offs, lambda j, v: np.full(n, -1.0), lambda: np.full(n, 6.0))


def aniso2d(nx: int, ny: int, eps: float) -> CSR:
    """Anisotropic 5-point operator: diag 2*eps+2, x-neighbours -eps, y-neighbours -1."""
    offs = _sorted_offsets({0, 1}, 2)
    n = nx * ny

    def off(j, v):
        dz, dy, dx = offs[j]
        return np.full(n, -eps if dx != 0 else -1.0)

    return _grid_csr((1, ny, nx), offs, off, lambda: np.full(n, 2.0 * eps + 2.0))


def varcoef27(m: int, seed: int, sigma: float = 1.0) -> CSR:
    """Cell-centred 27-point variable-coefficient diffusion on m^3 cells.

    Cell coefficients c ~ lognormal(0, sigma).  For each of the 26 offsets d,
    A_ij = -h(c_i, c_j)/|d|^2 with h the harmonic mean; the diagonal is the
    sum of those couplings plus c_i/|d|^2 for every offset that leaves the
    domain (Dirichlet ghost cells).  The result is a symmetric M-matrix with
    strict diagonal dominance on boundary rows, hence SPD.
    """
    rng = np.random.default_rng(seed)
    n = m ** 3
    c = rng.lognormal(0.0, sigma, size=n)
    offs = _sorted_offsets({0, 1, 2, 3}, 3)
    idx = np.arange(n, dtype=np.int64)
    x = idx % m
    y = (idx // m) % m
    z = idx // (m * m)

    def coupling(dz, dy, dx):
        d2 = float(dz * dz + dy * dy + dx * dx)
        valid = ((x + dx >= 0) & (x + dx < m) & (y + dy >= 0) & (y + dy < m)
                 & (z + dz >= 0) & (z + dz < m))
        cj = c[np.clip(idx + dz * m * m + dy * m + dx, 0, n - 1)]
        h = 2.0 * c * cj / (c + cj)
        return valid, h / d2, c / d2

    diag = np.zeros(n)
    for o in offs:
        if o == (0, 0, 0):
            continue
        valid, hd, gd = coupling(*o)
        diag += np.where(valid, hd, gd)

    def off(j, valid):
        return -coupling(*offs[j])[1]

    return _grid_csr((m, m, m), offs, off, lambda: diag)


def varcoef7(m: int, seed: int, sigma: float = 0.5) -> CSR:
    """7-point finite-volume diffusion on m^3 cells with random face coefficients.

    Each face (boundary faces included) carries a_f = exp(sigma * N(0,1)),
    drawn for x-faces, then y-faces, then z-faces.  A_ij = -a_f for the face
    shared by cells i and j; A_ii is the sum of the coefficients of all six
    faces of cell i (Dirichlet boundary faces included).
    """
    rng = np.random.default_rng(seed)
    ax = np.exp(sigma * rng.standard_normal((m, m, m + 1)))  # [z, y, xface]
    ay = np.exp(sigma * rng.standard_normal((m, m + 1, m)))  # [z, yface, x]
    az = np.exp(sigma * rng.standard_normal((m + 1, m, m)))  # [zface, y, x]
    n = m ** 3
    left = ax[:, :, :-1].reshape(n)
    right = ax[:, :, 1:].reshape(n)
    down = ay[:, :-1, :].reshape(n)
    up = ay[:, 1:, :].reshape(n)
    back = az[:-1, :, :].reshape(n)
    front = az[1:, :, :].reshape(n)
    offs = _sorted_offsets({0, 1}, 3)  # -z, -y, -x, 0, +x, +y, +z
    face = {(-1, 0, 0): back, (0, -1, 0): down, (0, 0, -1): left,
            (0, 0, 1): right, (0, 1, 0): up, (1, 0, 0): front}
    diag = left + right + down + up + back + front
    return _grid_csr((m, m, m), offs, lambda j, v: -face[offs[j]], lambda: diag)


def model_spectrum(n: int, lam1: float, lamn: float, rho: float) -> np.ndarray:
    """Strakos model spectrum (eq. model): lam_i = lam1 + (i-1)/(n-1)*(lamn-lam1)*rho^(n-i)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return lam1 + (i - 1.0) / (n - 1.0) * (lamn - lam1) * np.power(rho, n - i)


def diagonal_csr(d: np.ndarray) -> CSR:
    n = d.shape[0]
    return CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
               np.ascontiguousarray(d, dtype=np.float64))


def dense_csr(M: np.ndarray) -> CSR:
    """Store every entry of a dense matrix (zeros included) as CSR."""
    n = M.shape[0]
    row_ptr = (np.arange(n + 1, dtype=np.int64) * n).astype(np.int32)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    return CSR(n, row_ptr, col, np.ascontiguousarray(M, dtype=np.float64).reshape(-1).copy())


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with signs fixed."""
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))[None, :]


def model_dense(n: int, rho: float, kappa: float, seed: int) -> CSR:
    """Model problem of the numerical section: Q diag(lam) Q^T with lam_1 = 1/kappa, lam_n = 1."""
    rng = np.random.default_rng(seed)
    lam = model_spectrum(n, 1.0 / kappa, 1.0, rho)
    Q = haar_orthogonal(n, rng)
    M = (Q * lam[None, :]) @ Q.T
    M = 0.5 * (M + M.T)
    return dense_csr(M)


def kdistinct_diag(n: int, k: int) -> CSR:
    """Diagonal matrix whose eigenvalues are 1..k, each repeated about n/k times."""
    return diagonal_csr(1.0 + (np.arange(n) % k).astype(np.float64))


def random_spd(n: int, avg_offdiag: float, seed: int, diag_shift: float = 0.5) -> CSR:
    """Random sparse symmetric diagonally dominant matrix with ragged row lengths.

    Off-diagonal entries are negative, the diagonal is the absolute row sum
    plus U[diag_shift, diag_shift + 1], so the matrix is SPD and its diagonal
    varies from row to row.
    """
    rng = np.random.default_rng(seed)
    m = int(avg_offdiag * n / 2)
    i = rng.integers(0, n, size=m)
    j = rng.integers(0, n, size=m)
    keep = i != j
    i, j = i[keep], j[keep]
    w = rng.uniform(0.1, 1.0, size=i.shape[0])
    U = sp.coo_matrix((-w, (i, j)), shape=(n, n)).tocsr()
    U.sum_duplicates()
    S = (U + U.T).tocsr()
    rowsum = -np.asarray(S.sum(axis=1)).ravel()
    S = S + sp.diags(rowsum + rng.uniform(diag_shift, diag_shift + 1.0, size=n))
    S = S.tocsr()
    S.sort_indices()
    return CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))


def arrowhead(n: int, seed: int) -> CSR:
    """SPD arrowhead matrix: one dense first row/column, diagonal elsewhere."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(1.0, 2.0, size=n)
    off = rng.uniform(-1.0, 1.0, size=n - 1) / n
    d[0] = 2.0 + np.abs(off).sum()
    M = sp.diags(d).tolil()
    M[0, 1:] = off
    M[1:, 0] = off[:, None]
    S = M.tocsr()
    S.sort_indices()
    return CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))


def small_integer_spd(n: int, seed: int) -> np.ndarray:
    """Dense integer SPD matrix B^T B + I with small integer entries."""
    rng = np.random.default_rng(seed)
    B = rng.integers(-2, 3, size=(n, n))
    return (B.T @ B + np.eye(n, dtype=np.int64)).astype(np.int64)


def rhs_from_solution(A: CSR, xstar: np.ndarray) -> np.ndarray:
    return np.asarray(A.scipy() @ xstar, dtype=np.float64)


# ----------------------------------------------------------------------------
# The solver workloads
# ----------------------------------------------------------------------------

def config1(seed: int = 1) -> Problem:
    """2D Poisson 64x64 (n=4096), x* ~ U[-1,1], b = A x*, no preconditioner, tol 1e-10."""
    A = poisson2d(64)
    xs = np.random.default_rng(seed).uniform(-1.0, 1.0, A.n)
    return Problem("poisson2d_64", A, rhs_from_solution(A, xs), xs, "none", 1e-10, 10000)


def config2(seed: int = 2, m: int = 128) -> Problem:
    """3D Poisson m^3 (128^3: n=2,097,152), b ~ U[-1,1], Jacobi, fixed 1000 iterations."""
    A = poisson3d(m)
    b = np.random.default_rng(seed).uniform(-1.0, 1.0, A.n)
    return Problem(f"poisson3d_{m}_jacobi", A, b, None, "jacobi", 0.0, 1000)


def config3a(seed: int = 3, n: int = 1_000_000) -> Problem:
    """Diagonal Strakos spectrum, lam1=1e-3, lamn=1e3, rho=0.9, x* ~ U[-1,1], b = A x*."""
    A = diagonal_csr(model_spectrum(n, 1e-3, 1e3, 0.9))
    xs = np.random.default_rng(seed).uniform(-1.0, 1.0, n)
    return Problem(f"model_diag_{n}", A, rhs_from_solution(A, xs), xs, "none", 1e-10, 20000)


def config3b(seed: int = 3, m: int = 160) -> Problem:
    """27-point variable-coefficient diffusion on m^3 cells (160^3: n=4,096,000)."""
    A = varcoef27(m, seed)
    xs = np.random.default_rng(seed + 1000).uniform(-1.0, 1.0, A.n)
    return Problem(f"varcoef27_{m}", A, rhs_from_solution(A, xs), xs, "none", 1e-10, 20000)


def config5(seed: int = 5, m: int = 96) -> Problem:
    """7-point random-face-coefficient diffusion on m^3 cells, b ~ U[-1,1], w ~ N(0,1)."""
    A = varcoef7(m, seed)
    rng = np.random.default_rng(seed + 1000)
    b = rng.uniform(-1.0, 1.0, A.n)
    w = rng.standard_normal(A.n)
    return Problem(f"varcoef7_{m}", A, b, None, "none", 1e-10, 20000, {"w": w})


def batch_system(s: int, nmin: int = 1024, nmax: int = 65536):
    """System s of the batched workload: anisotropic 2D 5-point, b = A x*.

    n_target ~ U{nmin..nmax}; nx = round(sqrt(n_target)), ny = round(n_target/nx);
    eps = 10^U[-3,0]; x* ~ U[-1,1]; all drawn from default_rng(4000 + s).
    """
    rng = np.random.default_rng(4000 + s)
    nt = int(rng.integers(nmin, nmax + 1))
    nx = max(1, int(round(np.sqrt(nt))))
    ny = max(1, int(round(nt / nx)))
    eps = float(10.0 ** rng.uniform(-3.0, 0.0))
    A = aniso2d(nx, ny, eps)
    xs = rng.uniform(-1.0, 1.0, A.n)
    return A, rhs_from_solution(A, xs), xs, eps


def block_diag(mats):
    """Concatenate CSR matrices into one block-diagonal CSR plus row offsets (int64)."""
    n_tot = sum(M.n for M in mats)
    nnz_tot = sum(M.nnz for M in mats)
    if nnz_tot >= 2**31 or n_tot >= 2**31:
        raise ValueError("batch exceeds the int32 CSR limit")
    row_ptr = np.empty(n_tot + 1, dtype=np.int64)
    col = np.empty(nnz_tot, dtype=np.int32)
    val = np.empty(nnz_tot, dtype=np.float64)
    offs = np.zeros(len(mats) + 1, dtype=np.int64)
    r0 = 0
    e0 = 0
    for s, M in enumerate(mats):
        row_ptr[r0:r0 + M.n] = M.row_ptr[:-1].astype(np.int64) + e0
        col[e0:e0 + M.nnz] = M.col_idx + r0
        val[e0:e0 + M.nnz] = M.values
        r0 += M.n
        e0 += M.nnz
        offs[s + 1] = r0
    row_ptr[n_tot] = e0
    return CSR(n_tot, row_ptr.astype(np.int32), col, val), offs


def config4(nsys: int = 512, nmin: int = 1024, nmax: int = 65536):
    """Batched workload: nsys anisotropic systems of uneven size, block-diagonal CSR."""
    mats, bs, xss, epss = [], [], [], []
    for s in range(nsys):
        A, b, xs, eps = batch_system(s, nmin, nmax)
        mats.append(A)
        bs.append(b)
        xss.append(xs)
        epss.append(eps)
    A, offs = block_diag(mats)
    return A, offs, np.concatenate(bs), np.concatenate(xss), epss


def model_48_8_3(seed: int) -> Problem:
    """model_48_8_3 of Table 2: n=48, rho=0.8, kappa=1e3, Haar Q, x* = n^-1/2, x0 = 0."""
    A = model_dense(48, 0.8, 1e3, seed)
    xs = np.full(48, 1.0 / np.sqrt(48.0))
    return Problem("model_48_8_3", A, rhs_from_solution(A, xs), xs, "none", 0.0, 200)


def uniform_vector(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)
