"""Dense FP64 reference computations (oracle O2).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Everything here is the textbook definition written out with numpy/scipy
(LAPACK) in float64: the covariance matrix of the paper's Section 6
workloads, dense Cholesky, dense unpivoted LDL^T with scalar pivots, and
triangular solves.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

KERNEL_EXP = 0
KERNEL_MATERN15 = 1


def kernel_values(r: np.ndarray, kernel: int, ell: float) -> np.ndarray:
    """Isotropic covariance kernel of the distance r (Section 6).

    exp:        exp(-r/ell)                         (the paper's kernel)
    Matern-1.5: (1 + sqrt(3) r/ell) exp(-sqrt(3) r/ell)   (closed form for nu = 3/2)
    """
    if kernel == KERNEL_EXP:
        return np.exp(-r / ell)
    if kernel == KERNEL_MATERN15:
        s = math.sqrt(3.0) * r / ell
        return (1.0 + s) * np.exp(-s)
    raise ValueError("unknown kernel %r" % kernel)


def distances(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Euclidean distances between the rows of x and the rows of y."""
    d = x[:, None, :] - y[None, :, :]
    return np.sqrt(np.sum(d * d, axis=2))


def covariance_block(points: np.ndarray, rows: slice, cols: slice, kernel: int, ell: float,
                     diag_add: float) -> np.ndarray:
    """Block A[rows, cols] of the covariance matrix K(x_a, x_b) + diag_add * I."""
    r0, r1 = rows.start, rows.stop
    c0, c1 = cols.start, cols.stop
    blk = kernel_values(distances(points[r0:r1], points[c0:c1]), kernel, ell)
    lo, hi = max(r0, c0), min(r1, c1)
    for g in range(lo, hi):
        blk[g - r0, g - c0] += diag_add
    return blk


def covariance_matrix(points: np.ndarray, kernel: int, ell: float, diag_add: float) -> np.ndarray:
    """The full N x N covariance matrix (only for N small enough to hold)."""
    n = points.shape[0]
    return covariance_block(points, slice(0, n), slice(0, n), kernel, ell, diag_add)


class NotSPD(Exception):
    """Dense Cholesky met a non-positive pivot."""


class ZeroPivot(Exception):
    """Unpivoted LDL^T met a pivot that is zero to working accuracy."""

    def __init__(self, index):
        super().__init__("zero pivot at %d" % index)
        self.index = index


def cholesky(a: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor by LAPACK dpotrf (through numpy)."""
    try:
        return np.linalg.cholesky(a)
    except np.linalg.LinAlgError as exc:
        raise NotSPD(str(exc))


def cholesky_modified(a: np.ndarray, delta: float):
    """Modified Cholesky of a symmetric tile (Section 5.1.2, "Modified
    Cholesky in Diagonal Tiles"), with the diagonal modification made as the
    pivots are met: column by column, d_j = a_jj - sum_{p<j} L_jp^2; a pivot
    d_j <= 0 is replaced by max(|d_j|, delta) (the sign flip of the
    Gill-Murray-Wright and Schnabel-Eskow modified Cholesky, which keeps the
    pivot as large as the loss it repairs, so the later columns do not
    grow); L_jj = sqrt(d_j) and L_ij = (a_ij - sum_{p<j} L_ip L_jp) / L_jj.
    Then L L^T = a + diag(f) with f_j = max(|d_j|, delta) - d_j >= 0 for the
    replaced pivots and 0 elsewhere (f = 0, L the Cholesky factor, for a
    positive definite a).  Returns (L, f)."""
    n = a.shape[0]
    lo = np.tril(np.array(a, dtype=np.float64))
    ell = np.zeros((n, n))
    f = np.zeros(n)
    for j in range(n):
        d = lo[j, j] - np.dot(ell[j, :j], ell[j, :j])
        if not d > 0.0:
            dm = max(abs(d), delta)
            f[j] = dm - d
            d = dm
        ell[j, j] = math.sqrt(d)
        if j + 1 < n:
            ell[j + 1:, j] = (lo[j + 1:, j] - ell[j + 1:, :j] @ ell[j, :j]) / ell[j, j]
    return ell, f


def schur_compensation(d: np.ndarray, tau: float) -> np.ndarray:
    """Diagonal Schur compensation of an accumulated update (Section 5.1.1).

    d is the symmetric positive semidefinite update D_k = sum_j L_kj L_kj^T
    of a diagonal tile.  D_k compressed to the threshold tau is its
    truncated eigen-decomposition Dbar = sum_{lambda_j > tau} lambda_j v_j
    v_j^T (the optimal 2-norm approximation, error max dropped lambda <=
    tau); the difference D_k - Dbar (positive semidefinite) is added to the
    diagonal as its absolute row sums.  Returns the vector c with
    c_i = sum_j |(D_k - Dbar)_ij|; the compensated tile is
    A_kk - D_k + diag(c)."""
    lam, v = np.linalg.eigh(np.asarray(d, dtype=np.float64))
    drop = lam <= tau
    e = (v[:, drop] * lam[drop]) @ v[:, drop].T
    return np.abs(e).sum(axis=1)


def ldlt_unpivoted(a: np.ndarray, breakdown: float = 64.0):
    """Unpivoted scalar LDL^T: a = L diag(d) L^T with L unit lower triangular.

    Column-by-column definition: d_j = a_jj - sum_{p<j} L_jp^2 d_p and
    L_ij = (a_ij - sum_{p<j} L_ip L_jp d_p) / d_j.  Raises ZeroPivot when
    |d_j| <= breakdown * u * ||a||_F (u = 2^-53).
    """
    n = a.shape[0]
    lo = np.tril(np.array(a, dtype=np.float64))
    ell = np.eye(n)
    d = np.zeros(n)
    limit = breakdown * np.finfo(np.float64).eps / 2 * np.linalg.norm(a)
    for j in range(n):
        w = ell[j, :j] * d[:j]
        d[j] = lo[j, j] - np.dot(ell[j, :j], w)
        if abs(d[j]) <= limit:
            raise ZeroPivot(j)
        if j + 1 < n:
            ell[j + 1:, j] = (lo[j + 1:, j] - ell[j + 1:, :j] @ w) / d[j]
    return ell, d


def solve_lower(l: np.ndarray, b: np.ndarray, unit: bool = False, trans: bool = False) -> np.ndarray:
    """Solve L x = b (or L^T x = b) with LAPACK's triangular solver."""
    return sla.solve_triangular(l, b, lower=True, unit_diagonal=unit, trans=1 if trans else 0)


def norm2_power(apply, n: int, seed: int = 7, iters: int = 30, rtol: float = 1e-3) -> float:
    """2-norm of a symmetric operator by power iteration (Section 6 verification).

    Start from a seeded Gaussian vector; stop after `iters` steps or when the
    estimate changes by less than rtol relative.
    """
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n)
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = apply(x)
        new = float(np.linalg.norm(y))
        if new == 0.0:
            return 0.0
        x = y / new
        if lam > 0 and abs(new - lam) <= rtol * new:
            lam = new
            break
        lam = new
    return lam
