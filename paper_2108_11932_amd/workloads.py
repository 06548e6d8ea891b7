"""Seeded synthetic inputs shared by the GPU path, the tests and the oracle.

This module draws points and names workload parameters.  It holds none of
the factorization arithmetic: no compression or factorization happens here.
The one kernel evaluation is input-side: matern3d_norm_estimate sums rows
of the unshifted Matern matrix to size the diagonal shift that makes the 3D
workload indefinite.

The paper's covariance test matrices (Section 6) come from spatial Gaussian
processes with an isotropic exponential kernel, correlation length 0.1 in 2D
and 0.2 in 3D, with points on a uniform grid.  The paper orders the points
with a KD-tree; the workloads here use a Morton (Z-order) space-filling curve
instead, which the paper names as an alternative ordering (Section 2 and
Section 6).  Grid points are jittered: one uniform point per cell.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

KERNEL_EXP = 0        # exp(-r / ell)
KERNEL_MATERN15 = 1   # (1 + sqrt(3) r / ell) exp(-sqrt(3) r / ell)

EPS_ABS = 0
EPS_REL = 1


def grid_shape(n: int, dim: int) -> tuple:
    """Split n = 2^p into `dim` powers of two that differ by at most 2x.

    The first dimensions receive the larger factors: 131072 in 2D is
    512 x 256, in 3D 64 x 64 x 32.
    """
    p = int(round(math.log2(n)))
    if 1 << p != n:
        raise ValueError("jittered grid needs N to be a power of two, got %d" % n)
    base, extra = divmod(p, dim)
    return tuple(1 << (base + (1 if d < extra else 0)) for d in range(dim))


def jittered_grid(n: int, dim: int, seed: int) -> np.ndarray:
    """One uniform point inside each cell of a grid over the unit cube.

    Cells are enumerated with the first coordinate varying slowest; the
    jitter is one `rng.random((n, dim))` draw from numpy's default_rng(seed).
    Returns an (n, dim) float64 array in cell order (not yet Morton-sorted).
    """
    shape = grid_shape(n, dim)
    rng = np.random.default_rng(seed)
    jitter = rng.random((n, dim))
    idx = np.indices(shape).reshape(dim, -1).T.astype(np.float64)
    return (idx + jitter) / np.asarray(shape, dtype=np.float64)


def uniform_points(n: int, dim: int, seed: int) -> np.ndarray:
    """n i.i.d. uniform points in the unit cube (default_rng(seed))."""
    rng = np.random.default_rng(seed)
    return rng.random((n, dim))


def morton_codes(points: np.ndarray) -> np.ndarray:
    """Morton keys of points in [0,1)^dim.

    Each coordinate is quantized to `bits` bits (31 in 2D, 21 in 3D), then the
    bits are interleaved from the most significant one down, first dimension
    first at every bit level.  Keys fit in a uint64.
    """
    n, dim = points.shape
    bits = {1: 62, 2: 31, 3: 21}[dim]
    scale = float(1 << bits)
    q = np.clip(np.floor(points * scale), 0, (1 << bits) - 1).astype(np.uint64)
    key = np.zeros(n, dtype=np.uint64)
    for b in range(bits - 1, -1, -1):
        for d in range(dim):
            key = (key << np.uint64(1)) | ((q[:, d] >> np.uint64(b)) & np.uint64(1))
    return key


def morton_order(points: np.ndarray) -> np.ndarray:
    """Stable argsort of the Morton keys (ties keep the input order)."""
    return np.argsort(morton_codes(points), kind="stable")


@dataclasses.dataclass
class Workload:
    """One synthetic TLR factorization problem.

    points   : (N, dim) float64, already Morton-ordered, C-contiguous
    kernel   : KERNEL_EXP or KERNEL_MATERN15
    ell      : correlation length
    diag_add : added to every diagonal entry (nugget, or a negative shift)
    m        : tile size
    eps      : compression threshold
    eps_mode : EPS_ABS (threshold is eps) or EPS_REL (eps times ||A||_2)
    bs       : ARA block size
    factor   : "chol" or "ldlt"
    """
    name: str
    points: np.ndarray
    kernel: int
    ell: float
    diag_add: float
    m: int
    eps: float
    eps_mode: int
    bs: int
    factor: str = "chol"
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def dim(self) -> int:
        return int(self.points.shape[1])

    @property
    def nb(self) -> int:
        return -(-self.n // self.m)


def covariance_2d(n: int, m: int, eps: float, seed: int, eps_mode: int = EPS_ABS,
                  ell: float = 0.1, bs: int = 16, name: Optional[str] = None) -> Workload:
    """2D exponential covariance on a jittered grid with nugget 1e-4."""
    pts = jittered_grid(n, 2, seed)
    pts = np.ascontiguousarray(pts[morton_order(pts)])
    return Workload(name or "cov2d_n%d_m%d" % (n, m), pts, KERNEL_EXP, ell, 1e-4,
                    m, eps, eps_mode, bs, "chol", seed)


# Diagonal shift of the 3D Matern workload: -1e-2 times an estimate of
# ||A||_2, the mean absolute row sum over 1024 seeded rows of the unshifted
# matrix (matern3d_norm_estimate).
MATERN3D_SHIFT_FRACTION = 1e-2


def matern3d_norm_estimate(points: np.ndarray, ell: float = 0.2, rows: int = 1024,
                           seed: int = 5) -> float:
    """Mean absolute row sum of the Matern-1.5 kernel matrix over `rows`
    rows drawn by default_rng(seed) (the kernel is positive, so this is the
    mean row sum; it lies between the smallest and the largest row sum, and
    for these smooth kernels close to ||A||_2)."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(points.shape[0], size=min(rows, points.shape[0]), replace=False)
    s = 3.0 ** 0.5 / ell
    tot = 0.0
    for i in idx:
        r = np.sqrt(((points - points[i]) ** 2).sum(axis=1)) * s
        tot += float(((1.0 + r) * np.exp(-r)).sum())
    return tot / len(idx)


def matern_3d(n: int, m: int, eps: float, seed: int, shift: float = 0.0,
              bs: int = 32, name: Optional[str] = None) -> Workload:
    """3D Matern-1.5 covariance (ell = 0.2) with a diagonal shift -shift."""
    pts = jittered_grid(n, 3, seed)
    pts = np.ascontiguousarray(pts[morton_order(pts)])
    return Workload(name or "matern3d_n%d_m%d" % (n, m), pts, KERNEL_MATERN15, 0.2, -shift,
                    m, eps, EPS_ABS, bs, "ldlt", seed)


def covariance_3d(n: int, m: int, eps: float, seed: int, ell: float = 0.2, bs: int = 32,
                  name: Optional[str] = None) -> Workload:
    """3D exponential covariance on a jittered grid with nugget 1e-4 (the
    paper's 3D covariance: ell 0.2, ARA block 32)."""
    pts = jittered_grid(n, 3, seed)
    pts = np.ascontiguousarray(pts[morton_order(pts)])
    return Workload(name or "cov3d_n%d_m%d" % (n, m), pts, KERNEL_EXP, ell, 1e-4,
                    m, eps, EPS_ABS, bs, "chol", seed)


def batched_2d(count: int = 96, seed: int = 999, eps: float = 1e-6,
               m: Optional[int] = None) -> List[Workload]:
    """Independent 2D exponential problems with uneven sizes.

    N_p = round(exp(U(ln 2048, ln 32768))) and ell_p ~ U(0.05, 0.3), both from
    default_rng(seed); problem p draws its i.i.d. uniform points from seed
    1000 + p and is Morton-ordered.  The last tile is padded when m does not
    divide N_p.
    """
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(2048), math.log(32768), count))).astype(int)
    ells = rng.uniform(0.05, 0.3, count)
    out = []
    for p in range(count):
        pts = uniform_points(int(ns[p]), 2, 1000 + p)
        pts = np.ascontiguousarray(pts[morton_order(pts)])
        out.append(Workload("batch%02d_n%d" % (p, ns[p]), pts, KERNEL_EXP, float(ells[p]), 1e-4,
                            m or 512, eps, EPS_REL, 16, "chol", 1000 + p))
    return out


def standard(name: str) -> Workload:
    """The named workloads the tests and the benchmark use.

    cov2d_4k     : N=4096, 64x64 grid, tile 256, eps 1e-6 (absolute), seed 1
    cov2d_32k    : N=32768, 256x128 grid, tile 512, eps 1e-6, seed 2
    cov2d_32k_lo : same points, eps 1e-2
    cov2d_131k   : N=131072, 512x256 grid, tile 1024, eps 1e-6, seed 3
    matern3d_131k: N=131072, 64x64x32 grid, 3D Matern-1.5 (ell 0.2), tile
                   1024, eps 1e-4, bs 32, diagonal shift -1e-2 ||A|| (LDL^T)
    cov3d_131k   : N=131072, 64x64x32 grid, 3D exponential (ell 0.2), tile
                   512, eps 1e-6, bs 32, seed 6 (pivoted against unpivoted)
    """
    if name == "cov2d_4k":
        return covariance_2d(4096, 256, 1e-6, 1, name=name)
    if name == "cov2d_32k":
        return covariance_2d(32768, 512, 1e-6, 2, name=name)
    if name == "cov2d_32k_lo":
        return covariance_2d(32768, 512, 1e-2, 2, name=name)
    if name == "cov2d_131k":
        return covariance_2d(131072, 1024, 1e-6, 3, name=name)
    if name == "matern3d_131k":
        w = matern_3d(131072, 1024, 1e-4, 4, name=name)
        w.diag_add = -MATERN3D_SHIFT_FRACTION * matern3d_norm_estimate(w.points)
        return w
    if name == "cov3d_131k":
        return covariance_3d(131072, 512, 1e-6, 6, name=name)
    raise KeyError(name)
