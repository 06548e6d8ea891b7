"""TLR format, compression and the left-looking TLR factorizations (oracle O3-O7).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The factorization follows the paper's "Left Looking TLR Cholesky" (Section
4.3) and "Left Looking TLR LDL^T" (Section 5.3) column by column, with one
change: the randomized compression of every updated tile (the ARA step of
Section 4.2) is replaced by the optimal one, a truncated SVD of the assembled
Schur-complement tile.  The truncation keeps the singular values above the
per-tile absolute threshold tau (2-norm criterion).  Everything else -- the
order of the columns, the left-looking update of Eq. (1) (Eq. (3) for
LDL^T), the dense diagonal factorization and the triangular solve that turns
the projected factor B into V -- is the paper's.

Layout conventions (shared with the GPU library only by specification, not
by code):
* N is padded up to nb*m; the padded part of the last diagonal tile is the
  identity and the padded rows of U and V are zero (the paper pads the last
  block row and column, Section 6).
* Tile (i, j) with i > j is stored as U_ij (m x r) and V_ij (m x r) with
  A_ij ~ U_ij V_ij^T; A_ji = A_ij^T is implied.
"""
from __future__ import annotations

from typing import Dict, Optional, Tuple

import numpy as np

from . import dense


class NotSPDTile(Exception):
    """Dense Cholesky of an updated diagonal tile failed (Section 5.1)."""

    def __init__(self, k: int):
        super().__init__("diagonal tile %d is not positive definite after its update" % k)
        self.k = k


class ZeroPivotTile(Exception):
    """Unpivoted LDL^T of an updated diagonal tile met a zero pivot."""

    def __init__(self, k: int, index: int):
        super().__init__("zero pivot in diagonal tile %d, local row %d" % (k, index))
        self.k = k
        self.index = index


class TLR:
    """Symmetric tile low rank matrix (Section 1, Figure 1).

    diag[k]  : m x m dense diagonal tile k
    u[i, j], v[i, j] : m x r_ij factors of the off-diagonal tile (i > j)
    For a factor L, diag[k] is L_kk (lower; unit lower for LDL^T) and
    (i, j) holds L_ij = U_ij V_ij^T.
    """

    def __init__(self, n: int, m: int):
        self.n = int(n)
        self.m = int(m)
        self.nb = -(-self.n // self.m)
        self.diag = [np.eye(self.m) for _ in range(self.nb)]
        self.u: Dict[Tuple[int, int], np.ndarray] = {}
        self.v: Dict[Tuple[int, int], np.ndarray] = {}

    @property
    def npad(self) -> int:
        return self.nb * self.m

    def rank(self, i: int, j: int) -> int:
        return int(self.u[i, j].shape[1])

    def ranks(self) -> np.ndarray:
        """nb x nb int32 array, ranks of the strictly lower tiles, 0 elsewhere."""
        out = np.zeros((self.nb, self.nb), dtype=np.int32)
        for (i, j), u in self.u.items():
            out[i, j] = u.shape[1]
        return out

    def tile(self, i: int, j: int) -> np.ndarray:
        """Dense m x m tile (i, j) of the symmetric matrix."""
        if i == j:
            return self.diag[i]
        if i > j:
            return self.u[i, j] @ self.v[i, j].T
        return (self.u[j, i] @ self.v[j, i].T).T

    def blk(self, k: int) -> slice:
        return slice(k * self.m, (k + 1) * self.m)

    def dense_symmetric(self) -> np.ndarray:
        """Expand the symmetric matrix (padded size)."""
        a = np.zeros((self.npad, self.npad))
        for i in range(self.nb):
            for j in range(self.nb):
                a[self.blk(i), self.blk(j)] = self.tile(i, j)
        return a

    def dense_lower(self) -> np.ndarray:
        """Expand a lower triangular factor L (padded size)."""
        a = np.zeros((self.npad, self.npad))
        for i in range(self.nb):
            a[self.blk(i), self.blk(i)] = np.tril(self.diag[i])
            for j in range(i):
                a[self.blk(i), self.blk(j)] = self.u[i, j] @ self.v[i, j].T
        return a

    def memory_doubles(self) -> int:
        return self.nb * self.m * self.m + 2 * self.m * int(self.ranks().sum())


# ---------------------------------------------------------------------------
# Compression of an explicit tile (oracle O3)
# ---------------------------------------------------------------------------

def truncate_svd(s_tile: np.ndarray, tau: float):
    """Optimal low rank form Q B^T of a tile at absolute 2-norm threshold tau.

    Keeps the rho singular values sigma_j > tau: Q = u[:, :rho] (orthonormal,
    the basis the paper's ARA approximates) and B = v[:, :rho] diag(sigma), so
    that ||S - Q B^T||_2 = sigma_{rho+1} <= tau.  Returns Q, B and the
    singular values.
    """
    u, s, vt = np.linalg.svd(s_tile)
    rho = int(np.count_nonzero(s > tau))
    return u[:, :rho].copy(), (vt[:rho].T * s[:rho]).copy(), s


def pad_dense(a: np.ndarray, m: int) -> np.ndarray:
    """Pad an N x N matrix to nb*m with an identity block (Section 6 padding)."""
    n = a.shape[0]
    nb = -(-n // m)
    out = np.eye(nb * m)
    out[:n, :n] = a
    return out


def compress_dense(a: np.ndarray, m: int, tau: float) -> TLR:
    """TLR form of a dense symmetric matrix (Section 1): diagonal tiles copied,
    each strictly lower tile replaced by its truncated SVD at threshold tau."""
    n = a.shape[0]
    t = TLR(n, m)
    ap = pad_dense(a, m)
    for i in range(t.nb):
        t.diag[i] = ap[t.blk(i), t.blk(i)].copy()
        for j in range(i):
            t.u[i, j], t.v[i, j] = _compress_padded(ap[t.blk(i), t.blk(j)], _nreal(n, m, i), tau)
    return t


def _nreal(n: int, m: int, i: int) -> int:
    return max(0, min(m, n - i * m))


def _compress_padded(tile: np.ndarray, rows: int, tau: float):
    """Truncated SVD of the real rows of a tile; padded rows of U stay zero."""
    q, b, _ = truncate_svd(tile[:rows], tau)
    u = np.zeros((tile.shape[0], q.shape[1]))
    u[:rows] = q
    return u, b


def kernel_tile(points: np.ndarray, m: int, i: int, j: int, kernel: int, ell: float,
                diag_add: float) -> np.ndarray:
    """Tile (i, j) of the padded covariance matrix, generated from the points."""
    n = points.shape[0]
    r0, r1 = i * m, min((i + 1) * m, n)
    c0, c1 = j * m, min((j + 1) * m, n)
    out = np.zeros((m, m))
    if r1 > r0 and c1 > c0:
        out[:r1 - r0, :c1 - c0] = dense.covariance_block(points, slice(r0, r1), slice(c0, c1),
                                                          kernel, ell, diag_add)
    if i == j:
        for g in range(r1 - r0, m):
            out[g, g] = 1.0
    return out


def compress_kernel(points: np.ndarray, m: int, kernel: int, ell: float, diag_add: float,
                    tau: float) -> TLR:
    """TLR form of a covariance matrix built tile by tile, never densely."""
    n = points.shape[0]
    t = TLR(n, m)
    for i in range(t.nb):
        t.diag[i] = kernel_tile(points, m, i, i, kernel, ell, diag_add)
        for j in range(i):
            t.u[i, j], t.v[i, j] = _compress_padded(kernel_tile(points, m, i, j, kernel, ell, diag_add),
                                                    _nreal(n, m, i), tau)
    return t


# ---------------------------------------------------------------------------
# Left-looking TLR factorizations (oracle O4 / O5)
# ---------------------------------------------------------------------------

def schur_tile(a: TLR, l: TLR, i: int, k: int, d: Optional[list] = None) -> np.ndarray:
    """Assembled left-looking update of tile (i, k), Eq. (1):

        S_ik = A_ik - sum_{j<k} U_ij V_ij^T V_kj U_kj^T

    and, for LDL^T, Eq. (3) with D_jj between the two V factors.
    """
    s = a.tile(i, k).copy()
    for j in range(k):
        mid = l.v[i, j].T @ (l.v[k, j] if d is None else d[j][:, None] * l.v[k, j])
        s -= l.u[i, j] @ (mid @ l.u[k, j].T)
    return s


def tlr_cholesky(a: TLR, tau: float, shift: float = 0.0, record: Optional[dict] = None,
                 modified: bool = False, schur_comp: bool = False) -> TLR:
    """Left-looking TLR Cholesky with exact recompression (oracle O4).

    Column k (Algorithm "Left Looking TLR Cholesky"):
      1. updateDense: A_kk + shift*I - sum_j L_kj L_kj^T   (Eq. (1) with i = k)
      2. L_kk = chol(.)                                     (LAPACK dpotrf)
      3. for every i > k: S_ik from Eq. (1), S_ik ~ Q B^T by truncated SVD
         (stands in for cholARAUpdate)
      4. V_ik = L_kk^{-1} B (the batched triangular solve: Q B^T L_kk^{-T}
         = Q (L_kk^{-1} B)^T), U_ik = Q.
    The shift is the paper's diagonal shift A + sI (Section 5.1); it is
    applied to the real rows only, not to the padding.  With `modified`, step
    2 is the modified Cholesky of Section 5.1.2 (dense.cholesky_modified with
    delta = tau): a tile that lost definiteness is factored with its
    non-positive pivots raised to tau; record["modified"] (when record is
    given) receives the number of raised pivots.  With `schur_comp`, step 1
    adds the Schur compensation of Section 5.1.1: the accumulated update
    D_k = sum_j L_kj L_kj^T is compressed to tau and the absolute row sums of
    what the compression drops go to the diagonal,
    A_kk - D_k + diag(dense.schur_compensation(D_k, tau)); record["comp"][k]
    receives that vector.
    `record`, when given, receives per-tile truncation errors sigma_{rho+1}.
    """
    l = TLR(a.n, a.m)
    m = a.m
    nreal = [min(m, a.n - k * m) for k in range(a.nb)]
    for k in range(a.nb):
        dk = a.diag[k].copy()
        dk[np.arange(nreal[k]), np.arange(nreal[k])] += shift
        upd = np.zeros((m, m))
        for j in range(k):
            g = l.v[k, j].T @ l.v[k, j]
            upd += l.u[k, j] @ (g @ l.u[k, j].T)
        dk -= upd
        if schur_comp and k > 0:
            c = dense.schur_compensation(upd, tau)
            dk[np.arange(m), np.arange(m)] += c
            if record is not None:
                record.setdefault("comp", {})[k] = c
        if modified:
            l.diag[k], f = dense.cholesky_modified(dk, tau)
            if record is not None:
                record["modified"] = record.get("modified", 0) + int(np.count_nonzero(f))
        else:
            try:
                l.diag[k] = np.linalg.cholesky(dk)
            except np.linalg.LinAlgError:
                raise NotSPDTile(k)
        for i in range(k + 1, a.nb):
            q, b, s = truncate_svd(schur_tile(a, l, i, k), tau)
            l.u[i, k] = q
            l.v[i, k] = dense.solve_lower(l.diag[k], b)
            if record is not None:
                record[i, k] = float(s[q.shape[1]]) if q.shape[1] < len(s) else 0.0
    return l


def tlr_cholesky_pivoted(a: TLR, tau: float, shift: float = 0.0):
    """Pivoted left-looking TLR Cholesky with exact recompression (Section 5.2,
    Algorithm "Pivoted Left Looking TLR Cholesky").

    Symmetric tile pivoting on the diagonal: at step k every remaining
    diagonal tile is updated with all the low rank products of the columns
    already factored (the sums D_i of Section 5.2), the pivot is the position
    p >= k whose updated tile A(i, i) - D_i has the largest Frobenius norm
    (the norm the paper prefers over the 2-norm; ties go to the first), block
    rows and columns k and p are swapped, and the column then proceeds as in
    the unpivoted algorithm: dense Cholesky of the updated diagonal tile,
    truncated SVD of every Schur-complement tile of Eq. (1), triangular solve.

    Returns (L, perm) with L the factor of P A P^T in the permuted block
    order: position t of P A P^T is the original block perm[t].  The shift
    is added to the real rows of every original block, as in tlr_cholesky.
    """
    nb, m = a.nb, a.m
    perm = list(range(nb))
    nreal = [min(m, a.n - b * m) for b in range(nb)]
    l = TLR(a.n, a.m)

    def tile(pi, pj):
        return a.tile(perm[pi], perm[pj])

    for k in range(nb):
        upd = []
        for t in range(k, nb):
            d = tile(t, t).copy()
            nr = nreal[perm[t]]
            d[np.arange(nr), np.arange(nr)] += shift
            for j in range(k):
                d -= l.u[t, j] @ ((l.v[t, j].T @ l.v[t, j]) @ l.u[t, j].T)
            upd.append(d)
        p = k + int(np.argmax([np.linalg.norm(d, "fro") for d in upd]))
        if p != k:
            perm[k], perm[p] = perm[p], perm[k]
            for j in range(k):
                l.u[k, j], l.u[p, j] = l.u[p, j], l.u[k, j]
                l.v[k, j], l.v[p, j] = l.v[p, j], l.v[k, j]
            upd[0], upd[p - k] = upd[p - k], upd[0]
        try:
            l.diag[k] = np.linalg.cholesky(upd[0])
        except np.linalg.LinAlgError:
            raise NotSPDTile(k)
        for i in range(k + 1, nb):
            s = tile(i, k).copy()
            for j in range(k):
                s -= l.u[i, j] @ ((l.v[i, j].T @ l.v[k, j]) @ l.u[k, j].T)
            q, b, _ = truncate_svd(s, tau)
            l.u[i, k] = q
            l.v[i, k] = dense.solve_lower(l.diag[k], b)
    return l, perm


def permute(a: TLR, perm) -> TLR:
    """The TLR matrix P A P^T: position t holds the original block perm[t]
    (tile (i, j), i > j, of the result is A(perm[i], perm[j]) as a U V^T
    pair, transposed when perm[i] < perm[j])."""
    out = TLR(a.n, a.m)
    for i in range(a.nb):
        out.diag[i] = a.diag[perm[i]].copy()
        for j in range(i):
            bi, bj = perm[i], perm[j]
            if bi > bj:
                out.u[i, j], out.v[i, j] = a.u[bi, bj].copy(), a.v[bi, bj].copy()
            else:
                out.u[i, j], out.v[i, j] = a.v[bj, bi].copy(), a.u[bj, bi].copy()
    return out


def tlr_ldlt(a: TLR, tau: float, record: Optional[dict] = None):
    """Left-looking TLR LDL^T with exact recompression (oracle O5).

    Column k (Algorithm "Left Looking TLR LDL^T"):
      1. updateDenseLDL: A_kk - sum_j L_kj D_jj L_kj^T      (Eq. (3) with i = k)
      2. [L_kk, D_kk] = ldl(.), unpivoted with scalar pivots
      3. S_ik from Eq. (3), truncated SVD S_ik ~ Q B^T
      4. V_ik = D_kk^{-1} L_kk^{-1} B (triangular solve, then the inverse
         diagonal multiply), U_ik = Q.
    Returns (L, d) with d the list of diagonal blocks of D.
    """
    l = TLR(a.n, a.m)
    d = []
    for k in range(a.nb):
        dk = a.diag[k].copy()
        for j in range(k):
            g = l.v[k, j].T @ (d[j][:, None] * l.v[k, j])
            dk -= l.u[k, j] @ (g @ l.u[k, j].T)
        try:
            lk, dd = dense.ldlt_unpivoted(dk)
        except dense.ZeroPivot as exc:
            raise ZeroPivotTile(k, exc.index)
        l.diag[k] = lk
        d.append(dd)
        for i in range(k + 1, a.nb):
            q, b, s = truncate_svd(schur_tile(a, l, i, k, d), tau)
            l.u[i, k] = q
            l.v[i, k] = dense.solve_lower(lk, b, unit=True) / dd[:, None]
            if record is not None:
                record[i, k] = float(s[q.shape[1]]) if q.shape[1] < len(s) else 0.0
    return l, d


# ---------------------------------------------------------------------------
# Products and solves with TLR matrices (oracle O6 / O7)
# ---------------------------------------------------------------------------

def pad_vec(a: TLR, x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((a.npad,) + x.shape[1:])
    out[:a.n] = x
    return out


def matvec(a: TLR, x: np.ndarray) -> np.ndarray:
    """y = A x for the symmetric TLR matrix (Section 4.4): dense diagonal
    tiles, U (V^T x_j) below the diagonal and V (U^T x_i) above it."""
    xp = pad_vec(a, x)
    y = np.zeros_like(xp)
    for i in range(a.nb):
        y[a.blk(i)] += a.diag[i] @ xp[a.blk(i)]
        for j in range(i):
            u, v = a.u[i, j], a.v[i, j]
            y[a.blk(i)] += u @ (v.T @ xp[a.blk(j)])
            y[a.blk(j)] += v @ (u.T @ xp[a.blk(i)])
    return y[:a.n]


def lower_apply(l: TLR, x: np.ndarray, trans: bool = False, unit: bool = False) -> np.ndarray:
    """L x (or L^T x) for a lower TLR factor (padded input/output)."""
    y = np.zeros_like(x)
    for i in range(l.nb):
        lk = np.tril(l.diag[i], -1) + (np.eye(l.m) if unit else np.diag(np.diag(l.diag[i])))
        if trans:
            y[l.blk(i)] += lk.T @ x[l.blk(i)]
        else:
            y[l.blk(i)] += lk @ x[l.blk(i)]
        for j in range(i):
            u, v = l.u[i, j], l.v[i, j]
            if trans:
                y[l.blk(j)] += v @ (u.T @ x[l.blk(i)])
            else:
                y[l.blk(i)] += u @ (v.T @ x[l.blk(j)])
    return y


def solve(l: TLR, b: np.ndarray, d: Optional[list] = None) -> np.ndarray:
    """x = (L L^T)^{-1} b, or (L D L^T)^{-1} b (Algorithm "TLR Triangular Solve").

    Forward sweep: for k = 0..nb-1, x_k = L_kk^{-1} x_k, then every i > k
    receives x_i -= U_ik (V_ik^T x_k).  For LDL^T the diagonal D is applied
    next.  Backward sweep with L^T: for k = nb-1..0,
    x_k -= sum_{i>k} V_ik (U_ik^T x_i), then x_k = L_kk^{-T} x_k.
    """
    unit = d is not None
    x = pad_vec(l, b)
    for k in range(l.nb):
        x[l.blk(k)] = dense.solve_lower(l.diag[k], x[l.blk(k)], unit=unit)
        for i in range(k + 1, l.nb):
            x[l.blk(i)] -= l.u[i, k] @ (l.v[i, k].T @ x[l.blk(k)])
    if unit:
        dd = np.concatenate(d)
        x = x / (dd[:, None] if x.ndim == 2 else dd)
    for k in range(l.nb - 1, -1, -1):
        for i in range(k + 1, l.nb):
            x[l.blk(k)] -= l.v[i, k] @ (l.u[i, k].T @ x[l.blk(i)])
        x[l.blk(k)] = dense.solve_lower(l.diag[k], x[l.blk(k)], unit=unit, trans=True)
    return x[:l.n]


def factor_error_norm(a: TLR, l: TLR, d: Optional[list] = None, seed: int = 7,
                      iters: int = 30) -> float:
    """||A - L L^T||_2 (or ||A - L D L^T||_2) by power iteration (Section 6).

    A is applied as the TLR input, so the estimate isolates the error of the
    factorization from that of the input compression.
    """
    unit = d is not None
    dd = np.concatenate(d) if unit else None

    def apply(x):
        xp = pad_vec(a, x)
        y = lower_apply(l, xp, trans=True, unit=unit)
        if unit:
            y = y * dd
        y = lower_apply(l, y, unit=unit)
        return matvec(a, x) - y[:a.n]

    return dense.norm2_power(apply, a.n, seed=seed, iters=iters)


def norm2(a: TLR, seed: int = 11, iters: int = 20) -> float:
    """||A||_2 of a symmetric TLR matrix by power iteration."""
    return dense.norm2_power(lambda x: matvec(a, x), a.n, seed=seed, iters=iters, rtol=0.0)


# ---------------------------------------------------------------------------
# SVD post-recompression of the low rank tiles (Section 6.2)
# ---------------------------------------------------------------------------

def recompress(t: TLR, tau: float) -> TLR:
    """Minimal-rank form of every strictly lower tile at threshold tau.

    Section 6.2 observes that the ranks the ARA finds sit a few percent above
    the smallest ones the threshold allows, and that a post-processing pass
    applying the SVD to each low rank tile reduces them to that minimum.
    Each tile U V^T is expanded and replaced by its truncated SVD
    (truncate_svd: the singular values above tau are kept, U orthonormal,
    V = right vectors times singular values); the diagonal tiles are copied.
    Returns a new TLR of the same kind (matrix or factor).
    """
    out = TLR(t.n, t.m)
    out.diag = [d.copy() for d in t.diag]
    for (i, j), u in t.u.items():
        q, b, _ = truncate_svd(u @ t.v[i, j].T, tau)
        out.u[i, j], out.v[i, j] = q, b
    return out
