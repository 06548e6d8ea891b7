"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test ties the oracle to something other than itself: a library routine
the special case reduces to, an exactly low rank construction, the backward
error identity of the left-looking method, hand-computed fixtures or
published known-answer vectors.  All run on the CPU.
"""
import math
import os

import numpy as np
import pytest

from oracle import bookkeeping as bk
from oracle import dense
from oracle import philox
from oracle import tlr
from paper_2108_11932_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cov(n, m, seed=5, ell=0.1, dim=2, kernel=dense.KERNEL_EXP, nugget=1e-4):
    if n & (n - 1) == 0:
        pts = wl.jittered_grid(n, dim, seed)
    else:
        pts = wl.uniform_points(n, dim, seed)
    pts = pts[wl.morton_order(pts)]
    return pts, dense.covariance_matrix(pts, kernel, ell, nugget)


# ---------------------------------------------------------------- generators

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox_kat.txt")) if not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        assert philox.philox4x32_10(tuple(w[0:4]), tuple(w[4:6])) == tuple(w[6:10])


def test_box_muller_moments():
    z = philox.test_matrix(seed=12345, k=3, t=1, s=0, rows=4096, cols=4).ravel()
    assert abs(z.mean()) < 0.03
    assert abs(z.var() - 1.0) < 0.05
    # Kolmogorov-Smirnov distance to the normal CDF
    zs = np.sort(z)
    cdf = 0.5 * (1 + np.vectorize(math.erf)(zs / math.sqrt(2)))
    ks = np.max(np.abs(cdf - np.arange(1, len(zs) + 1) / len(zs)))
    assert ks < 1.63 / math.sqrt(len(zs))   # 1% critical value


def test_kernel_closed_forms():
    ell = 0.25
    r = np.array([0.0, ell, ell / math.sqrt(3.0)])
    e = dense.kernel_values(r, dense.KERNEL_EXP, ell)
    assert e[0] == 1.0 and abs(e[1] - math.exp(-1)) < 1e-15
    mt = dense.kernel_values(r, dense.KERNEL_MATERN15, ell)
    assert mt[0] == 1.0 and abs(mt[2] - 2.0 / math.e) < 1e-15


def test_grid_one_point_per_cell_and_shapes():
    assert wl.grid_shape(4096, 2) == (64, 64)
    assert wl.grid_shape(32768, 2) == (256, 128)
    assert wl.grid_shape(131072, 2) == (512, 256)
    assert wl.grid_shape(131072, 3) == (64, 64, 32)
    pts = wl.jittered_grid(1 << 10, 2, 3)
    shape = np.array(wl.grid_shape(1 << 10, 2))
    cells = np.floor(pts * shape).astype(int)
    keys = cells[:, 0] * shape[1] + cells[:, 1]
    assert sorted(keys.tolist()) == list(range(1 << 10))


def test_morton_order_hand_computed():
    # 4x4 grid, cell (a, b) has key a1 b1 a0 b0 (first coordinate first).
    pts = wl.jittered_grid(16, 2, 0)
    order = wl.morton_order(pts)
    assert order.tolist() == [0, 1, 4, 5, 2, 3, 6, 7, 8, 9, 12, 13, 10, 11, 14, 15]


# ---------------------------------------------------------------- dense oracle

def test_ldlt_hand_computed():
    vals = [l.split() for l in open(os.path.join(GOLDEN, "ldlt_3x3.txt")) if not l.startswith("#")]
    a = np.array(vals[0:3], dtype=float)
    lref = np.array(vals[3:6], dtype=float)
    dref = np.array(vals[6], dtype=float)
    l, d = dense.ldlt_unpivoted(a)
    assert np.array_equal(l, lref) and np.array_equal(d, dref)


def test_ldlt_reduces_to_cholesky_on_spd():
    _, a = _cov(256, 256)
    l, d = dense.ldlt_unpivoted(a)
    assert np.all(d > 0)
    c = np.linalg.cholesky(a)
    np.testing.assert_allclose(l * np.sqrt(d)[None, :], c, rtol=0, atol=1e-10)


def test_ldlt_inertia_sylvester():
    rng = np.random.default_rng(0)
    n = 60
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([-rng.uniform(1, 3, 17), rng.uniform(1, 3, n - 17)])
    a = (q * lam) @ q.T
    l, d = dense.ldlt_unpivoted(a)
    assert int(np.sum(d < 0)) == 17
    np.testing.assert_allclose(l @ np.diag(d) @ l.T, a, atol=1e-9)


def test_ldlt_zero_pivot_detected():
    a = np.array([[1.0, 1.0], [1.0, 1.0]])
    with pytest.raises(dense.ZeroPivot):
        dense.ldlt_unpivoted(a)


def test_power_iteration_norm():
    _, a = _cov(300, 300)
    est = dense.norm2_power(lambda x: a @ x, 300, iters=200, rtol=0)
    assert abs(est - np.linalg.norm(a, 2)) < 1e-8 * est


# ---------------------------------------------------------------- TLR compression

def test_compress_truncation_is_optimal():
    _, a = _cov(512, 128)
    tau = 1e-6
    t = tlr.compress_dense(a, 128, tau)
    for (i, j), u in t.u.items():
        blk = a[i * 128:(i + 1) * 128, j * 128:(j + 1) * 128]
        s = np.linalg.svd(blk, compute_uv=False)
        assert u.shape[1] == int(np.sum(s > tau))
        err = np.linalg.norm(blk - u @ t.v[i, j].T, 2)
        tail = s[u.shape[1]] if u.shape[1] < len(s) else 0.0
        assert abs(err - tail) <= 1e-12 * s[0] + 1e-15
        np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-12)


def test_compress_kernel_matches_dense_and_pads():
    pts, a = _cov(300, 128)
    t1 = tlr.compress_dense(a, 128, 1e-8)
    t2 = tlr.compress_kernel(pts, 128, dense.KERNEL_EXP, 0.1, 1e-4, 1e-8)
    assert t1.nb == t2.nb == 3
    assert np.array_equal(t1.ranks(), t2.ranks())
    np.testing.assert_allclose(t1.dense_symmetric(), t2.dense_symmetric(), atol=1e-12)
    # padding: identity on the padded diagonal, zero rows in U and V
    last = t2.diag[2]
    assert np.array_equal(last[44:, 44:], np.eye(84)) and not last[44:, :44].any()
    for j in range(2):
        assert not t2.u[2, j][44:].any()


def test_matvec_matches_dense():
    _, a = _cov(320, 64)
    t = tlr.compress_dense(a, 64, 1e-9)
    x = np.random.default_rng(1).standard_normal((320, 3))
    np.testing.assert_allclose(tlr.matvec(t, x), t.dense_symmetric()[:320, :320] @ x, atol=1e-10)


# ---------------------------------------------------------------- TLR Cholesky

def test_single_tile_is_dense_cholesky():
    _, a = _cov(128, 128)
    t = tlr.compress_dense(a, 128, 1e-6)
    l = tlr.tlr_cholesky(t, 1e-6)
    np.testing.assert_array_equal(l.diag[0], np.linalg.cholesky(a))


def test_tiny_threshold_reproduces_lapack():
    _, a = _cov(512, 64)
    tau = 1e-14 * np.linalg.norm(a, 2)
    l = tlr.tlr_cholesky(tlr.compress_dense(a, 64, tau), tau)
    ref = np.linalg.cholesky(a)
    err = np.max(np.abs(l.dense_lower() - ref))
    assert err < 1e-9 * np.max(np.abs(ref))


def _low_rank_plus_blockdiag(n, m, r, indefinite=False, seed=3):
    rng = np.random.default_rng(seed)
    nb = n // m
    a = np.zeros((n, n))
    for k in range(nb):
        if indefinite:
            sgn = np.where(rng.random(m) < 0.3, -1.0, 1.0)
            b = np.diag(sgn * rng.uniform(5, 6, m)) + 0.05 * rng.standard_normal((m, m))
            b = 0.5 * (b + b.T)
        else:
            g = rng.standard_normal((m, m))
            b = g @ g.T / m + np.eye(m)
        a[k * m:(k + 1) * m, k * m:(k + 1) * m] = b
    w = rng.standard_normal((n, r))
    return a + w @ w.T


@pytest.mark.parametrize("indefinite", [False, True])
def test_exactly_low_rank_ranks_recovered(indefinite):
    # Off-diagonal tiles of blockdiag(B) + W W^T are W_i W_j^T, and every
    # Schur-updated tile stays W_i C_k W_k^T (Woodbury), so rank is exactly r.
    n, m, r = 384, 64, 3
    a = _low_rank_plus_blockdiag(n, m, r, indefinite)
    tau = 1e-8
    t = tlr.compress_dense(a, m, tau)
    assert set(t.ranks()[np.tril_indices(n // m, -1)].tolist()) == {r}
    if indefinite:
        l, d = tlr.tlr_ldlt(t, tau)
        dd = np.concatenate(d)
        rec = l.dense_lower() @ np.diag(dd) @ l.dense_lower().T
        assert int(np.sum(dd < 0)) == int(np.sum(np.linalg.eigvalsh(a) < 0))
    else:
        l = tlr.tlr_cholesky(t, tau)
        rec = l.dense_lower() @ l.dense_lower().T
    assert set(l.ranks()[np.tril_indices(n // m, -1)].tolist()) == {r}
    assert np.max(np.abs(rec - a)) < 1e-10 * np.max(np.abs(a))


@pytest.mark.parametrize("factor", ["chol", "ldlt"])
def test_backward_error_identity(factor):
    # Left-looking: (A - L L^T)_ik equals the compression error of tile (i, k)
    # for i > k, and vanishes on the diagonal tiles.
    pts, a = _cov(448, 64, seed=9)
    tau = 1e-5
    t = tlr.compress_dense(a, 64, tau)
    rec = {}
    if factor == "chol":
        l = tlr.tlr_cholesky(t, tau, record=rec)
        r = t.dense_symmetric() - l.dense_lower() @ l.dense_lower().T
    else:
        l, d = tlr.tlr_ldlt(t, tau, record=rec)
        ld = l.dense_lower()
        r = t.dense_symmetric() - ld @ np.diag(np.concatenate(d)) @ ld.T
    scale = np.linalg.norm(a, 2)
    for k in range(t.nb):
        blk = r[t.blk(k), t.blk(k)]
        assert np.linalg.norm(blk, 2) < 1e-12 * scale
        for i in range(k + 1, t.nb):
            e = np.linalg.norm(r[t.blk(i), t.blk(k)], 2)
            assert abs(e - rec[i, k]) < 1e-11 * scale
            assert rec[i, k] <= tau
    # the global error is bounded by the per-tile errors
    est = tlr.factor_error_norm(t, l, None if factor == "chol" else d, iters=60)
    assert abs(est - np.linalg.norm(r, 2)) < 1e-2 * np.linalg.norm(r, 2)
    assert est <= (t.nb - 1) * tau


def test_error_within_sqrt_nb_tau():
    pts, a = _cov(1024, 128, seed=1)
    for tau in (1e-6, 1e-3):
        t = tlr.compress_dense(a, 128, tau)
        l = tlr.tlr_cholesky(t, tau)
        est = tlr.factor_error_norm(t, l)
        assert est <= math.sqrt(t.nb) * tau


def test_shift_keeps_error_with_unshifted_matrix():
    pts, a = _cov(512, 64, seed=4)
    tau = 1e-3
    t = tlr.compress_dense(a, 64, tau)
    l = tlr.tlr_cholesky(t, tau, shift=tau)
    est = tlr.factor_error_norm(t, l)
    assert est <= math.sqrt(t.nb) * tau + tau


def test_not_spd_reported_at_first_failing_tile():
    pts, a = _cov(256, 64, seed=2)
    a2 = a.copy()
    a2[130, 130] = -5.0
    with pytest.raises(tlr.NotSPDTile) as exc:
        tlr.tlr_cholesky(tlr.compress_dense(a2, 64, 1e-8), 1e-8)
    assert exc.value.k == 2


def test_ldlt_matches_cholesky_on_spd():
    _, a = _cov(384, 64, seed=6)
    tau = 1e-13 * np.linalg.norm(a, 2)
    t = tlr.compress_dense(a, 64, tau)
    l, d = tlr.tlr_ldlt(t, tau)
    c = tlr.tlr_cholesky(t, tau)
    dd = np.concatenate(d)
    assert np.all(dd > 0)
    np.testing.assert_allclose(l.dense_lower() * np.sqrt(dd)[None, :], c.dense_lower(), atol=1e-9)


# ---------------------------------------------------------------- TLR solve

@pytest.mark.parametrize("factor", ["chol", "ldlt"])
def test_solve_matches_dense_triangular_solves(factor):
    _, a = _cov(400, 64, seed=8)
    tau = 1e-7
    t = tlr.compress_dense(a, 64, tau)
    b = np.random.default_rng(2).standard_normal((400, 2))
    if factor == "chol":
        l = tlr.tlr_cholesky(t, tau)
        ld = l.dense_lower()
        y = dense.solve_lower(ld, tlr.pad_vec(t, b))
        x_ref = dense.solve_lower(ld, y, trans=True)[:400]
        x = tlr.solve(l, b)
    else:
        l, d = tlr.tlr_ldlt(t, tau)
        ld = l.dense_lower()
        y = dense.solve_lower(ld, tlr.pad_vec(t, b), unit=True) / np.concatenate(d)[:, None]
        x_ref = dense.solve_lower(ld, y, unit=True, trans=True)[:400]
        x = tlr.solve(l, b, d)
    np.testing.assert_allclose(x, x_ref, rtol=1e-9, atol=1e-9 * np.max(np.abs(x_ref)))
    # and it solves the original system to the factorization accuracy
    res = np.linalg.norm(a @ x - b) / (np.linalg.norm(a, 2) * np.linalg.norm(x))
    assert res < 1e-6


# ---------------------------------------------------------------- bookkeeping

def test_offsets_hand_computed():
    r = np.zeros((4, 4), dtype=int)
    r[1, 0], r[2, 0], r[2, 1], r[3, 0], r[3, 1], r[3, 2] = 5, 2, 7, 1, 0, 4
    off, total = bk.lower_offsets(r)
    assert total == 19
    assert [off[1, 0], off[2, 0], off[2, 1], off[3, 0], off[3, 1], off[3, 2]] == [0, 5, 7, 14, 15, 15]
    po = bk.row_panel_offsets(r)
    assert [po[3, 0], po[3, 1], po[3, 2], po[2, 1]] == [0, 1, 1, 2]
    assert bk.row_widths(r, 2).tolist() == [0, 5, 9, 1]
    assert bk.tile_rows(300, 128).tolist() == [128, 128, 44]


def test_sort_ranks_ties_ascending_row():
    a = np.zeros((6, 6), dtype=int)
    a[2:, 1] = [4, 9, 4, 7]           # rows 2..5 of column 1
    assert bk.sort_ranks(a, 1) == [3, 5, 2, 4]


def test_active_set_evolution_hand_computed():
    order = [7, 3, 9, 1, 4, 8]
    sets = bk.active_sets(order, 4, [[False, True, True, False], [True, False, False, False],
                                     [True, True, False], [True]])
    assert sets == [[7, 3, 9, 1], [7, 1, 4, 8], [1, 4, 8], [8], []]
    # without a cap the subset only shrinks
    assert bk.active_sets([2, 5], 99, [[True, False], [True]]) == [[2, 5], [5], []]


# ---------------------------------------------------------------- pivoted TLR Cholesky

def test_pivoted_scalar_tiles_match_lapack_dpstrf():
    # with 1 x 1 tiles the Frobenius-norm tile pivot is the largest remaining
    # diagonal entry: the pivoted Cholesky of LAPACK's dpstrf
    from scipy.linalg import lapack
    rng = np.random.default_rng(17)
    n = 12
    g = rng.standard_normal((n, n))
    a = g @ g.T + np.diag(rng.uniform(0.5, 3.0, n))
    t = tlr.compress_dense(a, 1, 1e-14)
    l, perm = tlr.tlr_cholesky_pivoted(t, 1e-14)
    c, piv, rank, info = lapack.dpstrf(a, lower=1)
    assert info == 0 and rank == n
    assert perm == [int(p) - 1 for p in piv]
    np.testing.assert_allclose(l.dense_lower(), np.tril(c), rtol=0, atol=1e-12 * np.abs(c).max())


def _block(m, *rows):
    """Symmetric block matrix from scalar multiples of the m x m identity."""
    return np.block([[v * np.eye(m) for v in row] for row in rows])


def test_pivoted_order_hand_computed():
    m = 2
    # diagonal scales 1, 3, 2 with weak coupling: the order of the scales
    a = _block(m, (1.0, 0.01, 0.0), (0.01, 3.0, 0.01), (0.0, 0.01, 2.0))
    _, perm = tlr.tlr_cholesky_pivoted(tlr.compress_dense(a, m, 1e-14), 1e-14)
    assert perm == [1, 2, 0]
    # block 2 (scale 2.2) is coupled to block 1 (scale 3) by 2 I: once block 1
    # is eliminated, its update is 2.2 - 4 / 3 < 2, so block 0 comes next
    a = _block(m, (2.0, 0.0, 0.0), (0.0, 3.0, 2.0), (0.0, 2.0, 2.2))
    l, perm = tlr.tlr_cholesky_pivoted(tlr.compress_dense(a, m, 1e-14), 1e-14)
    assert perm == [1, 0, 2]
    np.testing.assert_allclose(np.diag(l.diag[2]), math.sqrt(2.2 - 4.0 / 3.0) * np.ones(m), rtol=1e-14)


def test_pivoted_backward_error_identity_and_pivot_rule():
    _, a = _cov(1024, 128, seed=23)
    tau = 1e-6
    t = tlr.compress_dense(a, 128, tau)
    l, perm = tlr.tlr_cholesky_pivoted(t, tau)
    assert sorted(perm) == list(range(t.nb))
    tp = tlr.permute(t, perm)
    e = tp.dense_symmetric() - l.dense_lower() @ l.dense_lower().T
    for k in range(t.nb):
        assert np.abs(e[t.blk(k), t.blk(k)]).max() < 1e-12 * np.abs(a).max()
        for i in range(k + 1, t.nb):
            # exact SVD truncation: the tile error is below tau
            assert np.linalg.norm(e[t.blk(i), t.blk(k)], 2) <= tau * (1 + 1e-8)
        # the pivot of step k has the largest updated diagonal norm
        norms = []
        for s in range(k, t.nb):
            d = tp.diag[s].copy()
            for j in range(k):
                d -= l.u[s, j] @ ((l.v[s, j].T @ l.v[s, j]) @ l.u[s, j].T)
            norms.append(np.linalg.norm(d, "fro"))
        assert norms[0] >= max(norms) * (1 - 1e-12)


def test_pivoted_exact_low_rank_kept():
    n, m, r = 512, 64, 3
    rng = np.random.default_rng(29)
    a = np.zeros((n, n))
    for k in range(0, n, m):
        g = rng.standard_normal((m, m))
        a[k:k + m, k:k + m] = g @ g.T / m + (1.0 + 0.5 * (k // m)) * np.eye(m)
    w = rng.standard_normal((n, r))
    a += w @ w.T
    t = tlr.compress_dense(a, m, 1e-9)
    l, perm = tlr.tlr_cholesky_pivoted(t, 1e-9)
    assert perm != list(range(t.nb))
    assert set(l.ranks()[np.tril_indices(t.nb, -1)].tolist()) == {r}
    tp = tlr.permute(t, perm)
    assert np.abs(tp.dense_symmetric() - l.dense_lower() @ l.dense_lower().T).max() < 1e-10 * np.abs(a).max()


# ---------------------------------------------------------------- modified Cholesky

def test_modified_cholesky_hand_computed():
    # [[1, 2], [2, 1]] is indefinite: the second pivot 1 - 2^2 = -3 becomes
    # max(|-3|, delta) = 3, so L L^T = A + diag(0, 6); with [[1, 1], [1, 1]]
    # the second pivot is 0 and becomes delta
    l, f = dense.cholesky_modified(np.array([[1.0, 2.0], [2.0, 1.0]]), 0.25)
    np.testing.assert_allclose(l, [[1.0, 0.0], [2.0, math.sqrt(3.0)]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(f, [0.0, 6.0], rtol=0, atol=1e-15)
    l, f = dense.cholesky_modified(np.array([[1.0, 1.0], [1.0, 1.0]]), 0.25)
    np.testing.assert_allclose(l, [[1.0, 0.0], [1.0, 0.5]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(f, [0.0, 0.25], rtol=0, atol=1e-15)


def test_modified_cholesky_is_lapack_on_definite_tiles():
    rng = np.random.default_rng(61)
    g = rng.standard_normal((40, 40))
    a = g @ g.T + 0.5 * np.eye(40)
    l, f = dense.cholesky_modified(a, 1e-3)
    assert not f.any()
    np.testing.assert_allclose(l, np.linalg.cholesky(a), rtol=0, atol=1e-12 * np.abs(a).max())


def test_modified_cholesky_perturbation_is_diagonal_and_nonnegative():
    rng = np.random.default_rng(62)
    q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    # one eigenvalue slightly below zero: the case the method is for (a tile
    # that lost definiteness by a small perturbation)
    a = q @ np.diag(np.linspace(-1e-3, 5.0, 30)) @ q.T
    delta = 1e-2
    l, f = dense.cholesky_modified(a, delta)
    e = l @ l.T - a
    assert f.min() >= 0.0 and f.max() > 0.0
    np.testing.assert_allclose(np.diag(e), f, rtol=0, atol=1e-10 * np.abs(a).max() * f.max())
    off = e - np.diag(np.diag(e))
    assert np.abs(off).max() <= 1e-12 * (np.abs(a).max() + f.max())
    # the factor stays bounded (the raised pivot is as large as the loss)
    assert np.abs(l).max() <= 10 * math.sqrt(np.abs(a).max())


def test_tlr_modified_cholesky_exact_low_rank():
    # blockdiag(B) + W W^T with an indefinite B_1: the unmodified TLR
    # Cholesky fails at tile 1; the modified one factors A + diag(f), f >= 0
    # on the raised pivots of that tile only
    n, m, r = 384, 64, 3
    rng = np.random.default_rng(63)
    a = np.zeros((n, n))
    for k in range(0, n, m):
        g = rng.standard_normal((m, m))
        a[k:k + m, k:k + m] = g @ g.T / m + np.eye(m)
    w = rng.standard_normal((n, r))
    a += w @ w.T
    # tile 1's Schur complement (A_11 - A_10 A_00^-1 A_01) loses definiteness
    # by a rank-one change of A_11 just past its smallest eigenvalue
    s1 = a[m:2 * m, m:2 * m] - a[m:2 * m, :m] @ np.linalg.solve(a[:m, :m], a[:m, m:2 * m])
    lam, vec = np.linalg.eigh(s1)
    a[m:2 * m, m:2 * m] -= (lam[0] + 1e-4) * np.outer(vec[:, 0], vec[:, 0])
    t = tlr.compress_dense(a, m, 1e-11)
    with pytest.raises(tlr.NotSPDTile):
        tlr.tlr_cholesky(t, 1e-9)
    rec = {}
    l = tlr.tlr_cholesky(t, 1e-9, record=rec, modified=True)
    assert rec["modified"] > 0
    e = l.dense_lower() @ l.dense_lower().T - t.dense_symmetric()
    d = np.diag(e).copy()
    np.fill_diagonal(e, 0.0)
    assert np.abs(e).max() <= 1e-8 * np.abs(a).max()
    assert d.min() >= -1e-9 and np.count_nonzero(d > 1e-9) == rec["modified"]
    assert np.all(np.abs(d[:m]) <= 1e-9) and np.all(np.abs(d[2 * m:]) <= 1e-9)


# ---------------------------------------------------------------- SVD post-recompression

def _tile_with_spectrum(m, s, seed):
    """U V^T with orthonormal U and singular values s (in a scrambled order),
    V = Y diag(s) for an orthonormal Y: the exact spectrum is s."""
    rng = np.random.default_rng(seed)
    q = len(s)
    x, _ = np.linalg.qr(rng.standard_normal((m, q)))
    y, _ = np.linalg.qr(rng.standard_normal((m, q)))
    order = rng.permutation(q)
    return x, y[:, order] * np.asarray(s)[order]


def test_recompress_keeps_exactly_the_values_above_tau():
    """Eckart-Young: the kept count is #{sigma > tau}, the error is the first
    dropped singular value, U stays orthonormal and the columns of V carry
    the kept singular values (a dropped scaling or swapped factor fails)."""
    m, tau = 64, 1e-3
    s = tau * np.array([40.0, 9.0, 3.0, 1.0 + 1e-8, 1.0 - 1e-8, 0.5, 0.1, 1e-3])
    a = tlr.TLR(3 * m, m)
    a.u[1, 0], a.v[1, 0] = _tile_with_spectrum(m, s, 3)
    a.u[2, 0], a.v[2, 0] = _tile_with_spectrum(m, s[:3] * 1e-3, 4)   # all below tau
    a.u[2, 1], a.v[2, 1] = np.zeros((m, 0)), np.zeros((m, 0))
    a.diag = [np.eye(m) * (k + 2.0) for k in range(3)]
    r = tlr.recompress(a, tau)
    assert r.ranks()[1, 0] == 4 and r.ranks()[2, 0] == 0 and r.ranks()[2, 1] == 0
    u, v = r.u[1, 0], r.v[1, 0]
    np.testing.assert_allclose(u.T @ u, np.eye(4), atol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(v, axis=0), s[:4], rtol=1e-12)
    err = np.linalg.norm(a.tile(1, 0) - u @ v.T, 2)
    assert abs(err - s[4]) <= 1e-12 * s[0]
    # the upper tile is the transpose: the stored factors keep the lower orientation
    np.testing.assert_allclose(r.tile(0, 1), (u @ v.T).T, atol=1e-15)
    for k in range(3):
        np.testing.assert_array_equal(r.diag[k], a.diag[k])
    assert r.memory_doubles() == 3 * m * m + 2 * m * 4


def test_recompress_is_idempotent_and_never_raises_an_svd_rank():
    """A tile already at its minimal rank keeps it; on a truncated-SVD
    compression (the minimal ranks) nothing changes but rounding."""
    _, a = _cov(512, 128)
    tau = 1e-6
    t = tlr.compress_dense(a, 128, tau)
    r = tlr.recompress(t, tau)
    np.testing.assert_array_equal(r.ranks(), t.ranks())
    for (i, j) in t.u:
        np.testing.assert_allclose(r.tile(i, j), t.tile(i, j), atol=1e-13)
    r2 = tlr.recompress(r, tau)
    np.testing.assert_array_equal(r2.ranks(), r.ranks())


def test_recompress_of_a_padded_rank_surplus():
    """Extra directions of a tile (rank surplus, as the ARA leaves) are
    removed: U = [X | X2], V = [Y S | 0-weighted] collapses to the rank of
    the spectrum above tau; the result matches the dense truncated SVD."""
    rng = np.random.default_rng(9)
    m, tau = 48, 1e-4
    s = np.array([3.0, 1.0, 1e-2, 5e-4, 5e-5, 1e-6])
    x, v = _tile_with_spectrum(m, s, 11)
    extra, _ = np.linalg.qr(np.hstack([x, rng.standard_normal((m, 5))]))
    u_big = extra                                   # 11 orthonormal columns
    v_big = np.hstack([v, 1e-7 * rng.standard_normal((m, 5))])
    a = tlr.TLR(2 * m, m)
    a.u[1, 0], a.v[1, 0] = u_big, v_big
    r = tlr.recompress(a, tau)
    dense_s = np.linalg.svd(u_big @ v_big.T, compute_uv=False)
    assert r.rank(1, 0) == int(np.sum(dense_s > tau)) == 4
    err = np.linalg.norm(a.tile(1, 0) - r.tile(1, 0), 2)
    assert abs(err - dense_s[4]) <= 1e-12 * dense_s[0]


# ---------------------------------------------------------------- Schur compensation

def test_schur_compensation_hand_computed():
    """D = [[2, 1], [1, 2]] has eigenvalues 3 and 1 (vectors (1, 1)/sqrt2 and
    (1, -1)/sqrt2).  At tau = 2 the compression keeps 3: D - Dbar =
    [[.5, -.5], [-.5, .5]], absolute row sums (1, 1).  At tau = 0.5 nothing
    is dropped; at tau = 3.5 everything is, and c is the row sums of |D|."""
    d = np.array([[2.0, 1.0], [1.0, 2.0]])
    np.testing.assert_allclose(dense.schur_compensation(d, 2.0), [1.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(dense.schur_compensation(d, 0.5), [0.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(dense.schur_compensation(d, 3.5), [3.0, 3.0], atol=1e-14)
    # a diagonal update: the dropped entries stay on the diagonal
    np.testing.assert_allclose(dense.schur_compensation(np.diag([5.0, 1e-3, 2e-3]), 1e-2),
                               [0.0, 1e-3, 2e-3], atol=1e-18)


def test_schur_compensation_dominates_the_dropped_part():
    """diag(c) - (D - Dbar) is diagonally dominant, so the compensated tile
    is at least A - Dbar in the Loewner order, and c <= sqrt(m) tau per row
    (the row of a PSD matrix of 2-norm <= tau)."""
    rng = np.random.default_rng(2)
    m, tau = 40, 1e-3
    x = rng.standard_normal((m, m))
    q, _ = np.linalg.qr(x)
    lam = np.concatenate([np.logspace(1, -1, 10), np.logspace(-3.5, -8, 30)])
    d = (q * lam) @ q.T
    c = dense.schur_compensation(d, tau)
    keep = lam > tau
    dbar = (q[:, keep] * lam[keep]) @ q[:, keep].T
    e = d - dbar
    assert np.all(c >= 0) and np.all(c <= np.sqrt(m) * tau)
    assert np.linalg.eigvalsh(np.diag(c) - e).min() >= -1e-14
    np.testing.assert_allclose(c, np.abs(e).sum(axis=1), atol=1e-15)


def test_tlr_cholesky_schur_compensation_is_the_paper_update():
    """The column step with compensation factors A_kk - D_k + diag(c): the
    factor's diagonal tiles satisfy L_kk L_kk^T = that tile, with D_k from
    the factor's own tiles; the first column has no update and matches the
    plain factor; every c is within the sqrt(m) tau row bound."""
    _, a = _cov(512, 128)
    t = tlr.compress_dense(a, 128, 1e-6)
    rec = {}
    l = tlr.tlr_cholesky(t, 1e-4, schur_comp=True, record=rec)
    for k in range(1, t.nb):
        upd = sum(l.u[k, j] @ l.v[k, j].T @ l.v[k, j] @ l.u[k, j].T for j in range(k))
        want = t.diag[k] - upd + np.diag(dense.schur_compensation(upd, 1e-4))
        np.testing.assert_allclose(l.diag[k] @ l.diag[k].T, want, atol=1e-12)
        assert 0 < rec["comp"][k].max() <= np.sqrt(128) * 1e-4
    plain = tlr.tlr_cholesky(t, 1e-4)
    np.testing.assert_array_equal(l.diag[0], plain.diag[0])
