"""SVD post-recompression of the low rank tiles (Section 6.2) on the GPU
against the oracle's definition: every tile of the GPU's own factor (or
input), downloaded before the call, is truncated by a dense SVD on the host
(oracle.tlr.recompress) and compared with what the library left.

What is unique about a truncated SVD is compared directly: the kept rank
(except where a singular value lies within a hair of tau, where either
choice is right), the kept singular values, the error sigma_{r+1}, the
orthonormality of U and the product U V^T.  The bookkeeping (offsets of the
compacted panels) is compared bit for bit with the oracle's, and the solve
with the recompressed factor against the oracle's solve with the same
factor."""
import numpy as np
import pytest

from oracle import bookkeeping as bk
from oracle import dense
from oracle import tlr as otlr
from paper_2108_11932_amd import tlr
from paper_2108_11932_amd import workloads as wl

from gpu_util import oracle_tlr

pytestmark = pytest.mark.gpu

# A singular value within this relative distance of tau may fall on either
# side (the two-pass Gram solver resolves singular values to a relative
# error near m u; the band leaves three orders of magnitude of margin).
BAND = 1e-9


def _check_tiles(before, after, tau, ranks_or):
    """Per tile: rank, spectrum, error and orthonormality against the dense
    truncated SVD of the tile before the call."""
    n_band = 0
    for (i, j), u0 in before.u.items():
        t = u0 @ before.v[i, j].T
        s = np.linalg.svd(t, compute_uv=False)
        u1, v1 = after.u[i, j], after.v[i, j]
        r = u1.shape[1]
        r_or = int(ranks_or[i, j])
        near = np.abs(s / tau - 1.0) <= BAND if tau > 0 else np.zeros_like(s, bool)
        if r != r_or:
            # only values inside the band may change sides
            lo, hi = sorted((r, r_or))
            assert np.all(near[lo:hi]), (i, j, r, r_or, s[lo:hi] / tau)
            n_band += 1
        assert np.all(s[:r] > tau * (1 - BAND)), (i, j)
        if r < len(s):
            assert s[r] <= tau * (1 + BAND), (i, j, s[r] / tau)
        if r == 0:
            continue
        np.testing.assert_allclose(u1.T @ u1, np.eye(r), atol=1e-12, err_msg=str((i, j)))
        sv = np.linalg.norm(v1, axis=0)
        np.testing.assert_allclose(sv, s[:r], rtol=1e-9, atol=1e-13 * s[0], err_msg=str((i, j)))
        err = np.linalg.norm(t - u1 @ v1.T, 2)
        tail = s[r] if r < len(s) else 0.0
        assert abs(err - tail) <= 1e-11 * s[0] + 1e-9 * tail, (i, j, err, tail)
    return n_band


def _cov_factor(n, m, eps, ldl=False, pivoted=False, seed=21):
    pts = wl.jittered_grid(n, 2, seed)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-4, m, eps)
    o = tlr.opts(bs=16)
    if ldl:
        st = mat.ldlt(eps, o)[0]
    elif pivoted:
        st = mat.potrf_pivoted(eps, o)[0]
    else:
        st = mat.potrf(eps, o)
    return pts, mat, st


@pytest.mark.parametrize("kind", ["chol", "ldlt", "pivoted"])
def test_factor_recompression_matches_truncated_svd(kind):
    n, m, eps = 4096, 256, 1e-6
    _, mat, st = _cov_factor(n, m, eps, ldl=kind == "ldlt", pivoted=kind == "pivoted")
    tau = st["tau"]
    before = oracle_tlr(mat, tlr.FACTOR)
    r0 = mat.ranks(tlr.FACTOR)
    ref = otlr.recompress(before, tau)
    mat.recompress(tau)
    after = oracle_tlr(mat, tlr.FACTOR)
    r1 = mat.ranks(tlr.FACTOR)
    n_band = _check_tiles(before, after, tau, ref.ranks())
    assert n_band <= 1
    assert np.all(r1 <= r0) and r1.sum() < r0.sum()
    # the compacted panels: offsets as the oracle's bookkeeping lays them out
    np.testing.assert_array_equal(mat.offsets(tlr.FACTOR), bk.row_panel_offsets(r1))
    # diagonal tiles untouched
    for k in range(before.nb):
        np.testing.assert_array_equal(after.diag[k], before.diag[k])
    # the solve with the recompressed factor is the oracle's solve with it
    import torch
    b = np.random.default_rng(3).standard_normal((n, 2))
    x = mat.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    d = None
    if kind == "ldlt":
        piv = mat.pivots()
        d = [piv[k * m:(k + 1) * m] for k in range(before.nb)]
    if kind == "pivoted":
        # P A P^T = L L^T, position t holding original block perm[t] (n = nb m)
        idx = np.concatenate([np.arange(p * m, (p + 1) * m) for p in mat.perm()])
        want = np.zeros_like(b)
        want[idx] = otlr.solve(after, b[idx], d)
    else:
        want = otlr.solve(after, b, d)
    np.testing.assert_allclose(x, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())
    # a second pass at the same threshold keeps every rank
    mat.recompress(tau)
    np.testing.assert_array_equal(mat.ranks(tlr.FACTOR), r1)
    mat.close()


def test_input_recompression_and_matvec():
    n, m, eps = 4096, 256, 1e-6
    pts = wl.jittered_grid(n, 2, 5)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-4, m, eps)
    before = oracle_tlr(mat, tlr.INPUT)
    r0 = mat.ranks(tlr.INPUT)
    ref = otlr.recompress(before, eps)
    mat.recompress(eps, tlr.INPUT)
    after = oracle_tlr(mat, tlr.INPUT)
    r1 = mat.ranks(tlr.INPUT)
    assert _check_tiles(before, after, eps, ref.ranks()) <= 1
    assert r1.sum() < r0.sum()
    np.testing.assert_array_equal(mat.offsets(tlr.INPUT), bk.lower_offsets(r1)[0])
    import torch
    x = np.random.default_rng(4).standard_normal(n)
    y = mat.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    want = otlr.matvec(after, x)
    np.testing.assert_allclose(y, want, rtol=1e-11, atol=1e-11 * np.abs(want).max())
    # the recompressed input still factors, with the factor's usual bound
    st = mat.potrf(eps, tlr.opts(bs=16))
    l = oracle_tlr(mat, tlr.FACTOR)
    a = oracle_tlr(mat, tlr.INPUT)
    err = otlr.factor_error_norm(a, l)
    assert err <= 2.0 * np.sqrt(a.nb) * st["tau"]
    mat.close()


def _spectrum_tile(rng, m, q, decades):
    x, _ = np.linalg.qr(rng.standard_normal((m, q)))
    y, _ = np.linalg.qr(rng.standard_normal((m, q)))
    s = np.logspace(0, -decades, q)
    return (x * s) @ y.T


@pytest.mark.parametrize("m,qs", [
    # ranks <= 32 and <= 96 (G and W in LDS), 100 and 128 = m (G packed in
    # LDS; a full-rank tile)
    (128, {(1, 0): 20, (2, 0): 50, (2, 1): 100, (3, 0): 128, (3, 1): 7, (3, 2): 96}),
    # ranks above 180 (the global-memory solver; a full-rank tile) and 150
    (256, {(1, 0): 200, (2, 0): 150, (2, 1): 256}),
])
def test_all_solver_classes_and_full_rank_tiles(m, qs):
    """Tiles of every solver class with spectra spread over ten decades, cut
    at a threshold inside each spectrum."""
    nb = max(i for i, _ in qs) + 1
    n = m * nb
    rng = np.random.default_rng(17)
    a = np.eye(n) * 4.0
    for (i, j), q in qs.items():
        t = _spectrum_tile(rng, m, q, 10)
        a[i * m:(i + 1) * m, j * m:(j + 1) * m] = t
        a[j * m:(j + 1) * m, i * m:(i + 1) * m] = t.T
    import torch
    mat = tlr.TLRMatrix.compress(torch.from_numpy(a).cuda(), m, 1e-13)
    r0 = mat.ranks(tlr.INPUT)
    for (i, j), q in qs.items():
        assert r0[i, j] >= min(q, m) - 2, (i, j, r0[i, j], q)
    before = oracle_tlr(mat, tlr.INPUT)
    tau = 3.3e-6
    ref = otlr.recompress(before, tau)
    mat.recompress(tau, tlr.INPUT)
    after = oracle_tlr(mat, tlr.INPUT)
    assert _check_tiles(before, after, tau, ref.ranks()) == 0
    r1 = mat.ranks(tlr.INPUT)
    for (i, j), q in qs.items():
        s = np.logspace(0, -10, q)
        assert r1[i, j] == int(np.sum(s > tau)), (i, j, r1[i, j])
    # tau = 0 keeps every direction of the exact spectra (the smallest is 1e-10)
    mat2 = tlr.TLRMatrix.compress(torch.from_numpy(a).cuda(), m, 1e-13)
    mat2.recompress(0.0, tlr.INPUT)
    r2 = mat2.ranks(tlr.INPUT)
    for (i, j), q in qs.items():
        assert min(q, m) <= r2[i, j] <= r0[i, j], (i, j, r2[i, j], r0[i, j])
    mat.close()
    mat2.close()


def test_recompress_errors():
    n, m = 512, 128
    pts, mat, st = _cov_factor(n, m, 1e-6)
    with pytest.raises(tlr.TLRError) as e:
        mat.recompress(-1.0)
    assert e.value.status == -1
    with pytest.raises(tlr.TLRError) as e:
        mat.recompress(float("nan"))
    assert e.value.status == -1
    r = mat.ranks(tlr.FACTOR)
    mat.close()
    # input whose tiles were set from the host: U of unknown orthonormality
    t = otlr.compress_dense(dense.covariance_matrix(pts, dense.KERNEL_EXP, 0.1, 1e-4), m, 1e-6)
    h = tlr.TLRMatrix.from_tlr(n, m, t.diag, t.u, t.v)
    with pytest.raises(tlr.TLRError) as e:
        h.recompress(1e-6, tlr.INPUT)
    assert e.value.status == -4
    # no factor yet
    with pytest.raises(tlr.TLRError) as e:
        h.recompress(1e-6, tlr.FACTOR)
    assert e.value.status == -4
    h.close()
    assert r.sum() > 0


def test_headline_factor_sampled_tiles():
    """The benchmark's configuration: the N = 131072 2D covariance at tile
    1024, eps 1e-6 absolute, ARA block 16, the whole factor recompressed in
    one call (every solver class, one chunk); sampled tiles (the highest
    ranks, which take the packed-LDS solver, and a spread of others) against
    the dense truncated SVD of the same tiles before the call, the offsets
    of every row, and the random-vector residual of the result."""
    w = wl.standard("cov2d_131k")
    mat = tlr.TLRMatrix.compress_kernel(w.points, w.kernel, w.ell, w.diag_add, w.m, w.eps,
                                        tlr.opts(bs=w.bs))
    st = mat.potrf(w.eps, tlr.opts(bs=w.bs, eps_mode=w.eps_mode))
    tau = st["tau"]
    r0 = mat.ranks(tlr.FACTOR)
    low = np.tril_indices(mat.nb, -1)
    order = np.argsort(-r0[low], kind="stable")
    pick = list(order[:6]) + list(order[len(order) // 8::len(order) // 6][:6])
    tiles = [(int(low[0][p]), int(low[1][p])) for p in pick]
    assert max(r0[t] for t in tiles) > 96
    before = otlr.TLR(mat.n, mat.m)
    for t in tiles:
        before.u[t], before.v[t] = mat.tile(tlr.FACTOR, *t)
    mat.recompress(tau)
    after = otlr.TLR(mat.n, mat.m)
    for t in tiles:
        after.u[t], after.v[t] = mat.tile(tlr.FACTOR, *t)
    ref = otlr.recompress(before, tau)
    assert _check_tiles(before, after, tau, ref.ranks()) <= 1
    r1 = mat.ranks(tlr.FACTOR)
    assert r1.sum() < 0.9 * r0.sum()
    np.testing.assert_array_equal(mat.offsets(tlr.FACTOR), bk.row_panel_offsets(r1))
    import torch
    g = torch.Generator(device="cpu").manual_seed(7)
    b = torch.randn(mat.n, 4, generator=g, dtype=torch.float64).cuda()
    x = mat.solve(b)
    res = float(((mat.matvec(x) - b).norm(dim=0) / x.norm(dim=0)).max())
    assert res <= 2.0 * np.sqrt(mat.nb) * tau
    mat.close()


def test_recompress_mixed_precision_factor_then_refactor():
    """A factor made with the FP32 panel copies: the recompression releases
    the copies (they serve the sampling only), the solve uses the new
    panels, and the next mixed-precision factorization builds them again
    and gives the factor of a fresh handle."""
    n, m = 4096, 256
    pts = wl.jittered_grid(n, 2, 13)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-4, m, 1e-8)
    o = tlr.opts(bs=16, eps_mode=tlr.EPS_REL, precision=tlr.MIXED_FP32)
    st = mat.potrf(1e-6, o)
    r0 = mat.ranks(tlr.FACTOR)
    mat.recompress(st["tau"])
    assert mat.ranks(tlr.FACTOR).sum() <= r0.sum()
    import torch
    b = torch.randn(n, 2, dtype=torch.float64, generator=torch.Generator().manual_seed(1)).cuda()
    x = mat.solve(b)
    res = float(((mat.matvec(x) - b).norm(dim=0) / x.norm(dim=0)).max())
    assert res <= 2.0 * np.sqrt(mat.nb) * st["tau"]
    st2 = mat.potrf(1e-6, o)
    l2 = oracle_tlr(mat, tlr.FACTOR)
    fresh = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-4, m, 1e-8)
    fresh.potrf(1e-6, o)
    lf = oracle_tlr(fresh, tlr.FACTOR)
    np.testing.assert_array_equal(l2.ranks(), lf.ranks())
    for key in lf.u:
        np.testing.assert_array_equal(l2.v[key], lf.v[key])
    assert st2["fp32_tile_iters"] > 0
    fresh.close()
    mat.close()


def test_recompress_degenerate_shapes():
    """One block (no low rank tile), N below the tile size, and an input
    whose off-diagonal tiles are all of rank 0 (a block-diagonal matrix):
    nothing to cut, the call succeeds and the handle stays usable."""
    import torch
    # N < m: a single padded block
    pts = wl.uniform_points(100, 2, 3)
    mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-4, 128, 1e-8)
    st = mat.potrf(1e-8, tlr.opts(bs=16))
    mat.recompress(st["tau"])
    mat.recompress(1e-8, tlr.INPUT)
    b = np.random.default_rng(0).standard_normal(100)
    x = mat.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    d = dense.covariance_matrix(pts, dense.KERNEL_EXP, 0.1, 1e-4)
    np.testing.assert_allclose(d @ x, b, atol=1e-8 * np.abs(b).max())
    mat.close()
    # block diagonal: every off-diagonal tile of rank 0
    m, nb = 64, 3
    a = np.zeros((m * nb, m * nb))
    rng = np.random.default_rng(1)
    for k in range(nb):
        g = rng.standard_normal((m, m))
        a[k * m:(k + 1) * m, k * m:(k + 1) * m] = g @ g.T + m * np.eye(m)
    mat = tlr.TLRMatrix.compress(torch.from_numpy(a).cuda(), m, 1e-10)
    assert mat.ranks(tlr.INPUT).sum() == 0
    mat.recompress(1e-10, tlr.INPUT)
    mat.potrf(1e-10, tlr.opts(bs=16))
    mat.recompress(1e-10)
    assert mat.ranks(tlr.FACTOR).sum() == 0
    b = rng.standard_normal(m * nb)
    x = mat.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    np.testing.assert_allclose(a @ x, b, atol=1e-9 * np.abs(b).max())
    mat.close()
