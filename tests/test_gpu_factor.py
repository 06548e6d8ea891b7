"""End-to-end parity of the GPU TLR factorizations, solve and product with the
FP64 oracle, through the C ABI.

The ARA compression is randomized, so the factor is not unique: the tests
compare what is unique (L L^T against A, the first diagonal tile, solves and
products given a factor) and check the rest against the invariants the
method fixes: per-tile backward error equal to the compression error
(left-looking identity), the global error bound, Eckart-Young lower bounds
and exact ranks on exactly low rank inputs.
"""
import math

import numpy as np
import pytest

from oracle import dense
from oracle import tlr as otlr
from paper_2108_11932_amd import tlr
from paper_2108_11932_amd import workloads as wl

from gpu_util import RANK_RATIO, dev, host, oracle_tlr

pytestmark = pytest.mark.gpu


def _cov(n, seed, ell=0.1, nugget=1e-4, dim=2, kernel=dense.KERNEL_EXP):
    if n & (n - 1) == 0:
        pts = wl.jittered_grid(n, dim, seed)
    else:
        pts = wl.uniform_points(n, dim, seed)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    return pts, dense.covariance_matrix(pts, kernel, ell, nugget)


def _upload(t):
    return tlr.TLRMatrix.from_tlr(t.n, t.m, t.diag, t.u, t.v)


def _residual_tiles(a_tlr, l_tlr, d=None):
    ad = a_tlr.dense_symmetric()
    ld = l_tlr.dense_lower()
    rec = ld @ (np.diag(np.concatenate(d)) if d is not None else np.eye(ld.shape[0])) @ ld.T
    return ad - rec


def test_single_tile_is_dense_cholesky():
    _, a = _cov(200, 1)
    t = otlr.compress_dense(a, 200, 1e-6)
    mat = _upload(t)
    mat.potrf(1e-6)
    L = mat.diag(tlr.FACTOR, 0)
    ref = np.linalg.cholesky(a)
    np.testing.assert_allclose(L, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,m,r", [(768, 128, 3), (1000, 128, 5)])
def test_exactly_low_rank_recovered(n, m, r):
    rng = np.random.default_rng(n + r)
    a = np.zeros((n, n))
    for k in range(0, n, m):
        e = min(n, k + m)
        g = rng.standard_normal((e - k, e - k))
        a[k:e, k:e] = g @ g.T / (e - k) + np.eye(e - k)
    w = rng.standard_normal((n, r))
    a += w @ w.T
    tau = 1e-8
    t = otlr.compress_dense(a, m, tau)
    mat = _upload(t)
    st = mat.potrf(tau)
    ranks = mat.ranks(tlr.FACTOR)
    lower = ranks[np.tril_indices(t.nb, -1)]
    assert set(lower.tolist()) == {r}
    l = oracle_tlr(mat, tlr.FACTOR)
    res = _residual_tiles(t, l)
    assert np.abs(res).max() < 1e-10 * np.abs(a).max()
    assert st["max_rank"] == r


@pytest.mark.parametrize("n,m,eps", [(2048, 256, 1e-6), (1000, 128, 1e-6), (2048, 256, 1e-3)])
def test_cholesky_matches_oracle_invariants(n, m, eps):
    pts, a = _cov(n, 3)
    t = otlr.compress_dense(a, m, eps)
    mat = _upload(t)
    st = mat.potrf(eps)
    assert st["info"] == 0 and abs(st["tau"] - eps) == 0
    l = oracle_tlr(mat, tlr.FACTOR)
    ref = otlr.tlr_cholesky(t, eps)
    # the first diagonal tile sees no update: LAPACK's factor
    np.testing.assert_allclose(l.diag[0], ref.diag[0], rtol=0, atol=1e-12 * np.abs(ref.diag[0]).max())
    # left-looking identity: every residual tile is a compression error
    res = _residual_tiles(t, l)
    scale = np.linalg.norm(a, 2)
    for k in range(t.nb):
        assert np.linalg.norm(res[t.blk(k), t.blk(k)], 2) < 1e-11 * scale
        for i in range(k + 1, t.nb):
            e = np.linalg.norm(res[t.blk(i), t.blk(k)], 2)
            assert e <= 4 * eps, (i, k, e)
    err = np.linalg.norm(res, 2)
    assert err <= 2 * math.sqrt(t.nb) * eps
    # ranks: never below the optimal rank at the achieved tile error, and
    # within 10% (plus one block) of the oracle's optimal ranks in total
    rg = mat.ranks(tlr.FACTOR)
    ro = ref.ranks()
    assert rg.sum() <= RANK_RATIO * ro.sum() + t.nb
    for k in range(t.nb):
        for i in range(k + 1, t.nb):
            s_ik = otlr.schur_tile(t, l, i, k)
            sv = np.linalg.svd(s_ik, compute_uv=False)
            e = np.linalg.norm(res[t.blk(i), t.blk(k)], 2)
            assert rg[i, k] >= int(np.sum(sv > e * (1 + 1e-8) + 1e-14 * scale))


@pytest.mark.parametrize("bs,bs_tail,tail_active", [(16, 32, 0), (8, 24, 0), (16, 32, 2)])
def test_larger_tail_block_keeps_accuracy(bs, bs_tail, tail_active):
    # later ARA iterations of a column drawing more samples (all of them, or
    # only those with at most tail_active tiles left): same bounds
    pts, a = _cov(2048, 19)
    eps = 1e-6
    t = otlr.compress_dense(a, 256, eps)
    mat = _upload(t)
    st = mat.potrf(eps, tlr.opts(bs=bs, bs_tail=bs_tail, tail_active=tail_active))
    l = oracle_tlr(mat, tlr.FACTOR)
    res = _residual_tiles(t, l)
    for k in range(t.nb):
        for i in range(k + 1, t.nb):
            assert np.linalg.norm(res[t.blk(i), t.blk(k)], 2) <= 4 * eps
    assert np.linalg.norm(res, 2) <= 2 * math.sqrt(t.nb) * eps
    ref = otlr.tlr_cholesky(t, eps)
    assert mat.ranks(tlr.FACTOR).sum() <= RANK_RATIO * ref.ranks().sum() + t.nb


def test_dynamic_batching_subset_gives_same_quality():
    pts, a = _cov(2048, 5)
    eps = 1e-6
    t = otlr.compress_dense(a, 256, eps)
    mat = _upload(t)
    st = mat.potrf(eps, tlr.opts(max_active=2))
    l = oracle_tlr(mat, tlr.FACTOR)
    err = np.linalg.norm(_residual_tiles(t, l), 2)
    assert err <= 2 * math.sqrt(t.nb) * eps
    assert st["ara_iters"] >= t.nb - 1


def test_solve_matches_oracle_on_gpu_factor():
    pts, a = _cov(1000, 7)
    eps = 1e-7
    t = otlr.compress_dense(a, 128, eps)
    mat = _upload(t)
    mat.potrf(eps)
    l = oracle_tlr(mat, tlr.FACTOR)
    b = np.random.default_rng(4).standard_normal((1000, 3))
    ref = otlr.solve(l, b)
    import torch
    got = mat.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
    res = np.linalg.norm(a @ got - b) / (np.linalg.norm(a, 2) * np.linalg.norm(got))
    assert res < 1e-6


def test_matvec_matches_oracle():
    pts, a = _cov(1000, 8)
    t = otlr.compress_dense(a, 128, 1e-8)
    mat = _upload(t)
    x = np.random.default_rng(2).standard_normal((1000, 2))
    import torch
    got = mat.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = otlr.matvec(t, x)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_ldlt_indefinite_inertia_and_residual():
    n, m, r = 768, 128, 4
    rng = np.random.default_rng(9)
    a = np.zeros((n, n))
    for k in range(0, n, m):
        sgn = np.where(rng.random(m) < 0.3, -1.0, 1.0)
        b = np.diag(sgn * rng.uniform(5, 6, m)) + 0.05 * rng.standard_normal((m, m))
        a[k:k + m, k:k + m] = 0.5 * (b + b.T)
    w = rng.standard_normal((n, r))
    a += w @ w.T
    tau = 1e-9
    t = otlr.compress_dense(a, m, tau)
    mat = _upload(t)
    st, d = mat.ldlt(tau)
    dd = d.cpu().numpy()
    assert int(np.sum(dd < 0)) == int(np.sum(np.linalg.eigvalsh(a) < 0))
    l = oracle_tlr(mat, tlr.FACTOR)
    piv = mat.pivots()
    res = _residual_tiles(t, l, [piv[k * m:(k + 1) * m] for k in range(t.nb)])
    assert np.abs(res).max() < 1e-9 * np.abs(a).max()
    # and the solve with L D L^T
    import torch
    bvec = rng.standard_normal(n)
    x = mat.solve(torch.from_numpy(bvec).cuda()).cpu().numpy()
    assert np.linalg.norm(a @ x - bvec) / np.linalg.norm(bvec) < 1e-7


def test_ldlt_matches_cholesky_on_spd():
    pts, a = _cov(1024, 11)
    eps = 1e-6
    t = otlr.compress_dense(a, 128, eps)
    mat = _upload(t)
    st, d = mat.ldlt(eps)
    assert np.all(d.cpu().numpy() > 0)
    l = oracle_tlr(mat, tlr.FACTOR)
    piv = mat.pivots()
    res = _residual_tiles(t, l, [piv[k * 128:(k + 1) * 128] for k in range(t.nb)])
    assert np.linalg.norm(res, 2) <= 2 * math.sqrt(t.nb) * eps


def test_not_spd_reports_row():
    pts, a = _cov(512, 2)
    a[300, 300] = -4.0
    t = otlr.compress_dense(a, 128, 1e-8)
    mat = _upload(t)
    status, st = mat.potrf_status(1e-8)
    assert status == tlr.TLR_ERR_NOT_SPD
    assert (st["info"] - 1) // 128 == 2


def test_compress_kernel_matches_oracle_tiles():
    n, m, eps = 1500, 256, 1e-6
    pts = wl.uniform_points(n, 2, 12)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-4, m, eps)
    ref = otlr.compress_kernel(pts, m, dense.KERNEL_EXP, 0.1, 1e-4, eps)
    got = oracle_tlr(mat, tlr.INPUT)
    for k in range(ref.nb):
        np.testing.assert_allclose(got.diag[k], ref.diag[k], rtol=0, atol=1e-14)
    rg, ro = mat.ranks(tlr.INPUT), ref.ranks()
    for i in range(ref.nb):
        for j in range(i):
            exact = otlr.kernel_tile(pts, m, i, j, dense.KERNEL_EXP, 0.1, 1e-4)
            e = np.linalg.norm(exact - got.u[i, j] @ got.v[i, j].T, 2)
            assert e <= 4 * eps
            assert rg[i, j] >= ro[i, j] - 2 and rg[i, j] <= ro[i, j] + 16
            assert not got.u[i, j][mat.n - i * m:].any() if (i + 1) * m > n else True


def test_relative_threshold_uses_norm_estimate():
    pts, a = _cov(1024, 13)
    t = otlr.compress_dense(a, 128, 1e-9)
    mat = _upload(t)
    st = mat.potrf(1e-6, tlr.opts(eps_mode=tlr.EPS_REL))
    norm = np.linalg.norm(t.dense_symmetric()[:1024, :1024], 2)
    # 20 power iterations: a lower bound of ||A||_2 within a fraction of a percent
    assert 0.995 * norm <= st["norm_a"] <= norm * (1 + 1e-12)
    assert abs(st["tau"] - 1e-6 * st["norm_a"]) < 1e-12 * norm
    l = oracle_tlr(mat, tlr.FACTOR)
    err = np.linalg.norm(_residual_tiles(t, l), 2)
    assert err <= 2 * math.sqrt(t.nb) * st["tau"]


def test_mixed_fp32_sampling_equal_accuracy():
    # FP32 panels in the sampling (TLR_MIXED_FP32): at a relative threshold
    # most tile iterations pass the rounding guard (it grows with sqrt(R_i),
    # the FP32 accumulation over the row panel, so the longest panels of the
    # last block rows keep FP64); the factor must reach the same accuracy
    # bound as the FP64 form, and about the same error
    n, m, eps = 2048, 128, 1e-5
    pts = wl.jittered_grid(n, 2, 21)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    errs, stats = {}, {}
    for prec in (tlr.FP64, tlr.MIXED_FP32):
        mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-4, m, eps)
        a_t = oracle_tlr(mat, tlr.INPUT)
        st = mat.potrf(eps, tlr.opts(eps_mode=tlr.EPS_REL, precision=prec))
        l = oracle_tlr(mat, tlr.FACTOR)
        errs[prec] = np.linalg.norm(_residual_tiles(a_t, l), 2)
        stats[prec] = st
    tau = stats[tlr.MIXED_FP32]["tau"]
    assert stats[tlr.FP64]["fp32_tile_iters"] == 0
    assert stats[tlr.MIXED_FP32]["fp32_tile_iters"] >= 0.8 * stats[tlr.MIXED_FP32]["tile_iters"]
    nb = n // m
    assert errs[tlr.MIXED_FP32] <= 2 * math.sqrt(nb) * tau
    assert errs[tlr.MIXED_FP32] <= 2 * errs[tlr.FP64] + tau


def test_mixed_guard_keeps_fp64_below_fp32_rounding():
    # at a threshold far below FP32 rounding no tile may use the FP32 panels,
    # and the mixed form then runs the FP64 kernels: identical factor
    pts, a = _cov(1024, 17)
    eps = 1e-10
    t = otlr.compress_dense(a, 128, eps)
    out = []
    for prec in (tlr.FP64, tlr.MIXED_FP32):
        mat = _upload(t)
        st = mat.potrf(eps, tlr.opts(precision=prec))
        out.append((st, mat.ranks(tlr.FACTOR), oracle_tlr(mat, tlr.FACTOR)))
    assert out[1][0]["fp32_tile_iters"] == 0
    np.testing.assert_array_equal(out[0][1], out[1][1])
    for k in range(t.nb):
        np.testing.assert_array_equal(out[0][2].diag[k], out[1][2].diag[k])
        for i in range(k + 1, t.nb):
            np.testing.assert_array_equal(out[0][2].u[i, k], out[1][2].u[i, k])
            np.testing.assert_array_equal(out[0][2].v[i, k], out[1][2].v[i, k])


def test_mixed_bf16_loose_threshold_with_shift():
    # relative 1e-2 with the shift s = tau (the loose threshold loses
    # definiteness without it): the tiles that pass the BF16 guard sample
    # their panel term on the BF16 matrix cores (FP32 accumulation); the
    # factor keeps the accuracy of the FP64 form against the unshifted matrix
    w = wl.standard("cov2d_4k")
    mat = tlr.TLRMatrix.compress_kernel(w.points, tlr.KERNEL_EXP, w.ell, w.diag_add, w.m, 1e-9)
    a_t = oracle_tlr(mat, tlr.INPUT)
    eps = 1e-2
    res = {}
    for prec in (tlr.FP64, tlr.MIXED_FP32, tlr.MIXED_BF16, tlr.MIXED_AUTO):
        st = mat.potrf(eps, tlr.opts(eps_mode=tlr.EPS_REL, precision=prec, shift=-1.0))
        res[prec] = (st, otlr.factor_error_norm(a_t, oracle_tlr(mat, tlr.FACTOR)))
    tau = res[tlr.FP64][0]["tau"]
    s16 = res[tlr.MIXED_BF16][0]
    assert res[tlr.FP64][0]["bf16_tile_iters"] == 0 and res[tlr.FP64][0]["fp32_tile_iters"] == 0
    assert res[tlr.MIXED_FP32][0]["bf16_tile_iters"] == 0
    assert s16["bf16_tile_iters"] > 0
    # the automatic form keeps BF16 copies at this threshold: the same run
    sa = res[tlr.MIXED_AUTO][0]
    assert (sa["bf16_tile_iters"], sa["fp32_tile_iters"], sa["ara_iters"]) == \
        (s16["bf16_tile_iters"], s16["fp32_tile_iters"], s16["ara_iters"])
    nb = a_t.nb
    for prec in (tlr.MIXED_FP32, tlr.MIXED_BF16):
        err = res[prec][1]
        assert err <= 2 * math.sqrt(nb) * tau + tau, (prec, err, tau)
        assert err <= 2 * res[tlr.FP64][1] + tau, (prec, err, res[tlr.FP64][1])


def test_mixed_auto_uses_fp32_at_tight_threshold():
    # relative 1e-6: the automatic form keeps no BF16 copies
    pts, a = _cov(2048, 23)
    t = otlr.compress_dense(a, 128, 1e-9)
    mat = _upload(t)
    st = mat.potrf(1e-6, tlr.opts(eps_mode=tlr.EPS_REL, precision=tlr.MIXED_AUTO))
    assert st["bf16_tile_iters"] == 0 and st["fp32_tile_iters"] > 0
    l = oracle_tlr(mat, tlr.FACTOR)
    assert np.linalg.norm(_residual_tiles(t, l), 2) <= 2 * math.sqrt(t.nb) * st["tau"]


def _lost_definiteness(n=384, m=64, r=3, seed=63):
    """blockdiag(B) + W W^T whose tile-1 Schur complement is just indefinite
    (a rank-one change of A_11 past its smallest eigenvalue)."""
    rng = np.random.default_rng(seed)
    a = np.zeros((n, n))
    for k in range(0, n, m):
        g = rng.standard_normal((m, m))
        a[k:k + m, k:k + m] = g @ g.T / m + np.eye(m)
    w = rng.standard_normal((n, r))
    a += w @ w.T
    s1 = a[m:2 * m, m:2 * m] - a[m:2 * m, :m] @ np.linalg.solve(a[:m, :m], a[:m, m:2 * m])
    lam, vec = np.linalg.eigh(s1)
    a[m:2 * m, m:2 * m] -= (lam[0] + 1e-4) * np.outer(vec[:, 0], vec[:, 0])
    return a


def test_modified_cholesky_matches_oracle():
    # Section 5.1.2: without the flag the factorization stops at tile 1; with
    # it the non-positive pivots of that tile are raised (max(|d|, tau)) and
    # the factor equals the oracle's modified factorization
    n, m, eps = 384, 64, 1e-9
    a = _lost_definiteness(n, m)
    t = otlr.compress_dense(a, m, 1e-11)
    mat = _upload(t)
    with pytest.raises(tlr.TLRError):
        mat.potrf(eps)
    st = mat.potrf(eps, tlr.opts(flags=tlr.FLAG_MODIFIED_CHOL))
    assert st["info"] == 0 and st["modified_pivots"] > 0
    rec = {}
    ref = otlr.tlr_cholesky(t, eps, record=rec, modified=True)
    assert st["modified_pivots"] == rec["modified"]
    l = oracle_tlr(mat, tlr.FACTOR)
    np.testing.assert_array_equal(l.ranks(), ref.ranks())
    for k in range(t.nb):
        np.testing.assert_allclose(l.diag[k], ref.diag[k], rtol=0, atol=1e-8 * np.abs(ref.diag[k]).max())
    e = l.dense_lower() @ l.dense_lower().T - t.dense_symmetric()
    d = np.diag(e).copy()
    np.fill_diagonal(e, 0.0)
    assert np.abs(e).max() <= 1e-7 * np.abs(a).max()
    assert d.min() >= -1e-8 and np.count_nonzero(d > 1e-8) == st["modified_pivots"]
    # a definite input is unchanged by the flag
    t2 = otlr.compress_dense(_cov(512, 64)[1], 128, 1e-8)
    m1, m2 = _upload(t2), _upload(t2)
    m1.potrf(1e-8)
    s2 = m2.potrf(1e-8, tlr.opts(flags=tlr.FLAG_MODIFIED_CHOL))
    assert s2["modified_pivots"] == 0
    l1, l2 = oracle_tlr(m1, tlr.FACTOR), oracle_tlr(m2, tlr.FACTOR)
    for k in range(t2.nb):
        np.testing.assert_array_equal(l1.diag[k], l2.diag[k])


def _factor_arrays(mat):
    diag, u, v, ranks = mat.to_host(tlr.FACTOR)
    return diag, u, v, ranks


@pytest.mark.parametrize("form", ["chol", "ldlt", "modified"])
def test_diag_graph_replay_matches_launches(form):
    # With TLR_FLAG_DIAG_GRAPH the diagonal tiles' factorization is captured
    # once as a HIP graph and replayed for every column, with the column's
    # other work between the replays; its factor must equal the
    # kernel-by-kernel launches' bit for bit, on every column (each column is
    # one replay), over two calls in a row, the second with the graph
    # already built.
    if form == "modified":
        n, m, eps = 384, 64, 1e-9
        t = otlr.compress_dense(_lost_definiteness(n, m), m, 1e-11)
        base = tlr.FLAG_MODIFIED_CHOL
    else:
        n, m, eps = 2048, 256, 1e-6
        t = otlr.compress_dense(_cov(n, 11)[1], m, eps)
        base = 0
    ref, got = _upload(t), _upload(t)

    def run(mat, flags):
        o = tlr.opts(flags=flags)
        if form == "ldlt":
            st, d = mat.ldlt(eps, o)
            return st, d.cpu().numpy()
        return mat.potrf(eps, o), None

    st_r, d_r = run(ref, base)
    for call in range(2):
        st_g, d_g = run(got, base | tlr.FLAG_DIAG_GRAPH)
        assert st_g["info"] == st_r["info"] == 0
        assert st_g["modified_pivots"] == st_r["modified_pivots"]
        if form == "modified":
            assert st_g["modified_pivots"] > 0
        a, b = _factor_arrays(ref), _factor_arrays(got)
        np.testing.assert_array_equal(a[3], b[3])
        for k in range(t.nb):
            np.testing.assert_array_equal(a[0][k], b[0][k])
        for key in a[1]:
            np.testing.assert_array_equal(a[1][key], b[1][key])
            np.testing.assert_array_equal(a[2][key], b[2][key])
        if d_r is not None:
            np.testing.assert_array_equal(d_r, d_g)
    # a failing tile is reported at its global row through the replay too
    if form == "chol":
        bad = t.dense_symmetric().copy()
        bad[700, 700] = -1.0
        tb = otlr.compress_dense(bad, m, eps)
        m1, m2 = _upload(tb), _upload(tb)
        s1, i1 = m1.potrf_status(eps)
        s2, i2 = m2.potrf_status(eps, tlr.opts(flags=tlr.FLAG_DIAG_GRAPH))
        assert s1 == s2 != 0
        assert i1["info"] == i2["info"] > 512
        m1.close()
        m2.close()
    ref.close()
    got.close()
