"""The batched factorization (several independent matrices stepped through
their block columns together, the ARA of all their Schur-complement tiles
pooled into one set of launches) against the FP64 oracle, per matrix, and
against the single-matrix call."""
import math

import numpy as np
import pytest

from oracle import dense
from oracle import tlr as otlr
from paper_2108_11932_amd import tlr
from paper_2108_11932_amd import workloads as wl

from gpu_util import RANK_RATIO, oracle_tlr

pytestmark = pytest.mark.gpu


def _cov(n, seed, ell=0.1, nugget=1e-4):
    pts = wl.uniform_points(n, 2, seed)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    return dense.covariance_matrix(pts, dense.KERNEL_EXP, ell, nugget)


def _upload(t):
    return tlr.TLRMatrix.from_tlr(t.n, t.m, t.diag, t.u, t.v)


def _residual(t, l, d=None):
    ad = t.dense_symmetric()
    ld = l.dense_lower()
    mid = np.diag(np.concatenate(d)) if d is not None else np.eye(ld.shape[0])
    return ad - ld @ mid @ ld.T


def _check_bounds(t, mat, tau, d=None):
    l = oracle_tlr(mat, tlr.FACTOR)
    res = _residual(t, l, d)
    for k in range(t.nb):
        for i in range(k + 1, t.nb):
            e = np.linalg.norm(res[t.blk(i), t.blk(k)], 2)
            assert e <= 4 * tau, (i, k, e, tau)
    assert np.linalg.norm(res, 2) <= 2 * math.sqrt(t.nb) * tau


def test_batch_of_one_is_the_single_call():
    a = _cov(1536, 41)
    eps = 1e-6
    t = otlr.compress_dense(a, 256, eps)
    one, batch = _upload(t), _upload(t)
    st1 = one.potrf(eps)
    s, sts, _ = tlr.factor_batched([batch], eps)
    assert s == 0 and sts[0]["info"] == 0
    assert sts[0]["ara_iters"] == st1["ara_iters"]
    np.testing.assert_array_equal(one.ranks(tlr.FACTOR), batch.ranks(tlr.FACTOR))
    l1, l2 = oracle_tlr(one, tlr.FACTOR), oracle_tlr(batch, tlr.FACTOR)
    for k in range(t.nb):
        np.testing.assert_array_equal(l1.diag[k], l2.diag[k])
        for i in range(k + 1, t.nb):
            np.testing.assert_array_equal(l1.u[i, k], l2.u[i, k])
            np.testing.assert_array_equal(l1.v[i, k], l2.v[i, k])


def test_batched_cholesky_keeps_every_matrix_bounds():
    # three matrices of one tile size and different block counts (ragged
    # last tiles): pooled launches over 3, 5 and 7 tiles per column
    eps = 1e-6
    ts = [otlr.compress_dense(_cov(n, 50 + n), 256, eps) for n in (2048, 1500, 1000)]
    mats = [_upload(t) for t in ts]
    s, sts, _ = tlr.factor_batched(mats, eps)
    assert s == 0
    for t, mat, st in zip(ts, mats, sts):
        assert st["info"] == 0 and st["tau"] == eps
        _check_bounds(t, mat, eps)
        ref = otlr.tlr_cholesky(t, eps)
        assert mat.ranks(tlr.FACTOR).sum() <= RANK_RATIO * ref.ranks().sum() + t.nb


def test_batched_relative_thresholds_and_tile_sizes():
    # relative thresholds differ per matrix (eps ||A_i||); two tile sizes
    # form two groups
    eps = 1e-6
    specs = [(1024, 128, 0.1), (1536, 256, 0.2), (1200, 128, 0.05)]
    ts, mats = [], []
    for n, m, ell in specs:
        a = _cov(n, 70 + n, ell=ell) * (1.0 + n / 1000.0)
        t = otlr.compress_dense(a, m, eps * np.linalg.norm(a, 2))
        ts.append(t)
        mats.append(_upload(t))
    o = tlr.opts(eps_mode=tlr.EPS_REL)
    s, sts, _ = tlr.factor_batched(mats, eps, o)
    assert s == 0
    taus = [st["tau"] for st in sts]
    assert len(set(taus)) == 3
    for t, mat, st in zip(ts, mats, sts):
        assert st["info"] == 0 and st["tau"] == pytest.approx(eps * st["norm_a"])
        _check_bounds(t, mat, st["tau"])


def test_batched_ldlt_returns_each_matrix_pivots():
    eps = 1e-6
    ts = [otlr.compress_dense(_cov(n, 90 + n), 256, eps) for n in (1536, 1024)]
    mats = [_upload(t) for t in ts]
    s, sts, ds = tlr.factor_batched(mats, eps, ldl=True)
    assert s == 0
    for t, mat, st, d in zip(ts, mats, sts, ds):
        assert st["info"] == 0
        dv = d.cpu().numpy()
        np.testing.assert_allclose(dv, mat.pivots(), rtol=0, atol=0)
        dl = [dv[t.blk(k)] for k in range(t.nb)]
        _check_bounds(t, mat, eps, dl)


def test_batched_failure_stays_with_its_matrix():
    eps = 1e-6
    good = otlr.compress_dense(_cov(1024, 111), 256, eps)
    bad = otlr.compress_dense(_cov(1024, 112), 256, eps)
    bad.diag[2] = bad.diag[2] - 10.0 * np.eye(256)   # tile 2 indefinite
    mats = [_upload(good), _upload(bad)]
    s, sts, _ = tlr.factor_batched(mats, eps)
    assert s == tlr.TLR_ERR_NOT_SPD
    assert sts[0]["info"] == 0
    assert 2 * 256 < sts[1]["info"] <= 3 * 256
    _check_bounds(good, mats[0], eps)


def test_tune_tile_measures_then_caches():
    w = wl.batched_2d(count=3)[0]
    tlr.lib().tlr_tune_reset()
    best, ms = tlr.tune_tile(w.points, w.kernel, w.ell, w.diag_add, w.eps, (128, 256, 512))
    assert best in (128, 256, 512)
    assert ms is not None and all(np.isfinite(v) and v > 0 for v in ms.values())
    assert ms[best] == min(ms.values())
    # the same problem class (same ceil(log2 N), kernel, threshold, options)
    again, ms2 = tlr.tune_tile(w.points, w.kernel, w.ell, w.diag_add, w.eps, (128, 256, 512))
    assert again == best and ms2 is None
    tlr.lib().tlr_tune_reset()
    _, ms3 = tlr.tune_tile(w.points, w.kernel, w.ell, w.diag_add, w.eps, (128, 256, 512))
    assert ms3 is not None


def test_batched_workload_eight_problems_against_oracle():
    # 8 of the 96 problems of the batched workload (the smallest, so that the
    # oracle's TLR-SVD factorization stays quick), tile sizes from the
    # autotuner, one batched call with per-problem relative thresholds
    ws = sorted(wl.batched_2d(count=96), key=lambda w: w.n)[:8]
    tlr.lib().tlr_tune_reset()
    o = tlr.opts(eps_mode=tlr.EPS_REL)
    mats, tiles = [], []
    for w in ws:
        m, _ = tlr.tune_tile(w.points, w.kernel, w.ell, w.diag_add, w.eps, (256, 512, 1024), o)
        tiles.append(m)
        mats.append(tlr.TLRMatrix.compress_kernel(w.points, w.kernel, w.ell, w.diag_add, m, w.eps, o))
    s, sts, _ = tlr.factor_batched(mats, ws[0].eps, o)
    assert s == 0
    for w, mat, st in zip(ws, mats, sts):
        assert st["info"] == 0
        tau = st["tau"]
        assert tau == pytest.approx(w.eps * st["norm_a"])
        a_t = oracle_tlr(mat, tlr.INPUT)
        l = oracle_tlr(mat, tlr.FACTOR)
        assert otlr.factor_error_norm(a_t, l) <= 2 * math.sqrt(a_t.nb) * tau
        ref = otlr.tlr_cholesky(a_t, tau)
        assert l.ranks().sum() <= RANK_RATIO * ref.ranks().sum() + a_t.nb
        mat.close()
