"""Pivoted TLR Cholesky on the GPU (Algorithm "Pivoted Left Looking TLR
Cholesky", Section 5.2) against the oracle's pivoted factorization, through
the C ABI.

The pivot is an argmax of floating-point norms, and the GPU's factor comes
from a randomized compression, so two kinds of checks:

* matrices whose pivot choices are separated by a wide margin at every step
  (checked on the oracle's own run): the permutation must equal the
  oracle's exactly;
* a 3D covariance with close norms: every pivot the GPU took must be a
  largest updated diagonal norm of its own factor (recomputed on the host in
  FP64), and P A P^T = L L^T to the error bound of the unpivoted form.
"""
import math

import numpy as np
import pytest

from oracle import dense
from oracle import tlr as otlr
from paper_2108_11932_amd import tlr
from paper_2108_11932_amd import workloads as wl

from gpu_util import RANK_RATIO, oracle_tlr, tile_errors

pytestmark = pytest.mark.gpu


def _upload(t):
    return tlr.TLRMatrix.from_tlr(t.n, t.m, t.diag, t.u, t.v)


def _updated_norms(a_t, l, perm, k):
    """||A(perm t, perm t) - sum_{j<k} L_tj L_tj^T||_F for the positions t >= k
    of a factor l in its final block order."""
    ap = otlr.permute(a_t, perm)
    out = []
    for t in range(k, a_t.nb):
        d = ap.diag[t].copy()
        for j in range(k):
            d -= l.u[t, j] @ ((l.v[t, j].T @ l.v[t, j]) @ l.u[t, j].T)
        out.append(np.linalg.norm(d, "fro"))
    return np.array(out)


def _scaled_cov(n, m, seed, scales):
    pts = wl.jittered_grid(n, 2, seed)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    c = dense.covariance_matrix(pts, dense.KERNEL_EXP, 0.1, 1e-4)
    s = np.repeat(np.sqrt(np.asarray(scales, dtype=float)), m)[:n]
    return c * s[:, None] * s[None, :]


def test_pivoted_order_matches_oracle_when_separated():
    # block scales far apart: the oracle's choice wins by a wide margin at
    # every step, so the GPU must take the same permutation
    n, m, eps = 2048, 256, 1e-7
    scales = [1.0, 40.0, 6.0, 300.0, 2.5, 90.0, 15.0, 1000.0]
    a = _scaled_cov(n, m, 41, scales)
    t = otlr.compress_dense(a, m, eps)
    ref, perm_ref = otlr.tlr_cholesky_pivoted(t, eps)
    for k in range(t.nb - 1):
        nr = _updated_norms(t, ref, perm_ref, k)
        assert nr[0] >= 1.05 * np.sort(nr)[-2], k   # the margin the claim rests on
    mat = _upload(t)
    st, perm = mat.potrf_pivoted(eps)
    assert st["info"] == 0
    assert perm.tolist() == perm_ref
    assert perm.tolist() != list(range(t.nb))
    np.testing.assert_array_equal(mat.perm(), perm)
    l = oracle_tlr(mat, tlr.FACTOR)
    ap = otlr.permute(t, perm.tolist())
    off, diag = tile_errors(ap, l)
    assert max(off.values()) <= 4 * eps
    assert max(diag.values()) <= 1e-11 * np.linalg.norm(a, 2)
    assert otlr.factor_error_norm(ap, l) <= 2 * math.sqrt(t.nb) * eps
    # the first diagonal tile is the LAPACK Cholesky of the largest block
    b = perm[0]
    np.testing.assert_allclose(l.diag[0], np.linalg.cholesky(t.diag[b]), rtol=0,
                               atol=1e-11 * np.abs(t.diag[b]).max())
    # solve of A x = b with the pivoted factor against the oracle's
    import torch
    rhs = np.random.default_rng(3).standard_normal((n, 2))
    x = mat.solve(torch.from_numpy(rhs).cuda()).cpu().numpy()
    x_ref = np.linalg.solve(a, rhs)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 1e-3
    res = np.linalg.norm(a @ x - rhs) / (np.linalg.norm(a, 2) * np.linalg.norm(x))
    assert res <= 1e-7
    mat.close()


def test_pivoted_3d_covariance_pivot_rule_and_bound():
    # 3D exponential covariance (the paper's pivoting experiment, small):
    # norms are close, so the check is the pivot rule on the GPU's own factor
    n, m, eps = 4096, 256, 1e-6
    pts = wl.jittered_grid(n, 3, 7)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.2, 1e-4, m, eps)
    a_t = oracle_tlr(mat, tlr.INPUT)
    st, perm = mat.potrf_pivoted(eps)
    assert st["info"] == 0 and sorted(perm.tolist()) == list(range(a_t.nb))
    l = oracle_tlr(mat, tlr.FACTOR)
    for k in range(a_t.nb - 1):
        nr = _updated_norms(a_t, l, perm.tolist(), k)
        assert nr[0] >= nr.max() * (1 - 1e-10), (k, nr[0], nr.max())
    ap = otlr.permute(a_t, perm.tolist())
    off, diag = tile_errors(ap, l)
    assert max(off.values()) <= 4 * eps
    assert otlr.factor_error_norm(ap, l) <= 2 * math.sqrt(a_t.nb) * eps
    # ranks against the oracle's pivoted run on the same input
    ref, _ = otlr.tlr_cholesky_pivoted(a_t, eps)
    assert l.ranks().sum() <= RANK_RATIO * ref.ranks().sum() + a_t.nb
    # the unpivoted factorization of the same handle leaves no permutation
    mat.potrf(eps)
    np.testing.assert_array_equal(mat.perm(), np.arange(a_t.nb))
    mat.close()


def test_pivoted_rejects_mixed_precision():
    n, m = 512, 128
    a = _scaled_cov(n, m, 5, [1.0] * 4)
    mat = _upload(otlr.compress_dense(a, m, 1e-6))
    with pytest.raises(tlr.TLRError):
        mat.potrf_pivoted(1e-6, tlr.opts(precision=tlr.MIXED_FP32))
    mat.close()
