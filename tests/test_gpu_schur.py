"""Schur compensation (Section 5.1.1) on the GPU against the oracle's
definition, applied to the GPU's own factor: for every column k >= 1 the
accumulated update D_k = sum_j L_kj L_kj^T is formed on the host from the
downloaded factor tiles, the oracle's compensation vector
c = rowsum |D_k - Dbar_k| (dense.schur_compensation: truncated
eigen-decomposition at tau) is computed from it, and the GPU's diagonal
tile must satisfy L_kk L_kk^T = A_kk - D_k + diag(c)."""
import numpy as np
import pytest

from oracle import dense
from paper_2108_11932_amd import tlr
from paper_2108_11932_amd import workloads as wl

from gpu_util import oracle_tlr

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,m,eps", [(2048, 128, 1e-4), (2048, 256, 1e-5), (1900, 128, 1e-3)])
def test_schur_compensation_matches_oracle(n, m, eps):
    pts = wl.uniform_points(n, 2, 31) if n & (n - 1) else wl.jittered_grid(n, 2, 31)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-4, m, 1e-9)
    st = mat.potrf(eps, tlr.opts(bs=16, flags=tlr.FLAG_SCHUR_COMP))
    tau = st["tau"]
    a = oracle_tlr(mat, tlr.INPUT)
    l = oracle_tlr(mat, tlr.FACTOR)
    anorm = max(np.abs(a.diag[k]).max() for k in range(a.nb))
    comp_max = 0.0
    for k in range(a.nb):
        upd = np.zeros((m, m))
        for j in range(k):
            upd += l.u[k, j] @ (l.v[k, j].T @ l.v[k, j]) @ l.u[k, j].T
        c = dense.schur_compensation(upd, tau) if k > 0 else np.zeros(m)
        nr = min(m, n - k * m)
        c[nr:] = 0.0    # the padding keeps its identity
        want = a.diag[k] - upd + np.diag(c)
        got = np.tril(l.diag[k]) @ np.tril(l.diag[k]).T
        np.testing.assert_allclose(got, want, atol=1e-11 * anorm, err_msg="tile %d" % k)
        # the compensation the GPU applied, against the oracle's
        c_gpu = np.diag(got - a.diag[k] + upd)
        np.testing.assert_allclose(c_gpu[:nr], c[:nr], atol=1e-11 * anorm, err_msg="tile %d" % k)
        comp_max = max(comp_max, float(c.max()))
    assert 0.0 < comp_max <= np.sqrt(m) * tau
    # the solve still inverts the compensated factor
    import torch
    b = np.random.default_rng(2).standard_normal(n)
    x = mat.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    d = dense.covariance_matrix(pts, dense.KERNEL_EXP, 0.1, 1e-4)
    assert np.linalg.norm(d @ x - b) / np.linalg.norm(b) < 1e3 * tau * np.linalg.norm(x)
    mat.close()


def test_schur_compensation_rejected_outside_unpivoted_cholesky():
    pts = wl.jittered_grid(1024, 2, 3)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-4, 128, 1e-6)
    o = tlr.opts(bs=16, flags=tlr.FLAG_SCHUR_COMP)
    for call in (lambda: mat.ldlt(1e-6, o), lambda: mat.potrf_pivoted(1e-6, o)):
        with pytest.raises(tlr.TLRError) as e:
            call()
        assert e.value.status == -1
    # the batched entry returns its status
    assert tlr.factor_batched([mat], 1e-6, o)[0] == -1
    # the handle is untouched: the plain factorization still runs
    mat.potrf(1e-6, tlr.opts(bs=16))
    mat.close()


def test_schur_compensation_with_graph_replay_and_modified_cholesky():
    """The compensation is added to the updated tile before the diagonal
    factorization, so the captured-graph replay of that factorization gives
    the factor of the launches bit for bit, and modified Cholesky combines
    with it (a definite run raises no pivot and matches the plain one)."""
    pts = wl.jittered_grid(2048, 2, 9)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-4, 128, 1e-8)
    base = tlr.FLAG_SCHUR_COMP
    ref = None
    for fl in (base, base | tlr.FLAG_DIAG_GRAPH, base | tlr.FLAG_MODIFIED_CHOL,
               base | tlr.FLAG_DIAG_GRAPH | tlr.FLAG_MODIFIED_CHOL):
        st = mat.potrf(1e-5, tlr.opts(bs=16, flags=fl))
        l = oracle_tlr(mat, tlr.FACTOR)
        if ref is None:
            ref = l
            continue
        assert st["modified_pivots"] == 0
        for k in range(l.nb):
            np.testing.assert_array_equal(l.diag[k], ref.diag[k])
        for key in ref.u:
            np.testing.assert_array_equal(l.u[key], ref.u[key])
            np.testing.assert_array_equal(l.v[key], ref.v[key])
    mat.close()
