"""Parity of the GPU factorization with the FP64 oracle at the shapes of the
benchmark workloads, bit-exact integer bookkeeping, and the edge and error
paths of the C ABI.

* the 2D covariance at N = 4096, tile 256, absolute eps 1e-6 (seed 1)
  against the dense Cholesky (O2) and the left-looking TLR-SVD oracle (O4);
* the leading 12288 points of the N = 131072 workload at the benchmark's
  tile size 1024, with the sampling product forced onto its 64-row strips
  (the path that carries the full-size run) and checked bit for bit against
  the 16-row strips, in FP64 and with FP32 panels;
* a shifted, indefinite 3D Matern-1.5 LDL^T at ARA block 32 (the LDL^T
  workload's recipe at N = 4096), input generator against the oracle's,
  Sylvester inertia and the error bound;
* bookkeeping: offsets, sortRanks orders and the test matrices bit-exact;
* full-rank tiles (q = m), dense input, allocation failure, automatic
  shift, per-problem thresholds of the batched form and phase timers.

ARA is randomized, so the factor is not unique: the factor is checked
through what the method fixes (per-tile backward error equals the
compression error of the left-looking update, the global bound, Eckart-Young
lower bounds on the ranks), and against the oracle's optimal ranks.
"""
import ctypes
import math

import numpy as np
import pytest

from oracle import bookkeeping as bk
from oracle import dense
from oracle import philox as oph
from oracle import tlr as otlr
from paper_2108_11932_amd import tlr
from paper_2108_11932_amd import workloads as wl

from gpu_util import RANK_RATIO, oracle_tlr, tile_errors

pytestmark = pytest.mark.gpu

# Per-tile bound of the compressed Schur-complement tiles: none above 2 tau
# (the rate above tau is measured across seeds in test_gpu_ara_failure_rate).
TILE_BOUND = 2.0


def _points(n, dim, seed):
    pts = wl.jittered_grid(n, dim, seed)
    return np.ascontiguousarray(pts[wl.morton_order(pts)])


def _check_bookkeeping(mat):
    ra = mat.ranks(tlr.INPUT)
    rl = mat.ranks(tlr.FACTOR)
    off_in, _ = bk.lower_offsets(ra)
    np.testing.assert_array_equal(mat.offsets(tlr.INPUT), off_in)
    np.testing.assert_array_equal(mat.offsets(tlr.FACTOR), bk.row_panel_offsets(rl))
    for k in range(mat.nb):
        assert mat.sort_order(k) == bk.sort_ranks(ra, k), k


def _same_factor(l1, l2):
    np.testing.assert_array_equal(l1.ranks(), l2.ranks())
    for k in range(l1.nb):
        np.testing.assert_array_equal(l1.diag[k], l2.diag[k])
        for i in range(k + 1, l1.nb):
            np.testing.assert_array_equal(l1.u[i, k], l2.u[i, k])
            np.testing.assert_array_equal(l1.v[i, k], l2.v[i, k])


def _eckart_young(a_t, l, off, scale):
    """Every rank is at least the number of singular values of the GPU's own
    Schur tile above the error it reached."""
    rl = l.ranks()
    for (i, k), e in off.items():
        sv = np.linalg.svd(otlr.schur_tile(a_t, l, i, k), compute_uv=False)
        assert rl[i, k] >= int(np.sum(sv > e * (1 + 1e-8) + 1e-14 * scale)), (i, k)


def test_cov2d_4k_against_dense_and_tlr_oracles():
    w = wl.standard("cov2d_4k")   # N 4096, tile 256, eps 1e-6 absolute, seed 1
    eps, m = w.eps, w.m
    mat = tlr.TLRMatrix.compress_kernel(w.points, tlr.KERNEL_EXP, w.ell, w.diag_add, m, eps)
    a_t = oracle_tlr(mat, tlr.INPUT)
    # the input generator and compression against the exact tiles
    for i in range(a_t.nb):
        exact = otlr.kernel_tile(w.points, m, i, i, dense.KERNEL_EXP, w.ell, w.diag_add)
        np.testing.assert_allclose(a_t.diag[i], exact, rtol=0, atol=1e-14)
        for j in range(i):
            exact = otlr.kernel_tile(w.points, m, i, j, dense.KERNEL_EXP, w.ell, w.diag_add)
            assert np.linalg.norm(exact - a_t.tile(i, j), 2) <= TILE_BOUND * eps
    st = mat.potrf(eps)
    assert st["info"] == 0 and st["tau"] == eps
    l = oracle_tlr(mat, tlr.FACTOR)
    off, diag = tile_errors(a_t, l)
    a_dense = dense.covariance_matrix(w.points, dense.KERNEL_EXP, w.ell, w.diag_add)
    scale = np.linalg.norm(a_dense, 2)
    assert max(diag.values()) <= 1e-11 * scale
    assert max(off.values()) <= TILE_BOUND * eps
    nb = a_t.nb
    err_tlr = otlr.factor_error_norm(a_t, l)
    assert err_tlr <= 2 * math.sqrt(nb) * eps
    # O4 on the same input: its error is the reference the GPU's is held to
    ref = otlr.tlr_cholesky(a_t, eps)
    err_ref = otlr.factor_error_norm(a_t, ref)
    assert err_ref <= math.sqrt(nb) * eps
    assert err_tlr <= 2 * err_ref + eps
    rg, ro = l.ranks(), ref.ranks()
    assert rg.sum() <= RANK_RATIO * ro.sum() + nb
    _eckart_young(a_t, l, off, scale)
    # O2: the dense matrix, its Cholesky solve and the GPU solve
    n = w.n
    ld = l.dense_lower()[:n, :n]
    err_dense = dense.norm2_power(lambda x: a_dense @ x - ld @ (ld.T @ x), n, seed=3, iters=40)
    err_in = dense.norm2_power(lambda x: a_dense @ x - otlr.matvec(a_t, x), n, seed=3, iters=40)
    assert err_dense <= err_in + 2 * math.sqrt(nb) * eps
    import torch
    b = np.random.default_rng(5).standard_normal((n, 2))
    x = mat.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    lc = dense.cholesky(a_dense)
    x_ref = dense.solve_lower(lc, dense.solve_lower(lc, b), trans=True)
    berr = np.linalg.norm(b - a_dense @ x) / (scale * np.linalg.norm(x))
    assert berr <= (err_dense + 1e-12 * scale) / scale * 1.01
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 1e-3
    _check_bookkeeping(mat)


@pytest.fixture(scope="module")
def tile1024_sample():
    """The leading 12288 points of the N = 131072 workload at tile 1024."""
    w = wl.standard("cov2d_131k")
    pts = np.ascontiguousarray(w.points[:12288])
    mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, w.ell, w.diag_add, w.m, w.eps)
    return w, pts, mat, oracle_tlr(mat, tlr.INPUT)


def test_tile1024_fp64_strips_and_oracle(tile1024_sample):
    w, pts, mat, a_t = tile1024_sample
    eps = w.eps
    st16 = mat.potrf(eps, tlr.opts(sample_strip=16))
    l16 = oracle_tlr(mat, tlr.FACTOR)
    st64 = mat.potrf(eps, tlr.opts(sample_strip=64))
    l = oracle_tlr(mat, tlr.FACTOR)
    # the 64-row strips accumulate in the 16-row strips' order: same factor
    assert st64["ara_iters"] == st16["ara_iters"]
    _same_factor(l, l16)
    off, diag = tile_errors(a_t, l)
    nb = a_t.nb
    assert max(off.values()) <= TILE_BOUND * eps
    assert max(diag.values()) <= 1e-11 * otlr.norm2(a_t)
    assert otlr.factor_error_norm(a_t, l) <= 2 * math.sqrt(nb) * eps
    ref = otlr.tlr_cholesky(a_t, eps)
    assert l.ranks().sum() <= RANK_RATIO * ref.ranks().sum() + nb
    _check_bookkeeping(mat)


def test_sampling_lookahead_same_as_serial(tile1024_sample):
    # the samples of iteration t + 1 drawn on the sampling stream during
    # iteration t's orthogonalisation (the default) against every sampling
    # after the previous iteration on one stream: the same factor bit for
    # bit, in FP64 and with FP32 panels, and the same compression
    w, pts, mat, a_t = tile1024_sample
    for kw in ({}, {"eps_mode": tlr.EPS_REL, "precision": tlr.MIXED_FP32}):
        st_o = mat.potrf(w.eps, tlr.opts(**kw))
        l_o = oracle_tlr(mat, tlr.FACTOR)
        st_s = mat.potrf(w.eps, tlr.opts(flags=tlr.FLAG_SERIAL_SAMPLING, **kw))
        l_s = oracle_tlr(mat, tlr.FACTOR)
        assert st_o["ara_iters"] == st_s["ara_iters"]
        _same_factor(l_o, l_s)
    sub = np.ascontiguousarray(pts[:4096])
    c = [tlr.TLRMatrix.compress_kernel(sub, tlr.KERNEL_EXP, w.ell, w.diag_add, 512, 1e-6,
                                       tlr.opts(flags=f))
         for f in (0, tlr.FLAG_SERIAL_SAMPLING)]
    _same_factor(oracle_tlr(c[0], tlr.INPUT), oracle_tlr(c[1], tlr.INPUT))
    # LDL^T of the same input
    d = []
    for f in (0, tlr.FLAG_SERIAL_SAMPLING):
        c[0].ldlt(1e-6, tlr.opts(flags=f))
        d.append(oracle_tlr(c[0], tlr.FACTOR))
    _same_factor(d[0], d[1])
    for x in c:
        x.close()


def test_tile1024_mixed_strips_and_accuracy(tile1024_sample):
    w, pts, mat, a_t = tile1024_sample
    eps = w.eps
    errs, stats = {}, {}
    mat.potrf(eps, tlr.opts(eps_mode=tlr.EPS_REL, precision=tlr.MIXED_FP32, sample_strip=16))
    l16 = oracle_tlr(mat, tlr.FACTOR)
    for prec in (tlr.FP64, tlr.MIXED_FP32):
        st = mat.potrf(eps, tlr.opts(eps_mode=tlr.EPS_REL, precision=prec, sample_strip=64))
        l = oracle_tlr(mat, tlr.FACTOR)
        errs[prec] = otlr.factor_error_norm(a_t, l)
        stats[prec] = st
    _same_factor(l, l16)
    s32 = stats[tlr.MIXED_FP32]
    # the rounding guard grows with sqrt(R_i): at tile 1024 the long panels
    # of the later block rows keep FP64, the others take the FP32 copies
    assert s32["fp32_tile_iters"] > 0.1 * s32["tile_iters"]
    tau = s32["tau"]
    assert errs[tlr.MIXED_FP32] <= 2 * math.sqrt(a_t.nb) * tau
    assert errs[tlr.MIXED_FP32] <= 2 * errs[tlr.FP64] + tau


def test_ldlt_matern3d_shifted_indefinite():
    n, m, eps = 4096, 256, 1e-4
    pts = _points(n, 3, 4)
    shift = wl.MATERN3D_SHIFT_FRACTION * wl.matern3d_norm_estimate(pts)
    mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_MATERN15, 0.2, -shift, m, eps,
                                        tlr.opts(bs=32))
    a_t = oracle_tlr(mat, tlr.INPUT)
    ref_in = otlr.compress_kernel(pts, m, dense.KERNEL_MATERN15, 0.2, -shift, eps)
    for i in range(a_t.nb):
        np.testing.assert_allclose(a_t.diag[i], ref_in.diag[i], rtol=0, atol=1e-13)
        for j in range(i):
            exact = otlr.kernel_tile(pts, m, i, j, dense.KERNEL_MATERN15, 0.2, -shift)
            assert np.linalg.norm(exact - a_t.tile(i, j), 2) <= TILE_BOUND * eps
            assert a_t.rank(i, j) >= ref_in.rank(i, j) - 2
    st, d = mat.ldlt(eps, tlr.opts(bs=32))
    assert st["info"] == 0
    l = oracle_tlr(mat, tlr.FACTOR)
    piv = mat.pivots()
    dl = [piv[k * m:(k + 1) * m] for k in range(a_t.nb)]
    off, diag = tile_errors(a_t, l, dl)
    assert max(off.values()) <= TILE_BOUND * eps
    err = otlr.factor_error_norm(a_t, l, dl)
    assert err <= 2 * math.sqrt(a_t.nb) * eps
    # Sylvester: D has as many negative entries as A_tlr has negative
    # eigenvalues, whenever no eigenvalue lies within the error of zero
    ev = np.linalg.eigvalsh(a_t.dense_symmetric()[:n, :n])
    neg = int(np.sum(ev < 0))
    assert 0 < neg < n
    assert np.min(np.abs(ev)) > err, "an eigenvalue within the factor error of zero"
    assert int(np.sum(d.cpu().numpy() < 0)) == neg
    # O5 on the same input reaches the same inertia
    ref, dref = otlr.tlr_ldlt(a_t, eps)
    assert int(np.sum(np.concatenate(dref)[:n] < 0)) == neg


def test_gpu_ara_failure_rate():
    # the per-tile bound of the compressed Schur-complement tiles over
    # several inputs and test-matrix streams (the N = 4096, tile 256 recipe
    # at three grid seeds, two Philox seeds each): none above 2 tau, and at
    # most 1% of the tiles above tau
    eps, m = 1e-6, 256
    errs = []
    for seed in (1, 2, 3):
        pts = _points(4096, 2, seed)
        mat = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-4, m, eps)
        a_t = oracle_tlr(mat, tlr.INPUT)
        for ara_seed in (0x5eed, 1234):
            mat.potrf(eps, tlr.opts(seed=ara_seed))
            off, _ = tile_errors(a_t, oracle_tlr(mat, tlr.FACTOR))
            errs += list(off.values())
        mat.close()
    e = np.array(errs) / eps
    assert e.max() <= TILE_BOUND, e.max()
    assert (e > 1.0).mean() <= 0.01, (e > 1.0).mean()


@pytest.mark.parametrize("cols0,cols1,t0,nt", [(16, 16, 0, 16), (16, 32, 0, 5), (24, 8, 16, 3)])
def test_randn_iters_bit_exact(cols0, cols1, t0, nt):
    rows, seed, k = 257, 0x5EED, 9
    mats = tlr.randn_iters(rows, cols0, cols1, seed, k, t0, nt, 0)
    for i, got in enumerate(mats):
        t = t0 + i
        c = cols0 if t == 0 else cols1
        ref = oph.test_matrix(seed, k, t, 0, rows, c)
        np.testing.assert_array_equal(got, tlr.randn(rows, c, seed, k, t, 0))
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_full_rank_tiles():
    # every off-diagonal tile of G G^T / n + I is of full rank: the ARA must
    # stop at q = m and the factor stay exact
    n, m = 192, 32
    g = np.random.default_rng(41).standard_normal((n, n))
    a = g @ g.T / n + np.eye(n)
    tau = 1e-12
    t = otlr.compress_dense(a, m, tau)
    assert (t.ranks()[np.tril_indices(t.nb, -1)] == m).all()
    mat = tlr.TLRMatrix.from_tlr(t.n, t.m, t.diag, t.u, t.v)
    st = mat.potrf(tau)
    nlow = t.nb * (t.nb - 1) // 2
    assert st["full_rank_tiles"] == nlow and st["max_rank"] == m
    l = oracle_tlr(mat, tlr.FACTOR)
    res = a - l.dense_lower() @ l.dense_lower().T
    assert np.abs(res).max() <= 1e-10 * np.abs(a).max()


def test_compress_dense_input():
    import torch
    n, m, eps = 1500, 256, 1e-6
    pts = np.ascontiguousarray(wl.uniform_points(n, 2, 12)[wl.morton_order(wl.uniform_points(n, 2, 12))])
    a = dense.covariance_matrix(pts, dense.KERNEL_EXP, 0.1, 1e-4)
    mat = tlr.TLRMatrix.compress(torch.from_numpy(a).cuda(), m, eps)
    got = oracle_tlr(mat, tlr.INPUT)
    ap = otlr.pad_dense(a, m)
    for i in range(got.nb):
        np.testing.assert_allclose(got.diag[i], ap[got.blk(i), got.blk(i)], rtol=0, atol=0)
        for j in range(i):
            tile = ap[got.blk(i), got.blk(j)]
            e = np.linalg.norm(tile - got.tile(i, j), 2)
            assert e <= TILE_BOUND * eps
            sv = np.linalg.svd(tile, compute_uv=False)
            assert got.rank(i, j) >= int(np.sum(sv > e * (1 + 1e-8)))
            assert got.rank(i, j) <= int(np.sum(sv > eps)) + 16
    assert not got.u[got.nb - 1, 0][n - (got.nb - 1) * m:].any()
    np.testing.assert_array_equal(mat.offsets(tlr.INPUT), bk.lower_offsets(mat.ranks(tlr.INPUT))[0])


class _FailingAllocator(tlr.TorchAllocator):
    """torch-backed allocator that returns NULL once `budget` further
    allocations have been made (budget < 0: never fails)."""

    def __init__(self):
        self.budget = -1
        super().__init__()

    def _alloc(self, ctx, nbytes, stream):
        if self.budget == 0:
            return None
        if self.budget > 0:
            self.budget -= 1
        return super()._alloc(ctx, nbytes, stream)


def test_allocation_failures_report_oom_and_leave_a_usable_handle():
    l = tlr.lib()
    al = _FailingAllocator()
    al.budget = 0
    h = ctypes.c_void_p()
    assert l.tlr_create(1024, 128, None, ctypes.byref(al.struct), tlr._stream(),
                        ctypes.byref(h)) == tlr.TLR_ERR_OOM
    assert h.value is None
    # a handle whose factorization runs out of memory at several points
    pts = _points(2048, 2, 31)
    a = dense.covariance_matrix(pts, dense.KERNEL_EXP, 0.1, 1e-4)
    t = otlr.compress_dense(a, 256, 1e-6)
    al = _FailingAllocator()
    ranks = t.ranks()
    h = ctypes.c_void_p()
    tlr._check(l.tlr_create(t.n, t.m, ranks.ctypes.data_as(tlr._IP), ctypes.byref(al.struct),
                            tlr._stream(), ctypes.byref(h)))
    mat = tlr.TLRMatrix(h, al)
    for k in range(t.nb):
        d = np.asfortranarray(t.diag[k])
        tlr._check(l.tlr_set_diag(mat.h, k, d.ctypes.data_as(tlr._P), t.m, 0))
    for (i, j), u in t.u.items():
        if u.shape[1]:
            U, V = np.asfortranarray(u), np.asfortranarray(t.v[i, j])
            tlr._check(l.tlr_set_tile(mat.h, i, j, U.ctypes.data_as(tlr._P),
                                      V.ctypes.data_as(tlr._P), t.m, 0))
    import torch
    b = torch.ones(t.n, dtype=torch.float64, device="cuda")
    for budget in (0, 3, 12, 30):
        al.budget = budget
        status, st = mat.potrf_status(1e-6)
        if status == tlr.TLR_OK:
            continue
        assert status == tlr.TLR_ERR_OOM, (budget, status)
        assert l.tlr_solve(mat.h, 1, tlr._ptr(b), t.n, tlr._stream()) == tlr.TLR_ERR_STATE
        r = np.zeros((t.nb, t.nb), dtype=np.int32)
        assert l.tlr_get_ranks(mat.h, tlr.FACTOR, r.ctypes.data_as(tlr._IP)) == tlr.TLR_ERR_STATE
    al.budget = -1
    st = mat.potrf(1e-6)
    assert st["info"] == 0
    lf = oracle_tlr(mat, tlr.FACTOR)
    assert otlr.factor_error_norm(t, lf) <= 2 * math.sqrt(t.nb) * 1e-6
    mat.close()


def test_auto_shift_restores_definiteness():
    # at a relative threshold of 3e-2 the unshifted factorization of the
    # N = 4096 covariance loses definiteness in an early diagonal tile; with
    # auto_shift it is repeated with the shift s = tau of Section 5.1
    w = wl.standard("cov2d_4k")
    mat = tlr.TLRMatrix.compress_kernel(w.points, tlr.KERNEL_EXP, w.ell, w.diag_add, w.m, 1e-9)
    a_t = oracle_tlr(mat, tlr.INPUT)
    eps = 3e-2
    status, st = mat.potrf_status(eps, tlr.opts(eps_mode=tlr.EPS_REL))
    assert status == tlr.TLR_ERR_NOT_SPD and st["info"] > 0
    st = mat.potrf(eps, tlr.opts(eps_mode=tlr.EPS_REL, auto_shift=1))
    assert st["shift_retries"] == 1 and st["shift"] == st["tau"] > 0
    l = oracle_tlr(mat, tlr.FACTOR)
    # the factor is that of A + tau I: error against the unshifted A
    err = otlr.factor_error_norm(a_t, l)
    assert err <= 2 * math.sqrt(a_t.nb) * st["tau"] + st["tau"]
    # a definite run keeps shift 0
    st = mat.potrf(1e-6, tlr.opts(auto_shift=1))
    assert st["shift_retries"] == 0 and st["shift"] == 0.0


def test_batched_per_problem_thresholds():
    epss = [1e-5, 1e-6, 1e-7]
    ts, mats = [], []
    for n, e in zip((1536, 2048, 1000), epss):
        pts = np.ascontiguousarray(wl.uniform_points(n, 2, 60 + n)[wl.morton_order(wl.uniform_points(n, 2, 60 + n))])
        a = dense.covariance_matrix(pts, dense.KERNEL_EXP, 0.1, 1e-4)
        t = otlr.compress_dense(a, 256, e)
        ts.append(t)
        mats.append(tlr.TLRMatrix.from_tlr(t.n, t.m, t.diag, t.u, t.v))
    s, sts, _ = tlr.factor_batched_eps(mats, epss)
    assert s == 0
    for t, mat, st, e in zip(ts, mats, sts, epss):
        assert st["info"] == 0 and st["tau"] == e
        l = oracle_tlr(mat, tlr.FACTOR)
        off, _ = tile_errors(t, l)
        assert max(off.values()) <= TILE_BOUND * e
        _check_bookkeeping(mat)
    # a non-positive threshold is an argument error
    s, _, _ = tlr.factor_batched_eps(mats, [1e-6, 0.0, 1e-6])
    assert s == tlr.TLR_ERR_ARG


def test_phase_timers_cover_the_step():
    w = wl.standard("cov2d_4k")
    mat = tlr.TLRMatrix.compress_kernel(w.points, tlr.KERNEL_EXP, w.ell, w.diag_add, w.m, w.eps)
    st = mat.potrf(w.eps)
    assert st["t_total"] > 0 and not any(st["t_phase"])
    o = tlr.opts(flags=tlr.FLAG_PHASE_TIMING)
    mat.potrf(w.eps, o)
    st = mat.potrf(w.eps, o)
    ph = st["t_phase"]
    main = sum(ph[:7])
    assert min(ph) >= 0.0 and ph[tlr.PHASES.index("diag")] > 0.0
    for name in ("sample", "orth", "batch", "project", "trsm", "append"):
        assert ph[tlr.PHASES.index(name)] > 0.0, name
    # the main-stream phases tile the stream's span, which fits in the call
    assert 0.5 * st["t_total"] <= main <= 1.02 * st["t_total"]
