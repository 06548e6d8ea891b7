"""Parity of each HIP building block with the oracle (or the library routine
its definition reduces to), through the C ABI, on seeded inputs that span
several tiles of the kernels and ragged tails."""
import math

import numpy as np
import pytest

from oracle import bookkeeping as bk
from oracle import dense
from oracle import philox as oph
from paper_2108_11932_amd import tlr

from gpu_util import dev, host

pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps / 2


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


_GEMM_SIZES = {
    # batches whose largest K exceeds 32 run with 64-deep K slices
    "long": [(1, 1, 1), (3, 17, 5), (64, 16, 64), (65, 15, 4), (130, 70, 33), (7, 129, 0),
             (200, 16, 300), (16, 64, 1), (1, 300, 2), (70, 64, 1030)],
    # the others with 16-deep slices
    "short": [(1, 1, 1), (3, 17, 5), (65, 15, 4), (130, 70, 32), (7, 129, 0), (16, 64, 1),
              (1, 300, 2), (70, 64, 17)],
}


@pytest.mark.parametrize("kind", ["long", "short"])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_batched_ragged(ta, tb, kind):
    rng = np.random.default_rng(10 + 2 * ta + tb)
    sizes = _GEMM_SIZES[kind]
    probs, refs, outs = [], [], []
    for (M, N, K) in sizes:
        A = rng.standard_normal((K, M) if ta else (M, K))
        B = rng.standard_normal((N, K) if tb else (K, N))
        C = rng.standard_normal((M, N))
        alpha, beta = rng.uniform(-2, 2), [0.0, 1.0, -0.5][len(probs) % 3]
        ref = alpha * ((A.T if ta else A) @ (B.T if tb else B)) + beta * C
        dA, dB, dC = dev(A), dev(B), dev(C)
        probs.append(dict(M=M, N=N, K=K, A=dA, lda=max(1, A.shape[0]), B=dB, ldb=max(1, B.shape[0]),
                          C=dC, ldc=M, alpha=alpha, beta=beta))
        refs.append(ref)
        outs.append((dC, M, N, np.abs(A).max(initial=0) * np.abs(B).max(initial=0) * K))
    tlr.gemm_batched(bool(ta), bool(tb), probs)
    for ref, (dC, M, N, scale) in zip(refs, outs):
        got = host(dC, M, N)
        tol = 4 * (outs[0][1] + 64) * U64 * (scale + np.abs(ref).max() + 1)
        np.testing.assert_allclose(got, ref, rtol=0, atol=tol)


def test_gemm_tn_streamed_ragged():
    """Transposed-A batches whose problems all have an even K (and so even
    leading dimensions) run on the LDS-streamed kernel: ragged M, N, K around
    its 16 / 64-wide tiles and 64-row chunks, N past 32, beta 0 / 1 / -0.5."""
    rng = np.random.default_rng(77)
    sizes = [(1, 1, 2), (3, 17, 6), (16, 16, 64), (12, 12, 1024), (65, 15, 4), (130, 70, 34),
             (64, 33, 130), (200, 16, 300), (16, 64, 2), (1, 300, 2), (400, 16, 1024),
             (17, 5, 66)]
    probs, refs, outs = [], [], []
    for (M, N, K) in sizes:
        A = rng.standard_normal((K, M))
        B = rng.standard_normal((K, N))
        C = rng.standard_normal((M, N))
        alpha, beta = rng.uniform(-2, 2), [0.0, 1.0, -0.5][len(probs) % 3]
        ref = alpha * (A.T @ B) + beta * C
        dA, dB, dC = dev(A), dev(B), dev(C)
        probs.append(dict(M=M, N=N, K=K, A=dA, lda=K, B=dB, ldb=K, C=dC, ldc=M, alpha=alpha,
                          beta=beta))
        refs.append(ref)
        outs.append((dC, M, N, np.abs(A).max() * np.abs(B).max() * K))
    tlr.gemm_batched(True, False, probs)
    for ref, (dC, M, N, scale) in zip(refs, outs):
        got = host(dC, M, N)
        tol = 4 * (M + 64) * U64 * (scale + np.abs(ref).max() + 1)
        np.testing.assert_allclose(got, ref, rtol=0, atol=tol)


@pytest.mark.parametrize("m", [1, 7, 32, 33, 64, 65, 97, 200, 256, 513, 1024])
def test_potrf_tile_matches_lapack(m):
    g = _rand((m, m), m)
    a = g @ g.T / m + np.eye(m)
    d = dev(a)
    assert tlr.potrf_tile(d) == 0
    L = host(d, m, m)
    ref = np.linalg.cholesky(a)
    np.testing.assert_allclose(L, ref, rtol=0, atol=64 * m * U64 * np.abs(ref).max())
    assert not np.triu(L, 1).any()


def test_potrf_tile_reports_first_bad_pivot():
    m = 100
    g = _rand((m, m), 1)
    a = g @ g.T / m + np.eye(m)
    a[70, 70] = -1.0
    d = dev(a)
    assert tlr.potrf_tile(d) == 71


@pytest.mark.parametrize("m", [3, 64, 150, 320])
def test_ldlt_tile_matches_oracle(m):
    rng = np.random.default_rng(m)
    sgn = np.where(rng.random(m) < 0.4, -1.0, 1.0)
    a = np.diag(sgn * rng.uniform(4, 6, m)) + 0.1 * rng.standard_normal((m, m))
    a = 0.5 * (a + a.T)
    lref, dref = dense.ldlt_unpivoted(a)
    import torch
    da = dev(a)
    dd = torch.zeros(m, dtype=torch.float64, device="cuda")
    assert tlr.ldlt_tile(da, dd) == 0
    L = host(da, m, m)
    np.testing.assert_allclose(L, lref, rtol=0, atol=1e3 * m * U64)
    np.testing.assert_allclose(dd.cpu().numpy(), dref, rtol=1e3 * m * U64)


def test_ldlt_tile_zero_pivot():
    a = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    import torch
    da = dev(a)
    dd = torch.zeros(3, dtype=torch.float64, device="cuda")
    assert tlr.ldlt_tile(da, dd) == 2


@pytest.mark.parametrize("unit,trans", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("m,n", [(5, 3), (128, 17), (300, 70)])
def test_trsm_matches_lapack(unit, trans, m, n):
    rng = np.random.default_rng(m + n + 2 * unit + trans)
    L = np.tril(rng.standard_normal((m, m))) / math.sqrt(m) + np.eye(m) * 2
    B = rng.standard_normal((m, n))
    ref = dense.solve_lower(L, B, unit=bool(unit), trans=bool(trans))
    dL, dB = dev(L), dev(B)
    tlr.trsm(m, n, dL, dB, unit=bool(unit), trans=bool(trans))
    got = host(dB, m, n)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e3 * m * U64 * (np.abs(ref).max() + 1))


def test_philox_bit_exact():
    n = 1000
    got = tlr.philox(n, 0x123456789ABCDEF, 7, 8, 9).reshape(n, 4)
    for c in (0, 1, 2, 511, 999):
        ref = oph.philox4x32_10((c, 7, 8, 9), (0x89ABCDEF, 0x01234567))
        assert tuple(int(x) for x in got[c]) == ref


def test_randn_matches_reference_stream():
    rows, cols = 257, 16
    got = tlr.randn(rows, cols, 42, 5, 3, 0)
    ref = oph.test_matrix(42, 5, 3, 0, rows, cols)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def _lowrank_tile(m, r, seed, decay=None):
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng.standard_normal((m, max(r, 1))))
    v, _ = np.linalg.qr(rng.standard_normal((m, max(r, 1))))
    s = np.ones(r) if decay is None else decay ** np.arange(r)
    return (u[:, :r] * s) @ v[:, :r].T


@pytest.mark.parametrize("m,r", [(64, 0), (64, 1), (64, 5), (128, 16), (128, 17), (256, 40)])
def test_ara_recovers_exact_rank(m, r):
    import torch
    tile = 3.0 * _lowrank_tile(m, r, r + m) if r else np.zeros((m, m))
    tiles = torch.stack([dev(tile)]).reshape(1, m, m)
    Q, B, ranks, iters = tlr.ara(tiles, 1e-9, bs=16)
    assert ranks[0] == r
    q = host(Q[0].reshape(-1), m, m)[:, :r]
    b = host(B[0].reshape(-1), m, m)[:, :r]
    np.testing.assert_allclose(q.T @ q, np.eye(r), atol=1e-12)
    assert np.linalg.norm(tile - q @ b.T, 2) < 1e-10


def test_ara_threshold_and_eckart_young():
    import torch
    m, count, tau = 256, 24, 1e-6
    mats = []
    for t in range(count):
        base = _lowrank_tile(m, 60, 100 + t, decay=0.6 + 0.01 * t) * (10.0 ** (t % 4))
        mats.append(base)
    tiles = torch.stack([dev(a).reshape(m, m) for a in mats])
    Q, B, ranks, iters = tlr.ara(tiles, tau, bs=16, seed=7)
    over = 0
    for t in range(count):
        q = host(Q[t].reshape(-1), m, m)[:, :ranks[t]]
        b = host(B[t].reshape(-1), m, m)[:, :ranks[t]]
        err = np.linalg.norm(mats[t] - q @ b.T, 2)
        s = np.linalg.svd(mats[t], compute_uv=False)
        # Eckart-Young: no rank-q approximation beats sigma_{q+1}
        assert ranks[t] >= int(np.sum(s > err * (1 + 1e-9)))
        assert err <= 4 * tau
        over += err > tau
        # ranks stay close to the optimal ones
        assert ranks[t] <= int(np.sum(s > tau)) + 16
        np.testing.assert_allclose(q.T @ q, np.eye(ranks[t]), atol=1e-11)
    assert over <= 2


def test_ara_wide_launch_matches_narrow_launches():
    """A launch with enough active tiles samples on 64-row strips, narrower
    ones on 16-row strips; the accumulation order is the same, so a tile's
    basis and projection do not depend on how many tiles share its
    launches.  m = 80 leaves a ragged last strip block."""
    import torch
    m, count, tau = 80, 300, 1e-9
    mats = [3.0 * _lowrank_tile(m, t % 23, 500 + t) if t % 23 else np.zeros((m, m))
            for t in range(count)]
    tiles = torch.stack([dev(a).reshape(m, m) for a in mats])
    Q, B, ranks, iters = tlr.ara(tiles, tau, bs=16, seed=11)
    for lo in range(0, count, 100):
        q2, b2, r2, it2 = tlr.ara(tiles[lo:lo + 100].contiguous(), tau, bs=16, seed=11)
        assert list(r2) == list(ranks[lo:lo + 100])
        assert list(it2) == list(iters[lo:lo + 100])
        assert torch.equal(q2.cpu(), Q[lo:lo + 100].cpu())
        assert torch.equal(b2.cpu(), B[lo:lo + 100].cpu())
    for t in range(count):
        r = t % 23
        assert ranks[t] == r
        q = host(Q[t].reshape(-1), m, m)[:, :r]
        b = host(B[t].reshape(-1), m, m)[:, :r]
        assert np.linalg.norm(mats[t] - q @ b.T, 2) < 1e-10


def test_sort_ranks_bit_exact():
    rng = np.random.default_rng(3)
    for n in (1, 5, 127, 300):
        ranks = rng.integers(0, 6, n)
        rows = np.arange(n) + 11
        a = np.zeros((n + 11, n + 11), dtype=int)
        a[rows, 10] = ranks
        ref = bk.sort_ranks(a, 10)
        got = tlr.sort_ranks(ranks, rows)
        assert got.tolist() == ref


def test_compaction_bit_exact_against_active_set_evolution():
    rng = np.random.default_rng(5)
    for trial in range(40):
        n = int(rng.integers(1, 300))
        s_max = int(rng.integers(1, n + 1))
        order = rng.permutation(n).tolist()
        active = order[:s_max]
        waiting = order[s_max:]
        cursor = 0
        flags_seq = []
        flags_by_slot = np.zeros(n, dtype=np.int32)
        while active:
            f = (rng.random(len(active)) < 0.4).tolist()
            flags_seq.append(f)
            for slot, c in zip(active, f):
                flags_by_slot[slot] = int(c)
            active, cursor = tlr.compact(n, active, flags_by_slot, waiting, cursor, s_max)
            for slot in active:
                flags_by_slot[slot] = 0
            ref = bk.active_sets(order, s_max, flags_seq)[-1]
            assert active == ref
