"""TLR-preconditioned conjugate gradients (the factorization used as a
preconditioner, Section 6) against a textbook PCG on the host with the same
operator and preconditioner (the oracle's TLR product and solve applied to
the GPU's own input and factor, downloaded), and against the dense solve."""
import numpy as np
import pytest

from oracle import dense
from oracle import tlr as otlr
from paper_2108_11932_amd import tlr
from paper_2108_11932_amd import workloads as wl

from gpu_util import oracle_tlr

pytestmark = pytest.mark.gpu


def _host_pcg(apply_a, apply_m, b, rtol, maxit):
    """Plain preconditioned CG (x0 = 0), the iteration count at which the
    recurrence residual first drops to rtol ||b||."""
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_m(r)
    p = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    for it in range(1, maxit + 1):
        q = apply_a(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= rtol * nb:
            return x, it
        z = apply_m(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit


def test_pcg_with_tlr_preconditioners():
    # ill-conditioned 2D exponential covariance (nugget 1e-6): the operator
    # compressed at 1e-10, preconditioners factored at looser thresholds
    # (with the shift s = tau where definiteness is lost)
    n, m = 2048, 256
    pts = wl.jittered_grid(n, 2, 77)
    pts = np.ascontiguousarray(pts[wl.morton_order(pts)])
    a_dense = dense.covariance_matrix(pts, dense.KERNEL_EXP, 0.1, 1e-6)
    op = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-6, m, 1e-10)
    a_t = oracle_tlr(op, tlr.INPUT)
    import torch
    b = np.random.default_rng(8).standard_normal(n)
    bd = torch.from_numpy(b).cuda()
    rtol = 1e-8
    iters = {}
    for eps in (1e-2, 1e-4, 1e-6):
        f = tlr.TLRMatrix.compress_kernel(pts, tlr.KERNEL_EXP, 0.1, 1e-6, m, eps)
        f.potrf(eps, tlr.opts(auto_shift=1))
        x, it, rel = op.pcg(bd, f, rtol=rtol, maxit=500)
        assert rel <= rtol and it < 500
        xh = x.cpu().numpy()
        # the true residual against the dense matrix
        true = np.linalg.norm(b - a_dense @ xh) / np.linalg.norm(b)
        assert true <= 1e-6, (eps, true)
        # the same PCG on the host with the same operator and factor
        l = oracle_tlr(f, tlr.FACTOR)
        _, it_h = _host_pcg(lambda v: otlr.matvec(a_t, v), lambda v: otlr.solve(l, v), b, rtol, 500)
        assert abs(it - it_h) <= 1, (eps, it, it_h)
        iters[eps] = it
        f.close()
    # tighter preconditioners take fewer iterations
    assert iters[1e-6] <= iters[1e-4] <= iters[1e-2]
    # without a preconditioner CG needs far more
    _, it0, _ = op.pcg(bd, None, rtol=rtol, maxit=300)
    assert it0 >= 5 * iters[1e-2]
    # a zero right-hand side needs no iteration
    x, it, rel = op.pcg(torch.zeros_like(bd), None, rtol=rtol)
    assert it == 0 and float(x.abs().max()) == 0.0
    op.close()
