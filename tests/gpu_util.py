"""Helpers shared by the GPU tests: column-major transfers between numpy and
torch device tensors, and conversion of library handles into oracle TLR
objects (host copies of the GPU's results, compared against the oracle)."""
import numpy as np

# Total factor rank against the oracle's truncated-SVD ranks at the same
# threshold.  The ARA accepts a direction while a sample residual exceeds
# tau; a random sample's residual measures the Frobenius norm of what is
# left, so directions keep being added until the tail's Frobenius norm (not
# its 2-norm) is below tau, and tiles whose spectrum has many singular
# values just below tau end with more columns than the 2-norm-optimal SVD
# truncation: 18-29 % more on the covariance workloads (measured, half-block
# convergence rule).
RANK_RATIO = 1.35


def dev(a):
    """Column-major device copy (flat float64 torch tensor) of a 1-D/2-D array."""
    import torch
    a = np.asarray(a, dtype=np.float64)
    flat = a.ravel(order="F") if a.ndim == 2 else a
    return torch.from_numpy(np.ascontiguousarray(flat)).cuda()


def host(t, rows, cols):
    """rows x cols numpy array from a flat column-major device tensor."""
    return t.detach().cpu().numpy()[:rows * cols].reshape(cols, rows).T.copy()


def oracle_tlr(mat, which):
    """An oracle.tlr.TLR holding a copy of the handle's input or factor."""
    from oracle import tlr as otlr
    diag, u, v, _ = mat.to_host(which)
    t = otlr.TLR(mat.n, mat.m)
    t.diag = [np.array(d) for d in diag]
    t.u = {k: np.array(x) for k, x in u.items()}
    t.v = {k: np.array(x) for k, x in v.items()}
    return t


def tile_errors(a, l, d=None):
    """2-norms of the tiles of A - L L^T (or A - L D L^T) for the TLR input a
    and the factor l (oracle.tlr.TLR objects), computed tile by tile from the
    low rank factors (no dense N x N expansion).

    Returns (off, diag): off[(i, k)] for i > k, diag[k] for the diagonal tiles.
    By the left-looking identity, off[(i, k)] is the compression error of the
    Schur-complement tile S_ik."""
    nb, m = a.nb, a.m
    dv = [np.asarray(x) for x in d] if d is not None else None

    def lfull(i, j):
        # L_ij as (left, right) with L_ij = left @ right.T
        if i == j:
            return np.tril(l.diag[i]), np.eye(m)
        return l.u[i, j], l.v[i, j]

    off, diag = {}, {}
    for k in range(nb):
        for i in range(k, nb):
            e = a.tile(i, k).copy()
            for j in range(k + 1):
                li, ri = lfull(i, j)
                lk, rk = lfull(k, j)
                if li.shape[1] == 0 or lk.shape[1] == 0:
                    continue
                mid = ri.T @ ((dv[j][:, None] * rk) if dv is not None else rk)
                e -= li @ (mid @ lk.T)
            nrm = float(np.linalg.norm(e, 2))
            if i == k:
                diag[k] = nrm
            else:
                off[i, k] = nrm
    return off, diag
