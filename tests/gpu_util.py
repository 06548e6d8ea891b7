"""Helpers shared by the GPU tests: column-major transfers between numpy and
torch device tensors, and conversion of library handles into oracle TLR
objects (host copies of the GPU's results, compared against the oracle)."""
import numpy as np


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
