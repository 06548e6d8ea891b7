"""Write tests/golden/cfg2_ranks.txt: the ranks the oracle reaches on the
2D covariance workload with N = 32768 points, tile 512, at absolute eps 1e-2
and 1e-6.

The oracle compresses the covariance matrix tile by tile by truncated SVD
(O3) and factors it with the left-looking TLR Cholesky whose recompression
of every Schur-complement tile is an exact truncated SVD (O4).  Only
`oracle/` and the seeded point generator are used.  Takes several minutes
on 8 cores:

    python tests/golden/make_cfg2_ranks.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import dense  # noqa: E402
from oracle import tlr as otlr  # noqa: E402
from paper_2108_11932_amd import workloads as wl  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg2_ranks.txt")


def main():
    w = wl.standard("cov2d_32k")
    lines = ["# oracle ranks of the 2D exponential covariance, N=%d, tile %d, ell %g, nugget %g,"
             % (w.n, w.m, w.ell, w.diag_add),
             "# jittered 256x128 grid (seed %d), Morton order; written by make_cfg2_ranks.py" % w.seed,
             "# eps input_rank_sum factor_rank_sum factor_rank_max factor_rank_mean seconds"]
    for eps in (1e-2, 1e-6):
        t0 = time.perf_counter()
        a = otlr.compress_kernel(w.points, w.m, dense.KERNEL_EXP, w.ell, w.diag_add, eps)
        l = otlr.tlr_cholesky(a, eps)
        dt = time.perf_counter() - t0
        ri = a.ranks()[np.tril_indices(a.nb, -1)]
        rl = l.ranks()[np.tril_indices(a.nb, -1)]
        lines.append("%g %d %d %d %.4f %.0f" % (eps, ri.sum(), rl.sum(), rl.max(), rl.mean(), dt))
        print(lines[-1], flush=True)
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
