#!/usr/bin/env python3
"""Benchmark of the TLR Cholesky hot path on one MI355X.

One step is one complete left-looking TLR Cholesky (tlr_potrf: every column's
dense diagonal update and POTRF, batched ARA of the Schur-complement tiles
with dynamic batching, projection, triangular solve and panel append) of a
covariance matrix that is already resident in HBM in TLR form.  The input is
built on the GPU (tlr_compress_kernel) before the timed region.

Prints one JSON line: time-to-solution (ms_per_step) and the executed TFLOP/s
(value), the roofline of the dominant kernel (the Schur-complement sampling
product, timed live with HIP events), and the FP64 CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload cov2d_131k] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
# measured HBM traffic of the sampling kernel (rocprofv3 FETCH_SIZE and
# WRITE_SIZE, calibrated on a plain copy); valid only for the sources it was
# measured on: the sampling kernels and the engine that schedules them
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sampling_traffic_cov2d_131k.txt")
KERNEL_SOURCES = ["paper_2108_11932_amd/csrc/ara_iter.hip", "paper_2108_11932_amd/csrc/ara_orth.h",
                  "paper_2108_11932_amd/csrc/dd.h", "paper_2108_11932_amd/csrc/mfma_tiles.h",
                  "paper_2108_11932_amd/csrc/tlr_internal.h",
                  "paper_2108_11932_amd/csrc/ara_engine.cpp"]
# per-kernel roofline table of the headline factorization (time share, FP64
# matrix-core and HBM fractions from rocprofv3 counters); valid for the
# library sources it was measured on
TABLE_FILE = os.path.join(ROOT, "profiles", "roofline_table_cov2d_131k.txt")
CSRC = os.path.join(ROOT, "paper_2108_11932_amd", "csrc")


def _sha256(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in paths:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_source_hash() -> str:
    return _sha256(os.path.join(ROOT, f) for f in KERNEL_SOURCES)


def library_source_hash() -> str:
    return _sha256(os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)))


def _key_values(path):
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#") and "|" not in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def measured_traffic(workload: str):
    """HBM bytes per launch of the sampling kernel from the committed counter
    summary, or None when it is absent, for another workload, or taken on
    other kernel sources."""
    try:
        kv = _key_values(TRAFFIC_FILE)
        if kv.get("workload") != workload or kv.get("source_sha256") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def kernel_table(workload: str, top: int = 14):
    """The leading rows of the committed per-kernel roofline table (share of
    GPU time, FP64 matrix-core and HBM fractions, bound), and whether it was
    measured on the library sources of this tree."""
    try:
        kv = _key_values(TABLE_FILE)
        if kv.get("workload") != workload:
            return None
        rows, head = [], None
        with open(TABLE_FILE) as fh:
            for line in fh:
                if "|" not in line or line.startswith("#"):
                    continue
                cells = [c.strip() for c in line.split("|")]
                if head is None:
                    head = cells
                    continue
                r = dict(zip(head, cells))
                rows.append({"kernel": r["kernel"], "calls": int(r["calls"]),
                             "share": float(r["share"]), "avg_us": float(r["time_us"]) / int(r["calls"]),
                             "mfma_f64_tflops": float(r["mfma_f64_tflops"]),
                             "frac_mfma_f64": float(r["frac_mfma_f64"]),
                             "hbm_gbs": float(r["hbm_gbs"]), "frac_hbm": float(r["frac_hbm"]),
                             "bound": r["bound"]})
        return {"source": os.path.relpath(TABLE_FILE, ROOT),
                "measured_on_these_sources": kv.get("source_sha256") == library_source_hash(),
                "rows": rows[:top]}
    except (OSError, KeyError, ValueError):
        return None


METRIC = "TLR Cholesky time-to-solution + TFLOP/s, N=131072 eps=1e-6; FP64 vs mixed"


def _describe(w) -> str:
    kern = {0: "exponential", 1: "Matern-1.5"}[w.kernel]
    return ("%dD %s covariance (ell %g, diagonal %+g), N=%d jittered-grid points in Morton order, "
            "tile %d, eps %g %s, ARA block %d" % (w.dim, kern, w.ell, w.diag_add, w.n, w.m, w.eps,
                                                  "absolute" if w.eps_mode == 0 else "relative",
                                                  w.bs))


def cpu_baseline(w, n_sample: int, tlr, torch):
    """Time the FP64 oracle (left-looking TLR Cholesky with exact SVD
    recompression) on the leading n_sample x n_sample principal block of the
    same covariance matrix, and express it in the metric's unit: the
    executed-flop count of the GPU algorithm on that same block divided by the
    oracle's time."""
    from oracle import dense as odense
    from oracle import tlr as otlr
    try:
        from threadpoolctl import threadpool_info
        blas = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        cores = max((d.get("num_threads", 1) for d in blas), default=os.cpu_count())
        vendor = ", ".join("%s %s (%s)" % (d.get("internal_api"), d.get("version"),
                                           d.get("threading_layer")) for d in blas) or "unknown"
    except Exception:  # pragma: no cover
        cores, vendor = os.cpu_count(), "unknown"
    pts = np.ascontiguousarray(w.points[:n_sample])
    a_s = otlr.compress_kernel(pts, w.m, w.kernel, w.ell, w.diag_add, w.eps)
    t0 = time.perf_counter()
    otlr.tlr_cholesky(a_s, w.eps)
    t_cpu = time.perf_counter() - t0
    g = tlr.TLRMatrix.from_tlr(a_s.n, a_s.m, a_s.diag, a_s.u, a_s.v)
    o = tlr.opts(bs=w.bs, eps_mode=0)
    g.potrf(w.eps, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.potrf(w.eps, o)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    g.close()
    return {"value": st["flops"] / t_cpu / 1e12, "unit": "TFLOP/s", "cores": int(cores),
            "kind": "oracle",
            "sample": "leading %dx%d principal block (%d tiles of %d) of the same matrix; oracle = "
                      "left-looking TLR Cholesky with truncated-SVD recompression (numpy/LAPACK "
                      "FP64); work = the GPU algorithm's executed flops on that block (%.3g)"
                      % (n_sample, n_sample, a_s.nb, w.m, st["flops"]),
            "blas": vendor, "oracle_seconds": t_cpu, "gpu_seconds_same_sample": t_gpu}


def residual(mat, torch, nvec: int = 4, seed: int = 7, shift: float = 0.0) -> float:
    """Random-vector residual of the factor against the FP64 TLR input:
    max over Gaussian b of ||(A + shift I) x - b|| / ||x|| with
    x = (L L^T)^{-1} b, i.e. ||(A + shift I - L L^T) x|| / ||x|| (shift: the
    diagonal shift the factorization applied); A is applied by tlr_matvec
    (FP64), x by tlr_solve with the factor."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    b = torch.randn(mat.n, nvec, generator=g, dtype=torch.float64).cuda()
    x = mat.solve(b)
    r = mat.matvec(x) + shift * x - b
    return float((r.norm(dim=0) / x.norm(dim=0)).max())


def time_form(mat, w, eps_mode, precision, tlr, torch, steps, warmup, bs_tail=0, tail_active=0,
              timing=True, idle_s=0.0, serial=False, eps=None, shift=0.0):
    """Warm up, then time `steps` factorizations of one form (with the
    sampling launches timed by their own events when `timing`, which runs
    every sampling product in a launch of its own); the GPU idles idle_s
    seconds between the warm-up and the timed steps (a marker for profile
    reductions).  `serial` asks for that same launch schedule without the
    events (for counter runs that match the timed launches).  eps (default:
    the workload's) and shift (< 0: the shift tau of Section 5.1) select
    the form's threshold."""
    eps = w.eps if eps is None else eps
    o = tlr.opts(bs=w.bs, bs_tail=bs_tail, tail_active=tail_active, eps_mode=eps_mode,
                 precision=precision, shift=shift,
                 flags=(tlr.FLAG_KERNEL_TIMING if timing else 0) |
                       (tlr.FLAG_SERIAL_SAMPLING if serial else 0))
    for _ in range(warmup):
        mat.potrf(eps, o)
    torch.cuda.synchronize()
    if idle_s > 0:
        time.sleep(idle_s)
    t0 = time.perf_counter()
    stats = [mat.potrf(eps, o) for _ in range(steps)]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, stats


def phase_split(mat, w, tlr, torch):
    """One factorization with the phase timers on (HIP events at the phase
    boundaries of every column): GPU milliseconds per phase.  The phases of
    the caller's stream run one after another and add up to that stream's
    span; 'diag' (updateDense, chol and the next column's G blocks) runs on
    the second stream beside them."""
    o = tlr.opts(bs=w.bs, eps_mode=w.eps_mode, flags=tlr.FLAG_PHASE_TIMING)
    mat.potrf(w.eps, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = mat.potrf(w.eps, o)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    ph = dict(zip(tlr.PHASES, st["t_phase"]))
    main = sum(v for k, v in ph.items() if k != "diag")
    return {"ms": ph, "main_stream_sum_ms": main, "pass_ms": wall,
            "note": "phases other than diag run in sequence on the caller's stream; diag runs "
                    "on the second stream, overlapped"}


def pivoted_form(tlr, torch, wl, steps: int):
    """The 3D exponential covariance (N=131072, tile 512, eps 1e-6 absolute,
    ARA block 32) factored unpivoted and with the Frobenius-norm tile
    pivoting of Section 5.2: time, ranks and random-vector residual of
    each."""
    w = wl.standard("cov3d_131k")
    mat = tlr.TLRMatrix.compress_kernel(w.points, w.kernel, w.ell, w.diag_add, w.m, w.eps,
                                        tlr.opts(bs=w.bs))
    o = tlr.opts(bs=w.bs)
    out = {"workload": _describe(w), "N": w.n, "tile": w.m, "eps": w.eps, "bs": w.bs}
    for name in ("unpivoted", "pivoted"):
        run = (lambda: mat.potrf(w.eps, o)) if name == "unpivoted" else \
            (lambda: mat.potrf_pivoted(w.eps, o)[0])
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [run() for _ in range(steps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        rl = mat.ranks(tlr.FACTOR)[np.tril_indices(mat.nb, -1)]
        out[name] = {"ms_per_step": dt * 1e3, "tflops": sts[-1]["flops"] / dt / 1e12,
                     "residual": residual(mat, torch), "rank_mean": float(rl.mean()),
                     "rank_max": int(rl.max()), "rank_total": int(rl.sum()),
                     "ara_iterations": int(sts[-1]["ara_iters"])}
    mat.close()
    return out


def pcg_form(tlr, torch, wl):
    """TLR factorizations as preconditioners (Section 6): the N=32768 2D
    exponential covariance with nugget 1e-6 as the operator (compressed at
    1e-9), preconditioned CG to a relative residual of 1e-8 with the TLR
    Cholesky at eps 1e-2, 1e-4 and 1e-6 (shift tau where definiteness is
    lost), and without a preconditioner."""
    base = wl.standard("cov2d_32k")
    pts = base.points
    op = tlr.TLRMatrix.compress_kernel(pts, base.kernel, base.ell, 1e-6, base.m, 1e-9,
                                       tlr.opts(bs=base.bs))
    g = torch.Generator(device="cpu").manual_seed(9)
    b = torch.randn(op.n, generator=g, dtype=torch.float64).cuda()
    out = {"workload": "2D exponential covariance (ell 0.1, diagonal +1e-6), N=%d, tile %d; "
                       "operator eps 1e-9" % (op.n, base.m), "rtol": 1e-8}
    for eps in (1e-2, 1e-4, 1e-6):
        f = tlr.TLRMatrix.compress_kernel(pts, base.kernel, base.ell, 1e-6, base.m, eps,
                                          tlr.opts(bs=base.bs))
        o = tlr.opts(bs=base.bs, auto_shift=1)
        f.potrf(eps, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = f.potrf(eps, o)
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, it, rel = op.pcg(b, f, rtol=1e-8, maxit=2000)
        torch.cuda.synchronize()
        t_s = time.perf_counter() - t0
        out["eps_%g" % eps] = {"factor_ms": t_f * 1e3, "pcg_ms": t_s * 1e3, "iterations": it,
                               "relres": rel, "shift": st["shift"], "rank_mean": st["mean_rank"]}
        f.close()
    t0 = time.perf_counter()
    _, it, rel = op.pcg(b, None, rtol=1e-8, maxit=2000)
    torch.cuda.synchronize()
    out["none"] = {"pcg_ms": (time.perf_counter() - t0) * 1e3, "iterations": it, "relres": rel}
    op.close()
    return out


def recompress_form(mat, w, tlr, torch, o, reps: int = 2):
    """SVD post-recompression of the headline factor (Section 6.2): the
    factor's low rank tiles cut to their minimal ranks at the
    factorization's own threshold.  Per repetition: factor (untimed), time
    the solve with one right-hand side (median of 5), time tlr_recompress,
    time the solve again.  Reports the factor's memory (diagonal tiles plus
    U and V panels) before and after, the times, and the random-vector
    residual of the recompressed factor against its bound."""
    def solve_ms():
        g = torch.Generator(device="cpu").manual_seed(5)
        b = torch.randn(mat.n, generator=g, dtype=torch.float64).cuda()
        mat.solve(b)
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mat.solve(b)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ts))

    def mem(r):
        return 8.0 * (mat.nb * mat.m * mat.m + 2 * mat.m * int(r.sum()))

    runs = []
    for _ in range(reps):
        st = mat.potrf(w.eps, o)
        r0 = mat.ranks(tlr.FACTOR)
        s0 = solve_ms()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mat.recompress(st["tau"])
        torch.cuda.synchronize()
        t_rc = (time.perf_counter() - t0) * 1e3
        r1 = mat.ranks(tlr.FACTOR)
        runs.append({"recompress_ms": t_rc, "solve_ms_before": s0, "solve_ms_after": solve_ms(),
                     "rank_sum_before": int(r0.sum()), "rank_sum_after": int(r1.sum()),
                     "tau": st["tau"]})
    last = runs[-1]
    err = residual(mat, torch)
    bound = 2.0 * math.sqrt(mat.nb) * last["tau"]
    return {"workload": _describe(w) + ", the FP64 factor at the factorization's tau",
            "recompress_ms": min(x["recompress_ms"] for x in runs),
            "recompress_ms_runs": [x["recompress_ms"] for x in runs],
            "rank_sum_before": last["rank_sum_before"], "rank_sum_after": last["rank_sum_after"],
            "lowrank_rank_reduction": 1.0 - last["rank_sum_after"] / max(1, last["rank_sum_before"]),
            "factor_bytes_before": mem(np.array([last["rank_sum_before"]])),
            "factor_bytes_after": mem(np.array([last["rank_sum_after"]])),
            "solve_ms_before": last["solve_ms_before"], "solve_ms_after": last["solve_ms_after"],
            "residual_after": err, "residual_bound": bound,
            "residual_within_bound": bool(err <= bound)}


def schur_form(tlr, torch, wl):
    """Schur compensation (Section 5.1.1) on the N=32768 tile-512 2D
    covariance: the factorization at eps 1e-6 absolute with and without
    TLR_FLAG_SCHUR_COMP (time, residual against the unshifted input), and
    at a relative 1e-2 without a shift, where the plain factorization loses
    definiteness: the first failing row with and without the compensation."""
    w = wl.standard("cov2d_32k")
    mat = tlr.TLRMatrix.compress_kernel(w.points, w.kernel, w.ell, w.diag_add, w.m, w.eps,
                                        tlr.opts(bs=w.bs))
    out = {"workload": _describe(w)}
    for name, fl in (("plain", 0), ("schur", tlr.FLAG_SCHUR_COMP)):
        o = tlr.opts(bs=w.bs, flags=fl)
        mat.potrf(w.eps, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = mat.potrf(w.eps, o)
        torch.cuda.synchronize()
        out[name] = {"ms": (time.perf_counter() - t0) * 1e3, "residual": residual(mat, torch),
                     "bound": 2.0 * math.sqrt(mat.nb) * st["tau"]}
        s_rel, st_rel = mat.potrf_status(1e-2, tlr.opts(bs=w.bs, eps_mode=tlr.EPS_REL, flags=fl))
        out[name]["rel_1e-2_status"] = int(s_rel)
        out[name]["rel_1e-2_failing_row"] = int(st_rel["info"])
    mat.close()
    return out


def batched_form(tlr, torch, wl, count: int, m_fixed: int):
    """The batched workload (count independent 2D problems of uneven N,
    relative eps 1e-6).  Tile sizes come from the library's autotuner
    (tlr_tune_tile over 256 / 512 / 1024, one measurement per problem class
    of ceil(log2 N)); the problems are then factored by one batched call
    (FP64 and FP32-sampling) against the same problems factored one by one,
    and against one batched call at the fixed tile size m_fixed."""
    ws = wl.batched_2d(count=count, m=m_fixed)
    o_c = tlr.opts(bs=ws[0].bs, eps_mode=tlr.EPS_REL)
    o64 = tlr.opts(bs=ws[0].bs, eps_mode=tlr.EPS_REL, precision=tlr.FP64)
    o32 = tlr.opts(bs=ws[0].bs, eps_mode=tlr.EPS_REL, precision=tlr.MIXED_FP32)
    tlr.lib().tlr_tune_reset()
    t0 = time.perf_counter()
    tiles, measured = [], {}
    for w in ws:
        best, ms = tlr.tune_tile(w.points, w.kernel, w.ell, w.diag_add, w.eps, (256, 512, 1024), o64)
        tiles.append(best)
        if ms is not None:
            measured["N=%d" % w.n] = {str(k): v for k, v in ms.items()}
    t_tune = time.perf_counter() - t0

    def build(ms_):
        return [tlr.TLRMatrix.compress_kernel(w.points, w.kernel, w.ell, w.diag_add, mm, w.eps, o_c)
                for w, mm in zip(ws, ms_)]

    def timed(f):
        f()   # warm-up (workspaces, code objects)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = f()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    def bat(mats, o):
        def run():
            s, sts, _ = tlr.factor_batched(mats, ws[0].eps, o)
            if s != 0:
                raise RuntimeError("batched factorization failed: %d" % s)
            return sts
        return run

    fixed = build([m_fixed] * len(ws))
    t_fixed, _ = timed(bat(fixed, o64))
    for mt in fixed:
        mt.close()
    mats = build(tiles)
    t_seq, _ = timed(lambda: [mt.potrf(ws[0].eps, o64) for mt in mats])
    t_b64, st_b64 = timed(bat(mats, o64))
    t_b32, st_b32 = timed(bat(mats, o32))
    flops = sum(x["flops"] for x in st_b64)
    ns = [w.n for w in ws]
    for mt in mats:
        mt.close()
    choice = {str(mm): tiles.count(mm) for mm in sorted(set(tiles))}
    return {"count": count, "tiles_tuned": choice, "tuning_s": t_tune, "tuning_measured": measured,
            "N_min": min(ns), "N_max": max(ns), "N_total": sum(ns),
            "eps": ws[0].eps, "eps_mode": "relative",
            "sequential_fp64_s": t_seq, "batched_fp64_s": t_b64, "batched_mixed_fp32_s": t_b32,
            "batched_fp64_fixed_tile_s": t_fixed, "fixed_tile": m_fixed,
            "speedup_fp64": t_seq / t_b64, "speedup_mixed": t_seq / t_b32,
            "tuned_over_fixed": t_fixed / t_b64,
            "batched_fp64_tflops": flops / t_b64 / 1e12}


GOLDEN_CFG2 = os.path.join(ROOT, "tests", "golden", "cfg2_ranks.txt")


def cov2d_32k_form(tlr, torch, wl, steps: int):
    """The N = 32768 2D covariance at tile 512, absolute eps 1e-2 and 1e-6:
    time-to-solution, the random-vector residual against the bound
    2 sqrt(nb) tau, and the factor's total rank against the oracle's (O4,
    truncated-SVD recompression, from the committed golden file)."""
    gold = {}
    try:
        with open(GOLDEN_CFG2) as fh:
            for ln in fh:
                if ln.strip() and not ln.startswith("#"):
                    f = ln.split()
                    gold[float(f[0])] = int(f[2])
    except OSError:
        pass
    out = {}
    base = wl.standard("cov2d_32k")
    mat = None
    for eps in (1e-2, 1e-6):
        if mat is not None:
            mat.close()
        mat = tlr.TLRMatrix.compress_kernel(base.points, base.kernel, base.ell, base.diag_add,
                                            base.m, eps, tlr.opts(bs=base.bs))
        o = tlr.opts(bs=base.bs)
        mat.potrf(eps, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [mat.potrf(eps, o) for _ in range(steps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res = residual(mat, torch)
        bound = 2.0 * math.sqrt(mat.nb) * eps
        rl = mat.ranks(tlr.FACTOR)[np.tril_indices(mat.nb, -1)]
        out["eps_%g" % eps] = {
            "ms_per_step": dt * 1e3, "tflops": float(np.mean([s["flops"] for s in sts])) / dt / 1e12,
            "residual": res, "bound": bound, "within_bound": bool(res <= bound),
            "rank_total": int(rl.sum()), "rank_max": int(rl.max()), "rank_mean": float(rl.mean()),
            "rank_total_oracle": gold.get(eps), "ara_iterations": int(sts[-1]["ara_iters"])}
    mat.close()
    return {"workload": _describe(base).replace("eps 1e-06", "eps 1e-2 / 1e-6"), "forms": out}


def ldlt_form(tlr, torch, wl, steps: int):
    """The 3D Matern workload (N = 131072, tile 1024, eps 1e-4 absolute,
    ARA block 32, diagonal shift -1e-2 ||A||, indefinite): TLR LDL^T."""
    w = wl.standard("matern3d_131k")
    t0 = time.perf_counter()
    mat = tlr.TLRMatrix.compress_kernel(w.points, w.kernel, w.ell, w.diag_add, w.m, w.eps,
                                        tlr.opts(bs=w.bs))
    t_build = time.perf_counter() - t0
    o = tlr.opts(bs=w.bs, eps_mode=w.eps_mode)
    mat.ldlt(w.eps, o)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = [mat.ldlt(w.eps, o)[0] for _ in range(steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ra = mat.ranks(tlr.INPUT)[np.tril_indices(mat.nb, -1)]
    rl = mat.ranks(tlr.FACTOR)[np.tril_indices(mat.nb, -1)]
    out = {"workload": _describe(w), "N": w.n, "tile": w.m, "eps": w.eps, "bs": w.bs,
           "shift": -w.diag_add, "ms_per_step": dt * 1e3,
           "tflops": float(np.mean([x["flops"] for x in sts])) / dt / 1e12,
           "residual": residual(mat, torch), "input_build_s": t_build,
           "ranks_input": {"min": int(ra.min()), "mean": float(ra.mean()), "max": int(ra.max())},
           "ranks_factor": {"min": int(rl.min()), "mean": float(rl.mean()), "max": int(rl.max())},
           "ara_iterations": int(sts[-1]["ara_iters"])}
    mat.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cov2d_131k")
    ap.add_argument("--bs", type=int, default=0, help="ARA block size (0 = the workload's)")
    ap.add_argument("--bs-tail", type=int, default=0,
                    help="ARA block size after the first iteration of a column (0 = bs)")
    ap.add_argument("--tail-active", type=int, default=0,
                    help="use --bs-tail only once at most this many tiles of a column are active "
                         "(0 = from the second iteration on)")
    ap.add_argument("--cpu-sample", type=int, default=12288,
                    help="points of the leading block the CPU oracle factors (0 = skip)")
    ap.add_argument("--no-forms", dest="forms", action="store_false",
                    help="skip the relative-threshold FP64 / mixed-precision comparison")
    ap.add_argument("--no-kernel-timing", dest="kernel_timing", action="store_false",
                    help="skip the second pass that times the sampling launches with their own "
                         "events (no roofline figures)")
    ap.add_argument("--no-cfg2", dest="cfg2", action="store_false",
                    help="skip the N=32768 tile-512 line at eps 1e-2 and 1e-6")
    ap.add_argument("--no-phases", dest="phases", action="store_false",
                    help="skip the factorization with phase timers (per-phase GPU time)")
    ap.add_argument("--no-ldlt", dest="ldlt", action="store_false",
                    help="skip the LDL^T line (3D Matern, indefinite) after the main line")
    ap.add_argument("--no-pivoted", dest="pivoted", action="store_false",
                    help="skip the pivoted / unpivoted line (3D covariance, tile 512)")
    ap.add_argument("--no-pcg", dest="pcg", action="store_false",
                    help="skip the preconditioned CG line (N=32768)")
    ap.add_argument("--no-recompress", dest="recompress", action="store_false",
                    help="skip the SVD post-recompression line (the headline factor)")
    ap.add_argument("--no-schur", dest="schur", action="store_false",
                    help="skip the Schur compensation line (N=32768)")
    ap.add_argument("--profile-recompress", action="store_true",
                    help="with --profile: recompress the last factor after the timed steps")
    ap.add_argument("--batched", type=int, default=96,
                    help="problems of the batched workload timed after the main line (0 = skip)")
    ap.add_argument("--form", default="fp64",
                    choices=["fp64", "fp64_rel", "mixed_fp32_rel", "mixed_bf16_rel", "fp64_rel2"],
                    help="with --profile: the form to factor (fp64: the headline; fp64_rel: "
                         "relative 1e-6 in FP64; mixed_fp32_rel: relative 1e-6 with FP32 panels; "
                         "mixed_bf16_rel: relative 1e-2 with BF16 panels and the shift tau; "
                         "fp64_rel2: relative 1e-2 in FP64 with the shift tau)")
    ap.add_argument("--profile", action="store_true",
                    help="for profilers: build the input, run the --warmup and --steps "
                         "factorizations and stop (no second pass, residual or other lines)")
    ap.add_argument("--serial", action="store_true",
                    help="with --profile: run each sampling product in a launch of its own (the "
                         "schedule of the pass that times them with events), for the HBM counters "
                         "of the roofline")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates HBM "
                         "byte counters against a kernel of known traffic)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the factorization is a single-GPU code path "
              "(one GPU's share of the column step, at its real shape); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2108_11932_amd import tlr
    from paper_2108_11932_amd import workloads as wl

    torch.cuda.set_device(0)
    if a.copy_probe_mb > 0:
        n = a.copy_probe_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] copy probe: %d MiB read, %d MiB written" % (a.copy_probe_mb, a.copy_probe_mb),
              file=sys.stderr, flush=True)
        del src, dst
    w = wl.standard(a.workload)
    if a.bs:
        w.bs = a.bs
    print("[bench] building %s on the GPU" % w.name, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    mat = tlr.TLRMatrix.compress_kernel(w.points, w.kernel, w.ell, w.diag_add, w.m, w.eps,
                                        tlr.opts(bs=w.bs))
    t_build = time.perf_counter() - t0
    ra = mat.ranks(tlr.INPUT)[np.tril_indices(mat.nb, -1)]
    print("[bench] input built in %.1fs, ranks %d..%d mean %.1f" % (t_build, ra.min(), ra.max(),
                                                                     ra.mean()), file=sys.stderr,
          flush=True)
    # the headline steps run without per-launch events (they cost a few
    # percent of the step); the sampling kernel's durations come from the
    # dispatches' own events in a second pass of the same number of steps
    if a.profile and a.form != "fp64":
        prec, eps, shift = {"fp64_rel": (tlr.FP64, 1e-6, 0.0),
                            "mixed_fp32_rel": (tlr.MIXED_FP32, 1e-6, 0.0),
                            "mixed_bf16_rel": (tlr.MIXED_BF16, 1e-2, -1.0),
                            "fp64_rel2": (tlr.FP64, 1e-2, -1.0)}[a.form]
        o = tlr.opts(bs=w.bs, eps_mode=tlr.EPS_REL, precision=prec, shift=shift)
        for _ in range(a.warmup):
            mat.potrf(eps, o)
        torch.cuda.synchronize()
        time.sleep(0.05)
        t0 = time.perf_counter()
        sts = [mat.potrf(eps, o) for _ in range(a.steps)]
        torch.cuda.synchronize()
        print(json.dumps({"profile": w.name, "form": a.form,
                          "ms_per_step": (time.perf_counter() - t0) / a.steps * 1e3,
                          "fp32_tile_iters": sts[-1]["fp32_tile_iters"],
                          "bf16_tile_iters": sts[-1]["bf16_tile_iters"],
                          "tile_iters": sts[-1]["tile_iters"]}), flush=True)
        mat.close()
        return
    dt, stats = time_form(mat, w, w.eps_mode, tlr.FP64, tlr, torch, a.steps, a.warmup, a.bs_tail,
                          a.tail_active, False, 0.05 if a.profile else 0.0,
                          a.profile and a.serial)
    print("[bench] %d timed steps, %.1f ms each" % (a.steps, dt * 1e3), file=sys.stderr, flush=True)
    if a.profile:
        out = {"profile": w.name, "ms_per_step": dt * 1e3, "serial": a.serial,
               "ara_iterations": int(stats[-1]["ara_iters"]),
               "sample_bytes": stats[-1]["sample_bytes"]}
        if a.profile_recompress:
            # the last factor's SVD post-recompression, after a marker gap
            time.sleep(0.05)
            r0 = int(mat.ranks(tlr.FACTOR).sum())
            t0 = time.perf_counter()
            mat.recompress(stats[-1]["tau"])
            torch.cuda.synchronize()
            out.update({"recompress_ms": (time.perf_counter() - t0) * 1e3, "rank_sum_before": r0,
                        "rank_sum_after": int(mat.ranks(tlr.FACTOR).sum())})
        print(json.dumps(out), flush=True)
        mat.close()
        return
    dt_ev, stats_ev = (time_form(mat, w, w.eps_mode, tlr.FP64, tlr, torch, a.steps, 0, a.bs_tail, a.tail_active, True)
                       if a.kernel_timing else (0.0, []))
    phases = phase_split(mat, w, tlr, torch) if a.phases else None
    err_primary = residual(mat, torch)
    flops = float(np.mean([s["flops"] for s in stats]))
    flops_paper = float(np.mean([s["flops_paper"] for s in stats]))
    smp_bytes = sum(s["sample_bytes"] for s in stats_ev)
    smp_ms = sum(s["sample_ms"] for s in stats_ev)
    smp_n = sum(s["sample_launches"] for s in stats_ev)
    achieved = smp_bytes / (smp_ms * 1e-3) / 1e9 if smp_ms > 0 else 0.0
    rl = mat.ranks(tlr.FACTOR)[np.tril_indices(mat.nb, -1)]
    # FP64 against mixed precision at the relative threshold, where the FP32
    # rounding guard admits the tiles (at an absolute 1e-6 it admits almost
    # none, and the mixed form is the FP64 one), and BF16 against FP64 at a
    # relative 1e-2 with the shift tau
    forms = {}
    if a.forms:
        for name, mode, prec, feps, fshift in (
                ("fp64_rel", 1, tlr.FP64, 1e-6, 0.0), ("mixed_fp32_rel", 1, tlr.MIXED_FP32, 1e-6, 0.0),
                ("mixed_fp32_abs", 0, tlr.MIXED_FP32, 1e-6, 0.0),
                ("fp64_rel_1e-2", 1, tlr.FP64, 1e-2, -1.0),
                ("mixed_bf16_rel_1e-2", 1, tlr.MIXED_BF16, 1e-2, -1.0)):
            fdt, fst = time_form(mat, w, mode, prec, tlr, torch, a.steps, a.warmup, a.bs_tail,
                                 a.tail_active, False, eps=feps, shift=fshift)
            s0 = fst[-1]
            forms[name] = {"ms_per_step": fdt * 1e3,
                           "tflops": float(np.mean([x["flops"] for x in fst])) / fdt / 1e12,
                           "eps": feps, "shift": s0["shift"],
                           "eps_mode": "relative" if mode else "absolute", "tau": s0["tau"],
                           "residual": residual(mat, torch, shift=s0["shift"]),
                           "fp32_share": s0["fp32_tile_iters"] / max(1, s0["tile_iters"]),
                           "bf16_share": s0["bf16_tile_iters"] / max(1, s0["tile_iters"]),
                           "ara_iterations": int(s0["ara_iters"]),
                           "tile_iterations": int(s0["tile_iters"]),
                           "mean_rank": s0["mean_rank"], "max_rank": int(s0["max_rank"])}
            print("[bench] form %s: %.1f ms, residual %.3g" % (name, fdt * 1e3,
                                                               forms[name]["residual"]),
                  file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": flops / dt / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": _describe(w), "name": w.name, "N": w.n, "tile": w.m, "eps": w.eps,
                   "eps_mode": "absolute" if w.eps_mode == 0 else "relative", "bs": w.bs,
                   "bs_tail": a.bs_tail or w.bs, "tail_active": a.tail_active,
                   "precision": "fp64"},
        "time_to_solution_s": dt,
        "tflops_paper_count": flops_paper / dt / 1e12,
        "ranks_factor": {"min": int(rl.min()), "median": float(np.median(rl)),
                         "mean": float(rl.mean()), "max": int(rl.max())},
        "ara_iterations": int(stats[-1]["ara_iters"]),
        "tau": stats[-1]["tau"],
        "residual": err_primary,
        # the error bound the parity tests hold the factor to:
        # ||(A - L L^T) x|| / ||x|| <= ||A - L L^T||_2, each off-diagonal tile
        # of the error at most tau (the ARA threshold, both triangles), and
        # errors of independent tiles adding up like sqrt(nb) (the rigorous
        # worst case, (nb - 1) tau, is far looser)
        "residual_bound": 2.0 * math.sqrt(mat.nb) * stats[-1]["tau"],
        "residual_within_bound": bool(err_primary <= 2.0 * math.sqrt(mat.nb) * stats[-1]["tau"]),
        "forms": forms,
        "phases": phases,
        "kernels": kernel_table(w.name),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(w.name),
                     "kernel": "Schur-complement sampling product Y_i -= U_i* Z_i",
                     "launches": int(smp_n / max(1, a.steps)),
                     "bytes_per_launch": smp_bytes / max(1, smp_n),
                     "avg_launch_us": smp_ms * 1e3 / max(1, smp_n),
                     "events_pass_ms_per_step": dt_ev * 1e3},
    }
    if a.recompress:
        print("[bench] SVD post-recompression of the factor", file=sys.stderr, flush=True)
        line["recompress"] = recompress_form(
            mat, w, tlr, torch, tlr.opts(bs=w.bs, bs_tail=a.bs_tail, tail_active=a.tail_active,
                                        eps_mode=w.eps_mode))
        rc = line["recompress"]
        print("[bench] recompress: %.1f ms, ranks %d -> %d (-%.1f%%), factor %.2f -> %.2f GB, "
              "solve %.1f -> %.1f ms, residual %.3g (bound %.3g)"
              % (rc["recompress_ms"], rc["rank_sum_before"], rc["rank_sum_after"],
                 100 * rc["lowrank_rank_reduction"], rc["factor_bytes_before"] / 1e9,
                 rc["factor_bytes_after"] / 1e9, rc["solve_ms_before"], rc["solve_ms_after"],
                 rc["residual_after"], rc["residual_bound"]), file=sys.stderr, flush=True)
    mat.close()
    if a.cfg2:
        print("[bench] 2D covariance N=32768, tile 512", file=sys.stderr, flush=True)
        line["cov2d_32k"] = cov2d_32k_form(tlr, torch, wl, max(1, min(a.steps, 5)))
        for k, v in line["cov2d_32k"]["forms"].items():
            print("[bench] cov2d_32k %s: %.1f ms, residual %.3g (bound %.3g), rank total %d (oracle %s)"
                  % (k, v["ms_per_step"], v["residual"], v["bound"], v["rank_total"],
                     v["rank_total_oracle"]), file=sys.stderr, flush=True)
    if a.ldlt:
        print("[bench] LDL^T workload (3D Matern, N=131072)", file=sys.stderr, flush=True)
        line["ldlt"] = ldlt_form(tlr, torch, wl, max(1, min(a.steps, 2)))
        print("[bench] ldlt: %.1f ms, residual %.3g, ranks mean %.1f max %d"
              % (line["ldlt"]["ms_per_step"], line["ldlt"]["residual"],
                 line["ldlt"]["ranks_factor"]["mean"], line["ldlt"]["ranks_factor"]["max"]),
              file=sys.stderr, flush=True)
    if a.pivoted:
        print("[bench] pivoted workload (3D covariance, N=131072, tile 512)", file=sys.stderr,
              flush=True)
        line["pivoted"] = pivoted_form(tlr, torch, wl, max(1, min(a.steps, 2)))
        for k in ("unpivoted", "pivoted"):
            v = line["pivoted"][k]
            print("[bench] cov3d_131k %s: %.1f ms, residual %.3g, ranks mean %.1f max %d"
                  % (k, v["ms_per_step"], v["residual"], v["rank_mean"], v["rank_max"]),
                  file=sys.stderr, flush=True)
    if a.pcg:
        print("[bench] preconditioned CG (N=32768)", file=sys.stderr, flush=True)
        line["pcg"] = pcg_form(tlr, torch, wl)
        for k, v in line["pcg"].items():
            if isinstance(v, dict):
                print("[bench] pcg %s: %d iterations, %.1f ms" % (k, v["iterations"], v["pcg_ms"]),
                      file=sys.stderr, flush=True)
    if a.schur:
        print("[bench] Schur compensation (N=32768, tile 512)", file=sys.stderr, flush=True)
        line["schur"] = schur_form(tlr, torch, wl)
        for k in ("plain", "schur"):
            v = line["schur"][k]
            print("[bench] schur %s: %.1f ms, residual %.3g (bound %.3g); relative 1e-2: status %d, "
                  "row %d" % (k, v["ms"], v["residual"], v["bound"], v["rel_1e-2_status"],
                              v["rel_1e-2_failing_row"]), file=sys.stderr, flush=True)
    if a.batched > 0:
        print("[bench] batched workload: %d problems" % a.batched, file=sys.stderr, flush=True)
        line["batched"] = batched_form(tlr, torch, wl, a.batched, 512)
        b = line["batched"]
        print("[bench] batched: tiles %s (tuning %.1fs); sequential %.3fs, batched fp64 %.3fs "
              "(x%.2f), mixed %.3fs (x%.2f), fixed tile %d %.3fs"
              % (b["tiles_tuned"], b["tuning_s"], b["sequential_fp64_s"], b["batched_fp64_s"],
                 b["speedup_fp64"], b["batched_mixed_fp32_s"], b["speedup_mixed"], b["fixed_tile"],
                 b["batched_fp64_fixed_tile_s"]), file=sys.stderr, flush=True)
    if a.cpu_sample > 0:
        print("[bench] CPU oracle on a %d-point sample" % a.cpu_sample, file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, min(a.cpu_sample, w.n), tlr, torch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
