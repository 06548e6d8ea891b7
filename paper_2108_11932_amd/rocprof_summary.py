"""Reduce rocprofv3 CSV output of a bench.py run to the short text summaries
kept under profiles/.

    python -m paper_2108_11932_amd.rocprof_summary kernels  <kernel_trace.csv>
    python -m paper_2108_11932_amd.rocprof_summary counters <counter_collection.csv> \
        [--trace <kernel_trace.csv>] [--copy-mib N] [--durations <kernel_trace.csv>]
    python -m paper_2108_11932_amd.rocprof_summary table <mfma summary> \
        --fetch <FETCH_SIZE summary> --write <WRITE_SIZE summary>

Both select the dispatches of the last factorization of a bench.py --profile
run: those after the last input-generation kernel (k_gen_tiles) and after
the last idle gap of 20 ms between dispatches (bench.py --profile idles 50 ms
between factorizations).  `counters` takes that window from the kernel trace
given with --trace (dispatch ids are shared), else everything after
k_gen_tiles.

`kernels` prints, per kernel, calls, total and average duration and the
share of the summed kernel time, split by the queue (stream) the dispatches
ran on.  `counters` prints the per-kernel sums of every counter in the file
(plus, with --trace, the kernel durations of the same dispatches, matched by
dispatch id) and, for the FP64/FP32/BF16 MFMA op counters, the achieved
matrix-core rate against the MI355X dense peaks.  With --copy-mib, the
FETCH_SIZE / WRITE_SIZE of the largest __amd_rocclr_copyBuffer dispatch
(bench.py --copy-probe-mb) calibrates the byte counters.
"""
from __future__ import annotations

import argparse
import csv
import sys
from collections import OrderedDict, defaultdict

# dense matrix-core peaks of the MI355X (FLOP/s); MOPS counters count 512
# floating-point operations per unit
PEAK = {"F64": 78.6e12, "F32": 157.3e12, "BF16": 2.5e15, "F16": 2.5e15}
MOPS_UNIT = 512.0


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(names)


def _short(name: str) -> str:
    """Kernel name without namespaces, return type and parameter list."""
    n = name.replace("(anonymous namespace)::", "")
    if n.startswith("void "):
        n = n[5:]
    depth, cut = 0, len(n)
    for i, ch in enumerate(n):   # the parameter list: the first "(" outside <>
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    n = n[:cut].replace("tlr::", "")
    return n[:60]


# bench.py --profile idles this long between factorizations
IDLE_NS = 20_000_000


def _window(rows):
    """Rows of the last factorization: after the last k_gen_tiles dispatch
    and after the last idle gap of IDLE_NS in the dispatch start times."""
    rows = sorted(rows, key=lambda r: int(_col(r, "Dispatch_Id", "Dispatch_ID")))
    last_gen = -1
    for i, r in enumerate(rows):
        if "k_gen_tiles" in _col(r, "Kernel_Name"):
            last_gen = i
    rows = sorted(rows[last_gen + 1:], key=lambda r: int(_col(r, "Start_Timestamp")))
    cut = 0
    for i in range(1, len(rows)):
        if int(_col(rows[i], "Start_Timestamp")) - int(_col(rows[i - 1], "End_Timestamp")) > IDLE_NS:
            cut = i
    return rows[cut:]


def kernels(path: str) -> str:
    rows = _window(_rows(path))
    tot = defaultdict(float)
    calls = defaultdict(int)
    queue = defaultdict(set)
    t0, t1 = None, None
    for r in rows:
        k = _short(_col(r, "Kernel_Name"))
        s, e = int(_col(r, "Start_Timestamp")), int(_col(r, "End_Timestamp"))
        t0 = s if t0 is None else min(t0, s)
        t1 = e if t1 is None else max(t1, e)
        tot[k] += (e - s) / 1e3
        calls[k] += 1
        queue[k].add(_col(r, "Queue_Id", "Queue_ID", "Stream_Id"))
    summed = sum(tot.values())
    out = ["factorization window: %.1f ms, %d dispatches, summed kernel time %.1f ms" %
           ((t1 - t0) / 1e6 if rows else 0.0, len(rows), summed / 1e3), "",
           "%-60s %7s %12s %9s %6s  queues" % ("kernel", "calls", "total_us", "avg_us", "share")]
    for k in sorted(tot, key=lambda x: -tot[x]):
        out.append("%-60s %7d %12.1f %9.2f %5.1f%%  %s" %
                   (k, calls[k], tot[k], tot[k] / calls[k], 100 * tot[k] / summed,
                    ",".join(sorted(queue[k]))))
    return "\n".join(out)


def _avg_durations(path: str):
    """Per-kernel average duration (us) and calls of the last factorization
    of a plain --kernel-trace run."""
    tot = defaultdict(float)
    calls = defaultdict(int)
    for r in _window(_rows(path)):
        k = _short(_col(r, "Kernel_Name"))
        tot[k] += (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3
        calls[k] += 1
    return {k: (tot[k] / calls[k], calls[k]) for k in tot}


def counters(path: str, trace: str = None, copy_mib: int = 0, durations: str = None) -> str:
    rows = _rows(path)
    by_disp = OrderedDict()
    for r in rows:
        d = int(_col(r, "Dispatch_Id", "Dispatch_ID"))
        e = by_disp.setdefault(d, {"name": _col(r, "Kernel_Name"), "c": {}})
        e["c"][_col(r, "Counter_Name")] = e["c"].get(_col(r, "Counter_Name"), 0.0) + \
            float(_col(r, "Counter_Value"))
    disp = sorted(by_disp)
    cal = {}
    if copy_mib:
        copies = [d for d in disp if "copyBuffer" in by_disp[d]["name"]]
        if copies:
            big = max(copies, key=lambda d: by_disp[d]["c"].get("FETCH_SIZE", 0.0) +
                      by_disp[d]["c"].get("WRITE_SIZE", 0.0))
            kib = copy_mib * 1024.0
            for cn in ("FETCH_SIZE", "WRITE_SIZE"):
                v = by_disp[big]["c"].get(cn)
                if v:
                    cal[cn] = kib / v
    dur = {}
    if trace:
        tw = _window(_rows(trace))
        for r in tw:
            dur[int(_col(r, "Dispatch_Id", "Dispatch_ID"))] = \
                (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3
        win = [d for d in disp if d in dur]
    else:
        last_gen = max([i for i, d in enumerate(disp) if "k_gen_tiles" in by_disp[d]["name"]] or [-1])
        win = disp[last_gen + 1:]
    agg = defaultdict(lambda: defaultdict(float))
    calls = defaultdict(int)
    for d in win:
        k = _short(by_disp[d]["name"])
        calls[k] += 1
        for cn, v in by_disp[d]["c"].items():
            agg[k][cn] += v * cal.get(cn, 1.0)
        if d in dur:
            agg[k]["_us"] += dur[d]
    plain = _avg_durations(durations) if durations else {}
    if plain:
        # kernel time from the run without counters (counter collection
        # serialises and slows the dispatches): calls x plain average
        for k in agg:
            if k in plain:
                agg[k]["_us"] = plain[k][0] * calls[k]
    names = sorted({cn for k in agg for cn in agg[k] if cn != "_us"})
    out = ["dispatches of the last factorization: %d; counters: %s" % (len(win), ", ".join(names))]
    if plain:
        out.append("time_us: calls x the kernel's average duration in the run without counters")
    if cal:
        out.append("byte counters scaled by the copy calibration: %s" %
                   ", ".join("%s x%.4f" % kv for kv in sorted(cal.items())))
    out.append("")
    hdr = "%-60s %7s %11s" % ("kernel", "calls", "time_us")
    for cn in names:
        hdr += " %16s" % cn
    mops = [cn for cn in names if "MFMA_MOPS" in cn]
    for cn in mops:
        hdr += " %12s" % ("frac_" + cn.rsplit("_", 1)[-1])
    out.append(hdr)
    order = sorted(agg, key=lambda k: -(agg[k].get("_us", 0.0) or
                                        sum(agg[k][c] for c in mops)))
    for k in order:
        line = "%-60s %7d %11.1f" % (k, calls[k], agg[k].get("_us", 0.0))
        for cn in names:
            line += " %16.4g" % agg[k][cn]
        for cn in mops:
            prec = cn.rsplit("_", 1)[-1]
            t = agg[k].get("_us", 0.0) * 1e-6
            frac = (agg[k][cn] * MOPS_UNIT / t / PEAK.get(prec, float("nan"))) if t > 0 else 0.0
            line += " %12.4f" % frac
        out.append(line)
    return "\n".join(out)


def _parse_table(path: str):
    """Rows of a `counters` summary: {kernel: {column: value}}."""
    rows, hdr = {}, None
    with open(path) as fh:
        for ln in fh:
            if ln.startswith("kernel "):
                hdr = ln.split()
                continue
            if hdr is None or not ln.strip():
                continue
            name, rest = ln[:60].strip(), ln[60:].split()
            rows[name] = dict(zip(hdr[1:], [float(x) for x in rest]))
    return rows


HBM_PEAK = 8.0e12
LATENCY_FRAC = 0.10


def table(mfma: str, fetch: str, write: str) -> str:
    """Per-kernel roofline table of one factorization from the `counters`
    summaries of an MFMA-op run and of the FETCH_SIZE and WRITE_SIZE runs
    (calibrated KiB): time, achieved FP64 matrix-core rate and HBM rate, and
    their fractions of the MI355X peaks; `bound` names the larger one, or
    `latency` when neither reaches LATENCY_FRAC of its peak (a chain of
    dependent steps or a launch too small to fill the chip)."""
    mf, fe, wr = _parse_table(mfma), _parse_table(fetch), _parse_table(write)
    tot = sum(v.get("time_us", 0.0) for v in mf.values())
    out = ["kernel | calls | time_us | share | mfma_f64_tflops | frac_mfma_f64 | hbm_gbs | "
           "frac_hbm | bound"]
    for k in sorted(mf, key=lambda x: -mf[x].get("time_us", 0.0)):
        v = mf[k]
        t = v.get("time_us", 0.0) * 1e-6
        if t <= 0:
            continue
        fl = v.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * MOPS_UNIT
        by = (fe.get(k, {}).get("FETCH_SIZE", 0.0) + wr.get(k, {}).get("WRITE_SIZE", 0.0)) * 1024.0
        fm, fh = fl / t / PEAK["F64"], by / t / HBM_PEAK
        out.append("%s | %d | %.1f | %.3f | %.3f | %.4f | %.1f | %.4f | %s" %
                   (k, int(v.get("calls", 0)), v["time_us"], v["time_us"] / tot, fl / t / 1e12, fm,
                    by / t / 1e9, fh,
                    "latency" if max(fm, fh) < LATENCY_FRAC else ("mfma" if fm >= fh else "hbm")))
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("what", choices=["kernels", "counters", "table"])
    ap.add_argument("--fetch", default=None)
    ap.add_argument("--write", default=None)
    ap.add_argument("csv")
    ap.add_argument("--trace", default=None)
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--durations", default=None,
                    help="kernel_trace.csv of a run without counters (kernel times)")
    a = ap.parse_args(argv)
    if a.what == "kernels":
        print(kernels(a.csv))
    elif a.what == "table":
        print(table(a.csv, a.fetch, a.write))
    else:
        print(counters(a.csv, a.trace, a.copy_mib, a.durations))


if __name__ == "__main__":
    sys.exit(main())
