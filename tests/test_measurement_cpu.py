"""The profile reductions and the benchmark's readers of the committed
profile summaries, on the CPU: synthetic rocprofv3 CSV files whose sums,
calibrations and fractions can be worked out by hand."""
import csv
import os
import sys

import pytest

from paper_2108_11932_amd import rocprof_summary as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

TRACE_COLS = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id",
              "Kernel_Name", "Correlation_Id", "Start_Timestamp", "End_Timestamp"]
PMC_COLS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, cols, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow({c: r.get(c, "0") for c in cols})


def _trace(tmp_path):
    # one warm-up factorization, a 50 ms idle gap, then the profiled one:
    # k_a twice (2 and 4 us) on queue 1, k_b once (10 us) on queue 2, a copy
    # of 100 us before the window (dispatch 1, after the generator)
    us = 1000
    rows = [
        dict(Dispatch_Id=0, Kernel_Name="void tlr::(anonymous namespace)::k_gen_tiles(int)",
             Queue_Id=1, Start_Timestamp=0, End_Timestamp=5 * us),
        dict(Dispatch_Id=1, Kernel_Name="__amd_rocclr_copyBuffer", Queue_Id=1,
             Start_Timestamp=10 * us, End_Timestamp=110 * us),
        dict(Dispatch_Id=2, Kernel_Name="tlr::(anonymous namespace)::k_a<16, true>(tlr::AraDev, int)",
             Queue_Id=1, Start_Timestamp=200 * us, End_Timestamp=201 * us),
        dict(Dispatch_Id=3, Kernel_Name="tlr::(anonymous namespace)::k_a<16, true>(tlr::AraDev, int)",
             Queue_Id=1, Start_Timestamp=60_000 * us, End_Timestamp=60_002 * us),
        dict(Dispatch_Id=4, Kernel_Name="tlr::(anonymous namespace)::k_b(double*)",
             Queue_Id=2, Start_Timestamp=60_001 * us, End_Timestamp=60_011 * us),
        dict(Dispatch_Id=5, Kernel_Name="tlr::(anonymous namespace)::k_a<16, true>(tlr::AraDev, int)",
             Queue_Id=1, Start_Timestamp=60_020 * us, End_Timestamp=60_024 * us),
    ]
    p = tmp_path / "trace.csv"
    _write(p, TRACE_COLS, rows)
    return p


def test_short_names():
    assert rs._short("void tlr::(anonymous namespace)::k_gemm<false, true, 64, 16>(tlr::GemmDesc const*, int)") \
        == "k_gemm<false, true, 64, 16>"
    assert rs._short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_kernels_window_and_sums(tmp_path):
    out = rs.kernels(str(_trace(tmp_path)))
    head = out.splitlines()[0]
    # the window: dispatches 3, 4, 5 (after the 50 ms gap): 24 us span, 16 us summed
    assert "3 dispatches" in head and "summed kernel time 0.0 ms" in head
    lines = {l.split()[0]: l.split() for l in out.splitlines()[3:]}
    a = lines["k_a<16,"]
    assert a[2] == "2" and float(a[3]) == pytest.approx(6.0) and float(a[4]) == pytest.approx(3.0)
    assert lines["k_b"][1] == "1" and float(lines["k_b"][2]) == pytest.approx(10.0)
    assert lines["k_b"][-1] == "2" and a[-1] == "1"


def test_counters_calibration_and_fraction(tmp_path):
    tr = _trace(tmp_path)
    # the copy of 1 MiB reads FETCH_SIZE 512 KiB (factor 2) and WRITE_SIZE
    # 1024 KiB (factor 1); k_a runs 1e5 MOPS of F64 in its two calls
    pmc = [
        dict(Dispatch_Id=1, Kernel_Name="__amd_rocclr_copyBuffer", Counter_Name="FETCH_SIZE", Counter_Value=512),
        dict(Dispatch_Id=1, Kernel_Name="__amd_rocclr_copyBuffer", Counter_Name="WRITE_SIZE", Counter_Value=1024),
        dict(Dispatch_Id=3, Kernel_Name="k_a<16, true>(tlr::AraDev, int)", Counter_Name="FETCH_SIZE", Counter_Value=100),
        dict(Dispatch_Id=5, Kernel_Name="k_a<16, true>(tlr::AraDev, int)", Counter_Name="FETCH_SIZE", Counter_Value=50),
        dict(Dispatch_Id=3, Kernel_Name="k_a<16, true>(tlr::AraDev, int)",
             Counter_Name="SQ_INSTS_VALU_MFMA_MOPS_F64", Counter_Value=60000),
        dict(Dispatch_Id=5, Kernel_Name="k_a<16, true>(tlr::AraDev, int)",
             Counter_Name="SQ_INSTS_VALU_MFMA_MOPS_F64", Counter_Value=40000),
    ]
    p = tmp_path / "pmc.csv"
    _write(p, PMC_COLS, pmc)
    out = rs.counters(str(p), trace=str(tr), copy_mib=1)
    assert "FETCH_SIZE x2.0000" in out and "WRITE_SIZE x1.0000" in out
    row = [l for l in out.splitlines() if l.startswith("k_a<16")][0].split()
    # calls 2, time 6 us, FETCH (100 + 50) x 2 = 300 KiB
    vals = [float(x) for x in row[3:]]
    assert int(row[2]) == 2 and vals[0] == pytest.approx(6.0)
    assert 300.0 in [pytest.approx(v) for v in vals]
    # fraction of the FP64 peak: 1e5 x 512 flop in 6 us against 78.6 TF/s
    assert vals[-1] == pytest.approx(1e5 * 512 / 6e-6 / 78.6e12, abs=1e-4)


def test_table_bound(tmp_path):
    def summary(name, cols, rows):
        p = tmp_path / name
        with open(p, "w") as fh:
            fh.write("dispatches: x\n\n")
            fh.write("%-60s %7s %11s" % ("kernel", "calls", "time_us") + "".join(" %16s" % c for c in cols) + "\n")
            for k, calls, t, vs in rows:
                fh.write("%-60s %7d %11.1f" % (k, calls, t) + "".join(" %16.4g" % v for v in vs) + "\n")
        return str(p)
    # k_mf: 1e6 MOPS in 10 us = 51.2 TF/s (65 % of FP64), 1 KiB of traffic;
    # k_bw: 0 MOPS, 40000 KiB in 10 us = 4.1 TB/s (51 % of HBM);
    # k_lat: neither above 10 %
    mf = summary("mfma.txt", ["SQ_INSTS_VALU_MFMA_MOPS_F64"],
                 [("k_mf", 1, 10.0, [1e6]), ("k_bw", 1, 10.0, [0]), ("k_lat", 1, 10.0, [1e4])])
    fe = summary("fetch.txt", ["FETCH_SIZE"], [("k_mf", 1, 10.0, [1]), ("k_bw", 1, 10.0, [40000]),
                                                ("k_lat", 1, 10.0, [100])])
    wr = summary("write.txt", ["WRITE_SIZE"], [("k_mf", 1, 10.0, [0]), ("k_bw", 1, 10.0, [0]),
                                                ("k_lat", 1, 10.0, [0])])
    rows = {l.split(" | ")[0]: l.split(" | ") for l in rs.table(mf, fe, wr).splitlines()[1:]}
    assert rows["k_mf"][-1] == "mfma" and float(rows["k_mf"][5]) == pytest.approx(0.6514, abs=1e-3)
    assert rows["k_bw"][-1] == "hbm" and float(rows["k_bw"][7]) == pytest.approx(0.512, abs=1e-3)
    assert rows["k_lat"][-1] == "latency"


def test_bench_reads_committed_profiles():
    sys.path.insert(0, ROOT)
    import bench
    t = bench.kernel_table("cov2d_131k")
    assert t is not None and t["rows"], "profiles/roofline_table_cov2d_131k.txt unreadable"
    for r in t["rows"]:
        assert r["bound"] in ("mfma", "hbm", "latency")
        assert 0.0 <= r["frac_mfma_f64"] <= 1.0 and 0.0 <= r["frac_hbm"] <= 1.0
    assert bench.kernel_table("no_such_workload") is None
    kv = bench._key_values(bench.TRAFFIC_FILE)
    assert kv["workload"] == "cov2d_131k"
    assert 1.0 <= float(kv["traffic_over_algorithmic"]) <= 2.0
    # the traffic is reported exactly when the hashed sources match
    ok = kv["source_sha256"] == bench.kernel_source_hash()
    assert (bench.measured_traffic("cov2d_131k") is not None) == ok
