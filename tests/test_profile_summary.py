"""The rocprofv3 summariser (paper_2012_11075_amd/profile_summary.py) on
small synthetic CSV files of rocprofv3's layout: counter calibration and
traffic ratios, the per-dispatch clock table, and the SQ instruction mix.
No GPU is needed."""
import csv
import os

import pytest

from paper_2012_11075_amd import profile_summary as S

STEP = "void lbmk::(anonymous namespace)::march<double, 1, 512, 3, false>(lbmk::Geometry)"
OBS = "void lbmk::(anonymous namespace)::march<double, 1, 512, 3, true>(lbmk::Geometry)"
CAL = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<double, " \
      "double, double, at::native::binary_internal::MulFunctor<double>>>(int)"


def write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)


def trace(path, kernels):
    """kernels: [(name, start_ns, end_ns)]"""
    write_csv(path, [{"Kernel_Name": n, "Start_Timestamp": a, "End_Timestamp": b}
                     for n, a, b in kernels])


def counters(path, rows):
    """rows: [(dispatch, name, counter, value, start_ns, end_ns)]"""
    write_csv(path, [{"Dispatch_Id": d, "Kernel_Name": n, "Counter_Name": c, "Counter_Value": v,
                      "Start_Timestamp": a, "End_Timestamp": b} for d, n, c, v, a, b in rows])


def test_traffic_calibration(tmp_path):
    """FETCH and WRITE are scaled by what they read for the calibration
    kernel of known size; the ratios follow from the algorithmic bytes."""
    r = str(tmp_path)
    nodes = 1000
    trace(r + "/kt_fp64/run_kernel_trace.csv",
          [(STEP, 0, 2000), (STEP, 5000, 7000), (OBS, 8000, 9000), (CAL, 10000, 20000)])
    # calibration reads 1024 MiB and the counter shows half of it (scale 2);
    # the step reads 72 kB per launch (counter 36 kB) and writes 72 kB
    counters(r + "/fetch_fp64/run_counter_collection.csv",
             [(1, CAL, "FETCH_SIZE", 512 * 1024, 0, 1), (2, STEP, "FETCH_SIZE", 72000 / 2 / 1024, 0, 1)])
    counters(r + "/write_fp64/run_counter_collection.csv",
             [(1, CAL, "WRITE_SIZE", 1024 * 1024, 0, 1), (2, STEP, "WRITE_SIZE", 72000 / 1024, 0, 1)])
    S.KERNEL = "march<"
    out = S.summarise(r, "fp64", 1024, nodes)
    assert out["dispatches"] == 2 and out["avg_ns"] == 2000
    assert out["counters"]["FETCH_SIZE"]["scale"] == pytest.approx(2.0)
    assert out["counters"]["WRITE_SIZE"]["scale"] == pytest.approx(1.0)
    assert out["bytes_per_launch"] == pytest.approx(144000)
    assert out["traffic_over_algorithmic"] == pytest.approx(1.0)
    assert out["reads_over_algorithmic"] == pytest.approx(1.0)
    assert out["achieved_algorithmic_gbs"] == pytest.approx(144000 / 2000)


def test_dispatch_table_clock(tmp_path):
    """Clock of a dispatch = GRBM_GUI_ACTIVE summed over the XCDs / (XCDs x
    duration of that dispatch in the counter run)."""
    kt, pmc = str(tmp_path / "kt"), str(tmp_path / "pmc")
    trace(kt + "/run_kernel_trace.csv", [(STEP, 0, 400_000), (STEP, 500_000, 950_000)])
    counters(pmc + "/run_counter_collection.csv",
             [(1, STEP, "GRBM_GUI_ACTIVE", 8 * 2.0e9 * 410e-6, 0, 410_000),
              (2, STEP, "GRBM_GUI_ACTIVE", 8 * 1.8e9 * 420e-6, 600_000, 1_020_000)])
    rows = S.dispatch_table(kt, pmc, "march<double")
    assert [r["launch"] for r in rows] == [1, 2]
    assert rows[0]["kernel_trace_us"] == pytest.approx(400.0)
    assert rows[1]["kernel_trace_us"] == pytest.approx(450.0)
    assert rows[0]["counter_run_us"] == pytest.approx(410.0)
    assert rows[0]["clock_mhz"] == pytest.approx(2000.0)
    assert rows[1]["clock_mhz"] == pytest.approx(1800.0)


def test_sq_instruction_mix(tmp_path):
    """Instructions per 64 node updates and cycle fractions, averaged over
    the dispatches of the named kernel after the first; other kernels and
    other instances (march3 for march) are not counted."""
    mix, cyc = str(tmp_path / "mix"), str(tmp_path / "cyc")
    other = STEP.replace("march<", "march3<")
    rows = []
    for d, valu in [(1, 999.0), (2, 256.0), (3, 512.0)]:  # dispatch 1 is left out
        rows += [(d, STEP, "SQ_INSTS_VALU", valu, 0, 1), (d, STEP, "SQ_INSTS_SALU", 64.0, 0, 1),
                 (d, other, "SQ_INSTS_VALU", 1e9, 0, 1)]
    counters(mix + "/run_counter_collection.csv", rows)
    rows = []
    for d in (1, 2, 3):
        rows += [(d, STEP, "SQ_WAVE_CYCLES", 1000.0, 0, 1), (d, STEP, "SQ_ACTIVE_INST_VALU", 250.0, 0, 1),
                 (d, STEP, "SQ_WAIT_INST_ANY", 400.0, 0, 1)]
    counters(cyc + "/run_counter_collection.csv", rows)
    out = S.sq_table(["2-D|%s|%s|march<double|128" % (mix, cyc)])
    (r,) = out
    assert r["dispatches"] == [2, 2]
    # (256 + 512) / 2 wave instructions for 128 nodes = 2 waves of 64 nodes
    assert r["SQ_INSTS_VALU_per_64_nodes"] == pytest.approx(192.0)
    assert r["SQ_INSTS_SALU_per_64_nodes"] == pytest.approx(32.0)
    assert r["SQ_ACTIVE_INST_VALU_fraction_of_wave_cycles"] == pytest.approx(0.25)
    assert r["SQ_WAIT_INST_ANY_fraction_of_wave_cycles"] == pytest.approx(0.4)
