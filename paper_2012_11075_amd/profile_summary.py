"""Summarise rocprofv3 output of ``profile_step.py`` runs into profiles/.

For each precision it reads three rocprofv3 output directories (CSV format):

  kt    --kernel-trace --stats       average duration of the step kernel
  fetch --pmc FETCH_SIZE             KiB fetched per dispatch
  write --pmc WRITE_SIZE             KiB written per dispatch

and scales each counter by what it reads for the calibration kernel of known
traffic (an elementwise kernel that reads and writes ``copy_mib`` MiB).  It
writes ``<out>.json`` (read by bench.py together with the kernel source hash
the counters were taken on) and ``<out>.md``.

    python -m paper_2012_11075_amd.profile_summary --root <rocprofv3 output dir> \
        --out profiles/step_droplet_4096 --copy-mib 1024 --nodes 16777216 \
        --command-kt "..." --command-pmc "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BYTES_PER_UPDATE = {"fp64": 144, "fp32s": 72}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ["lbm_kernels.hip", "lbm_kernels.h"]:
        with open(os.path.join(ROOT, "paper_2012_11075_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _csv(d, suffix):
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not files:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


KERNEL = "march<"


def _is_step(name):
    return KERNEL in name and "true>" not in name


def _is_calib(name):
    return "AUnaryFunctor" in name and "MulFunctor" in name


def summarise(root, precision, copy_mib, nodes, bytes_per_update=None):
    kt = _csv(os.path.join(root, "kt_" + precision), "kernel_trace.csv")
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in kt if _is_step(r["Kernel_Name"])]
    names = sorted({r["Kernel_Name"] for r in kt if _is_step(r["Kernel_Name"])})
    out = {"kernel": names[0] if names else None, "dispatches": len(durs),
           "avg_ns": statistics.mean(durs), "min_ns": min(durs), "max_ns": max(durs)}
    per = {}
    for ctr, sub in [("FETCH_SIZE", "fetch_"), ("WRITE_SIZE", "write_")]:
        rows = _csv(os.path.join(root, sub + precision), "counter_collection.csv")
        step = [float(r["Counter_Value"]) for r in rows
                if _is_step(r["Kernel_Name"]) and r["Counter_Name"] == ctr]
        cal = [float(r["Counter_Value"]) for r in rows
               if _is_calib(r["Kernel_Name"]) and r["Counter_Name"] == ctr]
        cal_kib = statistics.mean(cal)
        scale = copy_mib * 1024.0 / cal_kib
        per[ctr] = {"raw_kib_per_dispatch": statistics.mean(step), "calibration_raw_kib": cal_kib,
                    "scale": scale, "bytes_per_launch": statistics.mean(step) * 1024.0 * scale}
    alg = (bytes_per_update or BYTES_PER_UPDATE[precision]) * nodes
    total = per["FETCH_SIZE"]["bytes_per_launch"] + per["WRITE_SIZE"]["bytes_per_launch"]
    out.update(counters=per, bytes_per_launch=total, algorithmic_bytes_per_launch=alg,
               traffic_over_algorithmic=total / alg,
               reads_over_algorithmic=per["FETCH_SIZE"]["bytes_per_launch"] / (alg / 2),
               writes_over_algorithmic=per["WRITE_SIZE"]["bytes_per_launch"] / (alg / 2),
               achieved_algorithmic_gbs=alg / out["avg_ns"],
               achieved_measured_gbs=total / out["avg_ns"])
    return out


def durations(root, precision, nodes, bytes_per_update=None):
    """Kernel-trace summary only (no counters)."""
    kt = _csv(os.path.join(root, "kt_" + precision), "kernel_trace.csv")
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in kt if _is_step(r["Kernel_Name"])]
    names = sorted({r["Kernel_Name"] for r in kt if _is_step(r["Kernel_Name"])})
    alg = (bytes_per_update or BYTES_PER_UPDATE[precision]) * nodes
    avg = statistics.mean(durs)
    return {"kernel": names[0] if names else None, "dispatches": len(durs), "avg_ns": avg,
            "min_ns": min(durs), "max_ns": max(durs), "algorithmic_bytes_per_launch": alg,
            "achieved_algorithmic_gbs": alg / avg}


def dispatch_table(kt_root, pmc_root, kernel, xcds=8):
    """Per-dispatch duration of `kernel` from a kernel trace, and the mean
    clock over each dispatch from a GRBM_GUI_ACTIVE counter run of the same
    command (the counter sums the busy cycles of the `xcds` XCDs)."""
    kt = [r for r in _csv(kt_root, "kernel_trace.csv") if kernel in r["Kernel_Name"]]
    kt.sort(key=lambda r: int(r["Start_Timestamp"]))
    pmc = [r for r in _csv(pmc_root, "counter_collection.csv")
           if kernel in r["Kernel_Name"] and r["Counter_Name"] == "GRBM_GUI_ACTIVE"]
    pmc.sort(key=lambda r: int(r["Start_Timestamp"]))
    rows = []
    for i, r in enumerate(kt):
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        row = {"launch": i + 1, "kernel_trace_us": d / 1e3}
        if i < len(pmc):
            dp = int(pmc[i]["End_Timestamp"]) - int(pmc[i]["Start_Timestamp"])
            row["counter_run_us"] = dp / 1e3
            row["clock_mhz"] = float(pmc[i]["Counter_Value"]) / xcds / dp * 1e3
        rows.append(row)
    return rows


SQ_MIX = ["SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
          "SQ_INSTS_BRANCH"]
SQ_CYC = ["SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_ANY"]


def sq_counters(root, kernel):
    """Mean per dispatch of every counter of `kernel` in a --pmc run, the
    first dispatch (cold caches) left out."""
    by = {}
    for r in _csv(root, "counter_collection.csv"):
        if "::" + kernel in r["Kernel_Name"]:
            d = by.setdefault(int(r["Dispatch_Id"]), {})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    ids = sorted(by)[1:] or sorted(by)
    return {k: sum(by[i].get(k, 0.0) for i in ids) / len(ids) for k in by[ids[0]]}, len(ids)


def sq_table(specs):
    """Rows of instruction counts per 64 node updates (one wave instruction
    covers 64 lanes) and per-wave cycle fractions, one per spec
    'label|mix_dir|cycles_dir|kernel prefix|nodes per launch'."""
    rows = []
    for spec in specs:
        label, mix, cyc, kernel, nodes = spec.split("|")
        m, n1 = sq_counters(mix, kernel)
        c, n2 = sq_counters(cyc, kernel)
        waves64 = int(nodes) / 64.0
        row = {"label": label, "kernel": kernel, "nodes": int(nodes), "dispatches": [n1, n2]}
        for k in SQ_MIX:
            row[k + "_per_64_nodes"] = m.get(k, float("nan")) / waves64
        for k in SQ_CYC:
            row[k + "_fraction_of_wave_cycles"] = c.get(k, float("nan")) / c["SQ_WAVE_CYCLES"]
        rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--root", default="")
    ap.add_argument("--out", required=True)
    ap.add_argument("--dispatch-table", default="",
                    help="KT_DIR,PMC_DIR: per-dispatch durations and clocks of --kernel from a "
                         "kernel trace and a GRBM_GUI_ACTIVE counter run of one command")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--nodes", type=int, default=4096 * 4096)
    ap.add_argument("--precisions", default="fp64,fp32s")
    ap.add_argument("--command-kt", default="")
    ap.add_argument("--command-pmc", default="")
    ap.add_argument("--tile", default="")
    ap.add_argument("--kernel", default="march<",
                    help="name prefix of the kernel to summarise (march< or march_batch<), or one "
                         "per precision: fp64=march<,fp32s=march2<")
    ap.add_argument("--title", default="Step kernel on the 4096 x 4096 droplet lattice")
    ap.add_argument("--bytes", default="",
                    help="algorithmic bytes per node and launch per precision, e.g. "
                         "fp64=304,fp32s=152 (default 144 and 72)")
    ap.add_argument("--kt-only", action="store_true",
                    help="kernel trace only (no counter runs): durations, no traffic")
    ap.add_argument("--sq", action="append", default=[],
                    help="'label|mix_dir|cycles_dir|kernel prefix|nodes per launch': instruction "
                         "mix and cycle fractions from two SQ counter runs (repeatable)")
    args = ap.parse_args()
    global KERNEL
    KERNEL = args.kernel
    per_prec = dict(kv.split("=", 1) for kv in args.kernel.split(",")) if "=" in args.kernel else {}
    if args.sq:
        rows = sq_table(args.sq)
        with open(args.out + ".json", "w") as fh:
            json.dump({"commands": {"mix": args.command_kt, "cycles": args.command_pmc},
                       "rows": rows}, fh, indent=1)
        lines = ["# %s (rocprofv3)" % args.title, "",
                 "Commands (run from `/tmp`, `TMPDIR=/tmp`, repository at `$R`):", "",
                 "```", args.command_kt, args.command_pmc, "```", "",
                 "Instructions are wave instructions per 64 node updates (one per lane and node); "
                 "cycle columns are the counter over SQ_WAVE_CYCLES, the fraction of a resident "
                 "wave's time spent issuing that kind of instruction or waiting on one.", "",
                 "| workload | VALU | SALU | LDS | VMEM rd | VMEM wr | branch | VALU active | "
                 "scalar active | LDS active | waiting |",
                 "|---|---|---|---|---|---|---|---|---|---|---|"]
        for r in rows:
            lines.append("| %s | %s | %.3f | %.3f | %.3f | %.3f |" % (
                r["label"] + " (`%s`)" % r["kernel"],
                " | ".join("%.1f" % r[k + "_per_64_nodes"] for k in SQ_MIX),
                *[r[k + "_fraction_of_wave_cycles"] for k in SQ_CYC]))
        with open(args.out + ".md", "w") as fh:
            fh.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return
    if args.dispatch_table:
        kt_dir, pmc_dir = args.dispatch_table.split(",")
        rows = dispatch_table(kt_dir, pmc_dir, args.kernel)
        with open(args.out + ".json", "w") as fh:
            json.dump({"kernel": args.kernel, "commands": {"kernel_trace": args.command_kt,
                                                           "pmc": args.command_pmc},
                       "dispatches": rows}, fh, indent=1)
        lines = ["# %s (rocprofv3)" % args.title, "",
                 "Commands (run from `/tmp`, `TMPDIR=/tmp`, repository at `$R`):", "",
                 "```", args.command_kt, args.command_pmc, "```", "",
                 "Clock = GRBM_GUI_ACTIVE (busy cycles summed over the 8 XCDs) / (8 x duration "
                 "of the same dispatch in the counter run).", "",
                 "| launch | duration, kernel trace (us) | duration, counter run (us) | clock (MHz) |",
                 "|---|---|---|---|"]
        for r in rows:
            lines.append("| %d | %.1f | %s | %s |" % (
                r["launch"], r["kernel_trace_us"],
                "%.1f" % r["counter_run_us"] if "counter_run_us" in r else "-",
                "%.0f" % r["clock_mhz"] if "clock_mhz" in r else "-"))
        with open(args.out + ".md", "w") as fh:
            fh.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return
    res = {"kernel_source_hash": kernel_source_hash(), "nodes": args.nodes,
           "commands": {"kernel_trace": args.command_kt, "pmc": args.command_pmc},
           "tile": args.tile}
    bpu = dict(kv.split("=") for kv in args.bytes.split(",")) if args.bytes else {}
    for prec in args.precisions.split(","):
        b = int(bpu[prec]) if prec in bpu else None
        if per_prec:
            KERNEL = per_prec[prec]
        res[prec] = (durations(args.root, prec, args.nodes, b) if args.kt_only
                     else summarise(args.root, prec, args.copy_mib, args.nodes, b))
    with open(args.out + ".json", "w") as fh:
        json.dump(res, fh, indent=1)
    lines = ["# %s (rocprofv3)" % args.title, "",
             "Kernel source hash: `%s`; tile (block, rows, depth): %s" % (res["kernel_source_hash"], args.tile), "",
             "Commands (run from `/tmp`, `TMPDIR=/tmp`, repository at `$R`):", "",
             "```", args.command_kt, args.command_pmc, "```", "",
             "| precision | kernel | dispatches | avg us | algorithmic B/launch | measured B/launch (FETCH+WRITE, calibrated) | measured/algorithmic | reads/alg. | writes/alg. | GB/s algorithmic | GB/s measured |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    for prec in args.precisions.split(","):
        r = res[prec]
        short = (r["kernel"] or "").replace("lbmk::(anonymous namespace)::", "").replace(
            "void ", "").split("(")[0]
        if "counters" in r:
            lines.append("| %s | `%s` | %d | %.1f | %.4g | %.4g | %.3f | %.3f | %.3f | %.0f | %.0f |" % (
                prec, short, r["dispatches"], r["avg_ns"] / 1e3, r["algorithmic_bytes_per_launch"],
                r["bytes_per_launch"], r["traffic_over_algorithmic"], r["reads_over_algorithmic"],
                r["writes_over_algorithmic"], r["achieved_algorithmic_gbs"],
                r["achieved_measured_gbs"]))
        else:
            lines.append("| %s | `%s` | %d | %.1f | %.4g | - | - | - | - | %.0f | - |" % (
                prec, short, r["dispatches"], r["avg_ns"] / 1e3, r["algorithmic_bytes_per_launch"],
                r["achieved_algorithmic_gbs"]))
    if not args.kt_only:
        lines += ["", "Counter calibration: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by "
                  "(calibration bytes / counter reading) of an elementwise kernel that reads and writes "
                  "%d MiB each:" % args.copy_mib, ""]
        for prec in args.precisions.split(","):
            if "counters" not in res[prec]:
                continue
            for ctr, c in res[prec]["counters"].items():
                lines.append("- %s %s: raw %.1f KiB/dispatch, calibration kernel %.1f KiB -> scale %.3f" % (
                    prec, ctr, c["raw_kib_per_dispatch"], c["calibration_raw_kib"], c["scale"]))
    with open(args.out + ".md", "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
