"""Summaries of rocprofv3 runs of the benchmark, written under ``profiles/``.

Inputs are rocprofv3 output directories written with ``--output-format csv``:

* a ``--kernel-trace --stats`` run (``*_kernel_stats.csv``): per-kernel call
  counts and durations;
* optionally one ``--pmc FETCH_SIZE`` and one ``--pmc WRITE_SIZE`` run
  (``*_counter_collection.csv``) of a benchmark started with
  ``--copy-calibration-mib M``: the device copy of M MiB is the reference
  that turns the counters (KiB per dispatch) into bytes.

The summary (markdown) states the command lines, the kernel table and the
traffic figures; a key/value file next to it carries the figures the
benchmark reports, with the hash of the kernel source they were taken from.

* optionally any number of further ``--pmc`` runs (``--counters DIR``):
  every counter they hold is reported for the kernel's largest-grid
  dispatches (median over them), with the ratios named in RATIOS.

python -m paper_2511_02742_amd.prof_summary --trace DIR [--fetch DIR --write DIR --copy-mib M]
        [--counters DIR ...] --name NAME --command "..." [--command "..."]
        [--kernel k_find_cf --source hough_cf.hip]
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import statistics
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
KERNEL_SOURCE = os.path.join(PKG, "csrc", "hough_kernels.hip")
# The benchmark's calibration kernel: torch.mul over M MiB of float32, which
# reads and writes exactly M MiB each.
COPY_KERNEL = "MulFunctor"


def kernel_source_hash(source: str = KERNEL_SOURCE) -> str:
    """sha256/16 of a kernel source file (csrc/ name or path)."""
    path = source if os.path.isabs(source) else os.path.join(PKG, "csrc", os.path.basename(source))
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _is(name: str, kernel: str) -> bool:
    # "k_find" must not match "k_find_cf": the template argument list or the
    # end of the name follows the kernel's own name
    i = name.find(kernel)
    if i < 0:
        return False
    rest = name[i + len(kernel):]
    return rest == "" or rest[0] in "<("


def _short(name: str) -> str:
    name = name.replace("hough::(anonymous namespace)::", "")
    return name.split("(")[0][:60]


def kernel_stats(trace_dir: str):
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise FileNotFoundError("no kernel_stats.csv under %s" % trace_dir)
    rows = list(csv.DictReader(open(files[0])))
    out = []
    for r in rows:
        out.append({"name": _short(r["Name"]), "calls": int(r["Calls"]),
                     "total_ns": float(r["TotalDurationNs"]), "avg_ns": float(r["AverageNs"]),
                     "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"]),
                     "pct": float(r["Percentage"])})
    return out


def dispatches_by_grid(trace_dir: str, kernel: str = "k_find"):
    """{(grid_x, workgroup_x): [durations in ns]} of one kernel's dispatches,
    from the per-dispatch kernel trace."""
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise FileNotFoundError("no kernel_trace.csv under %s" % trace_dir)
    out = defaultdict(list)
    for r in csv.DictReader(open(files[0])):
        if not _is(r["Kernel_Name"], kernel):
            continue
        key = (int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]))
        out[key].append(float(r["End_Timestamp"]) - float(r["Start_Timestamp"]))
    return out


def counter_per_dispatch(pmc_dir: str, counter: str):
    files = glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError("no counter_collection.csv under %s" % pmc_dir)
    per = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(files[0])):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        per[d] += float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    return per, names


def counters_of_largest_grid(pmc_dir: str, kernel: str):
    """{counter: median value over the kernel's dispatches of the largest
    grid} of every counter in one --pmc run, and the number of dispatches."""
    files = glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError("no counter_collection.csv under %s" % pmc_dir)
    val = defaultdict(lambda: defaultdict(float))
    grid = {}
    for r in csv.DictReader(open(files[0])):
        if not _is(r["Kernel_Name"], kernel):
            continue
        d = int(r["Dispatch_Id"])
        val[r["Counter_Name"]][d] += float(r["Counter_Value"])
        grid[d] = int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0)
    if not grid:
        return {}, 0
    gmax = max(grid.values())
    sel = [d for d, g in grid.items() if g == gmax]
    return {c: statistics.median(per[d] for d in sel if d in per) for c, per in val.items()}, len(sel)


# Ratios reported when both counters were collected: (label, numerator,
# denominator, scale).
RATIOS = [
    ("share of wave time waiting on any dependency (SQ_WAIT_ANY / SQ_WAVE_CYCLES)", "SQ_WAIT_ANY",
     "SQ_WAVE_CYCLES", 1.0),
    ("share of wave time issuing any instruction (SQ_ACTIVE_INST_ANY / SQ_WAVE_CYCLES)", "SQ_ACTIVE_INST_ANY",
     "SQ_WAVE_CYCLES", 1.0),
    # SQ_WAVE_CYCLES counts in units of 4 cycles, SQ_BUSY_CU_CYCLES in cycles
    # (SQ_LEVEL_WAVES reads 0 on this device)
    ("mean resident waves per busy CU (4 SQ_WAVE_CYCLES / SQ_BUSY_CU_CYCLES)", "SQ_WAVE_CYCLES",
     "SQ_BUSY_CU_CYCLES", 4.0),
    ("LDS bank-conflict cycles per LDS-active cycle (SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE)",
     "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", 1.0),
    ("VALU instructions per LDS instruction (SQ_INSTS_VALU / SQ_INSTS_LDS)", "SQ_INSTS_VALU", "SQ_INSTS_LDS", 1.0),
    ("VALU share of issued wave instructions (SQ_INSTS_VALU / SQ_INSTS_*)", "SQ_INSTS_VALU", "_ALL_INSTS", 1.0),
]


def traffic(fetch_dir: str, write_dir: str, copy_mib: int, kernel: str = "k_find"):
    """HBM bytes per launch of `kernel` (median over dispatches of the largest
    grid), scaled by the counters of the calibration kernel."""
    copy_bytes = float(copy_mib) * (1 << 20)
    res = {}
    for label, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        per, names = counter_per_dispatch(d, counter)
        copies = [v for k, v in per.items() if COPY_KERNEL in names[k]]
        if not copies:
            raise ValueError("no calibration kernel (%s) in %s" % (COPY_KERNEL, d))
        ref = max(copies) * 1024.0           # counter in KiB
        scale = copy_bytes / ref if ref > 0 else float("nan")
        mine = [v for k, v in per.items() if _is(names[k], kernel)]
        big = max(mine)
        batched = [v for v in mine if v >= 0.5 * big]
        res[label + "_bytes"] = statistics.median(batched) * 1024.0 * scale
        res[label + "_scale"] = scale
        res[label + "_dispatches"] = len(batched)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--counters", action="append", default=[], help="a further --pmc run directory")
    ap.add_argument("--name", required=True, help="summary base name under profiles/")
    ap.add_argument("--command", action="append", default=[], help="a command line that produced the data")
    ap.add_argument("--note", default="")
    ap.add_argument("--kernel", default="k_find", help="kernel whose dispatches and traffic are summarised")
    ap.add_argument("--source", default="hough_kernels.hip", help="its source file under csrc/")
    args = ap.parse_args()

    stats = kernel_stats(args.trace)
    h = kernel_source_hash(args.source)
    K = args.kernel
    lines = ["# %s" % args.name, ""]
    if args.note:
        lines += [args.note, ""]
    lines += ["Kernel source hash (sha256/16 of csrc/%s): `%s`" % (args.source, h), "", "Commands:", ""]
    lines += ["    %s" % c for c in args.command] + [""]
    lines += ["| kernel | calls | avg us | min us | max us | total ms | % |", "|---|---|---|---|---|---|---|"]
    for r in stats:
        lines.append("| %s | %d | %.2f | %.2f | %.2f | %.3f | %.1f |" % (
            r["name"], r["calls"], r["avg_ns"] / 1e3, r["min_ns"] / 1e3, r["max_ns"] / 1e3,
            r["total_ns"] / 1e6, r["pct"]))
    grids = dispatches_by_grid(args.trace, K)
    lines += ["", "%s dispatches by launch size (the batched call is the largest grid):" % K, "",
              "| workgroups | threads/wg | dispatches | avg us | min us | max us |", "|---|---|---|---|---|---|"]
    for (gx, wx), d in sorted(grids.items(), key=lambda kv: -kv[0][0]):
        lines.append("| %d | %d | %d | %.2f | %.2f | %.2f |" % (gx // wx, wx, len(d), statistics.mean(d) / 1e3,
                                                              min(d) / 1e3, max(d) / 1e3))
    kv = {"kernel_sha256_16": h}
    big = max(grids) if grids else None
    if big:
        kv["batched_%s_avg_us" % K] = "%.2f" % (statistics.mean(grids[big]) / 1e3)
    if args.fetch and args.write and args.copy_mib:
        t = traffic(args.fetch, args.write, args.copy_mib, K)
        lines += ["", "HBM traffic of the batched %s launch (median over %d dispatches), from "
                  "FETCH_SIZE / WRITE_SIZE scaled by a %d MiB device copy (scale fetch %.3f, write %.3f):"
                  % (K, t["fetch_dispatches"], args.copy_mib, t["fetch_scale"], t["write_scale"]), "",
                  "| read bytes | written bytes | total |", "|---|---|---|",
                  "| %.0f | %.0f | %.0f |" % (t["fetch_bytes"], t["write_bytes"], t["fetch_bytes"] + t["write_bytes"])]
        kv.update({"fetch_bytes_per_launch": "%.0f" % t["fetch_bytes"],
                   "write_bytes_per_launch": "%.0f" % t["write_bytes"]})
    if args.counters:
        allc = {}
        nd = 0
        for d in args.counters:
            c, n = counters_of_largest_grid(d, K)
            allc.update(c)
            nd = max(nd, n)
        insts = [k for k in allc if k.startswith("SQ_INSTS_")]
        if insts:
            allc["_ALL_INSTS"] = sum(allc[k] for k in insts)
        lines += ["", "Counters of the batched %s launch (median over %d largest-grid dispatches, summed over "
                  "the device):" % (K, nd), "", "| counter | value |", "|---|---|"]
        for k in sorted(c for c in allc if not c.startswith("_")):
            lines.append("| %s | %.0f |" % (k, allc[k]))
            kv["pmc_" + k] = "%.0f" % allc[k]
        rows = [(lab, allc[a] / allc[b] * sc) for lab, a, b, sc in RATIOS if a in allc and allc.get(b)]
        if rows:
            lines += ["", "| ratio | value |", "|---|---|"] + ["| %s | %.4f |" % r for r in rows]
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", args.name + ".md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(ROOT, "profiles", args.name + ".txt"), "w") as f:
        for k, v in kv.items():
            f.write("%s: %s\n" % (k, v))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
