"""Summaries of rocprofv3 output (kernel-trace stats and PMC byte counters).

Reads the CSV files rocprofv3 writes with ``--output-format csv``:
  <name>_kernel_stats.csv          (from --kernel-trace --stats)
  <name>_counter_collection.csv    (from --pmc ...)
and prints short text tables for ``profiles/``.

    python -m paper_1907_09575_amd.rocprof_summary stats DIR/NAME_kernel_stats.csv
    python -m paper_1907_09575_amd.rocprof_summary pmc DIR/NAME_counter_collection.csv COUNTER

The PMC summary also reports the counter for the largest plain copy kernel in
the same run (a known-size calibration copy), so byte counts can be scaled.
"""
from __future__ import annotations

import csv
import sys
from collections import defaultdict


def short_name(name: str) -> str:
    for p in ("void ", "tc::(anonymous namespace)::", "tc::"):
        name = name.replace(p, "")
    return name.split("(")[0]


def kernel_stats(path: str, top: int = 30):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        name = r.get("Name") or r.get("KernelName") or r.get("name")
        calls = int(float(r.get("Calls", r.get("calls", 0))))
        total = float(r.get("TotalDurationNs", r.get("total_duration", 0)))
        avg = float(r.get("AverageNs", total / max(calls, 1)))
        pct = float(r.get("Percentage", 0))
        out.append((total, calls, avg, pct, name))
    out.sort(reverse=True)
    lines = ["%-64s %6s %12s %12s %7s" % ("kernel", "calls", "total_ms", "avg_ms", "pct")]
    for total, calls, avg, pct, name in out[:top]:
        lines.append("%-64s %6d %12.3f %12.4f %7.2f" % (short_name(name)[:64], calls, total / 1e6,
                                                        avg / 1e6, pct))
    return "\n".join(lines)


def pmc(path: str, counter: str):
    rows = list(csv.DictReader(open(path)))
    per = defaultdict(list)
    for r in rows:
        if r.get("Counter_Name", r.get("counter_name")) != counter:
            continue
        name = r.get("Kernel_Name", r.get("kernel_name"))
        grid = r.get("Grid_Size", r.get("grid_size", ""))
        lds = r.get("LDS_Block_Size", r.get("lds_block_size", ""))
        val = float(r.get("Counter_Value", r.get("counter_value", 0)))
        per[(name, grid, lds)].append(val)
    lines = ["%-64s %10s %8s %6s %16s" % ("kernel", "grid", "lds", "n", counter + "_KiB_avg")]
    items = sorted(per.items(), key=lambda kv: -sum(kv[1]) / len(kv[1]))
    for (name, grid, lds), vals in items[:25]:
        lines.append("%-64s %10s %8s %6d %16.1f" % (short_name(name)[:64], grid, lds, len(vals),
                                                   sum(vals) / len(vals)))
    return "\n".join(lines)


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(kernel_stats(argv[1]))
    elif len(argv) >= 3 and argv[0] == "pmc":
        print(pmc(argv[1], argv[2]))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
