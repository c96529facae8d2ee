"""Summaries of rocprofv3 output (kernel-trace stats and PMC byte counters).

Reads the CSV files rocprofv3 writes with ``--output-format csv``:
  <name>_kernel_stats.csv          (from --kernel-trace --stats)
  <name>_counter_collection.csv    (from --pmc ...)
and prints short text tables for ``profiles/``.

    python paper_1907_09575_amd/rocprof_summary.py stats DIR/NAME_kernel_stats.csv
    python paper_1907_09575_amd/rocprof_summary.py pmc DIR/NAME_counter_collection.csv COUNTER
    python paper_1907_09575_amd/rocprof_summary.py launches DIR/NAME_kernel_trace.csv [SUBSTRING]
    python paper_1907_09575_amd/rocprof_summary.py traffic FETCH.csv WRITE.csv BENCH.json LABEL OUT.json
    python paper_1907_09575_amd/rocprof_summary.py ratios DIR/NAME_counter_collection.csv

``ratios`` averages every counter of a run per (kernel, grid) and prints the
LDS bank-conflict rate (SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE: the share of
LDS-active cycles stalled by bank conflicts) and the L2 hit rate
(TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)) where those counters are present.

``launches`` groups the kernel trace by (kernel, grid size), which separates
the launch classes that share one kernel instantiation.

``traffic`` turns one FETCH_SIZE run and one WRITE_SIZE run of
``bench.py --copy-calibration`` into bytes per launch of the count class
LABEL (e.g. count:wg_large): both counters are scaled by what they read for
the 1 GiB calibration copy, and the launch is found by kernel name and grid
size (the class's work-groups from the bench line, 64 threads per wave).
FETCH_SIZE and WRITE_SIZE count the L2's requests to the fabric: L2 misses,
served by the Infinity Cache (MALL) or by HBM, so the figure is reported as
fabric traffic (an upper bound on HBM bytes, not a DRAM measurement).

The PMC summary also reports the counter for the largest plain copy kernel in
the same run (a known-size calibration copy), so byte counts can be scaled.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
CALIBRATION_BYTES = 1 << 30


def source_digest() -> str:
    """Digest of the count-kernel sources a traffic measurement belongs to."""
    h = hashlib.sha256()
    for name in ("tc_count.hip", "tc_internal.h"):
        with open(os.path.join(_CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


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


def launches(path: str, top: int = 25, only: str = ""):
    per = defaultdict(list)
    for r in csv.DictReader(open(path)):
        name = r.get("Kernel_Name", "")
        if only and only not in name:
            continue
        grid = int(r.get("Grid_Size_X", r.get("Grid_Size", 0)) or 0)
        dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        per[(name, grid)].append(dur)
    items = sorted(per.items(), key=lambda kv: -sum(kv[1]))
    lines = ["%-52s %11s %6s %12s %12s" % ("kernel", "grid", "calls", "total_ms", "avg_ms")]
    for (name, grid), d in items[:top]:
        lines.append("%-52s %11d %6d %12.3f %12.4f" % (short_name(name)[:52], grid, len(d), sum(d) / 1e6,
                                                      sum(d) / len(d) / 1e6))
    return "\n".join(lines)


def ratios(path: str, top: int = 20):
    per = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(path)):
        name = r.get("Kernel_Name", r.get("kernel_name"))
        grid = int(float(r.get("Grid_Size", r.get("grid_size", 0)) or 0))
        cn = r.get("Counter_Name", r.get("counter_name"))
        per[(name, grid)][cn].append(float(r.get("Counter_Value", r.get("counter_value", 0))))
    def avg(d, k):
        v = d.get(k)
        return sum(v) / len(v) if v else None
    rows = []
    for (name, grid), d in per.items():
        bc, act = avg(d, "SQ_LDS_BANK_CONFLICT"), avg(d, "SQ_LDS_IDX_ACTIVE")
        hit, miss = avg(d, "TCC_HIT_sum"), avg(d, "TCC_MISS_sum")
        weight = act if act is not None else (hit or 0) + (miss or 0)
        rows.append((weight, name, grid, len(next(iter(d.values()))),
                     None if not act else bc / act,
                     None if hit is None or miss is None or hit + miss == 0 else hit / (hit + miss)))
    rows.sort(key=lambda r: -r[0])
    lines = ["%-52s %11s %5s %16s %10s" % ("kernel", "grid", "n", "lds_conflict", "l2_hit")]
    for _, name, grid, n, lc, l2 in rows[:top]:
        lines.append("%-52s %11d %5d %16s %10s" % (short_name(name)[:52], grid, n,
                                                   "-" if lc is None else "%.4f" % lc,
                                                   "-" if l2 is None else "%.4f" % l2))
    return "\n".join(lines)


def _counter_rows(path, counter):
    out = []
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", r.get("counter_name")) != counter:
            continue
        out.append((r.get("Kernel_Name", r.get("kernel_name")), int(float(r.get("Grid_Size", r.get("grid_size", 0)))),
                    float(r.get("Counter_Value", r.get("counter_value", 0)))))
    return out


def traffic(fetch_csv, write_csv, bench_json, label, out_json, commands=()):
    bench = json.loads(open(bench_json).read().strip().splitlines()[-1])
    cls = label.split(":", 1)[1]
    waves = 8 if cls in ("wg_huge", "wg_giant") else 4
    grid = bench["classes"][cls]["workgroups"] * 64 * waves
    kname = "k_count_packs" if cls.startswith("pack") else "k_count_items"
    res = {"kernel": label, "workload": bench["config"]["workload"] + " seed %d" % bench["config"]["seed"],
           "source_digest": source_digest()}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _counter_rows(path, counter)
        # calibration: the largest plain copy kernel of the run (1 GiB each way)
        copies = [v for k, g, v in rows if "copy" in k.lower() and "count" not in k.lower()]
        assert copies, "no calibration copy in %s" % path
        cal = max(copies)
        sel = [v for k, g, v in rows if short_name(k).startswith(kname) and "<0" in k and g == grid]
        assert sel, "no launch of %s with grid %d in %s" % (kname, grid, path)
        res[key + "_kib_per_launch"] = sum(sel) / len(sel)
        res.setdefault("calibration", {"copy_bytes": CALIBRATION_BYTES})
        res["calibration"][key + "_kib"] = cal
        res["calibration"][key + "_scale"] = CALIBRATION_BYTES / 1024.0 / cal
    fab = sum(res[k + "_kib_per_launch"] * 1024.0 * res["calibration"][k + "_scale"] for k in ("fetch", "write"))
    res["fabric_bytes_per_launch"] = fab
    res["note"] = ("FETCH_SIZE + WRITE_SIZE: the L2's requests to the fabric (misses served by the Infinity "
                   "Cache or HBM), scaled by a 1 GiB copy in the same run")
    res["algorithmic_bytes_per_launch"] = bench["roofline"]["algorithmic_bytes_per_launch"] \
        if bench["roofline"].get("kernel") == label else None
    res["commands"] = list(commands)
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    return res


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(kernel_stats(argv[1]))
    elif len(argv) >= 2 and argv[0] == "launches":
        print(launches(argv[1], only=argv[2] if len(argv) >= 3 else ""))
    elif len(argv) >= 2 and argv[0] == "ratios":
        print(ratios(argv[1]))
    elif len(argv) >= 3 and argv[0] == "pmc":
        print(pmc(argv[1], argv[2]))
    elif len(argv) >= 6 and argv[0] == "traffic":
        print(json.dumps(traffic(argv[1], argv[2], argv[3], argv[4], argv[5], argv[6:]), indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
