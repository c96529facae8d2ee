#!/usr/bin/env python3
"""Benchmark: exact triangle counting of an RMAT scale-24 graph on one MI355X.

One step = the whole single-graph hot path on a resident input: tc_preprocess
(raw int32 edge list in HBM -> simple graph -> degree order -> upper CSR ->
tasks and work items) + tc_count (exact int64 total) + tc_graph_free. The
input is a seeded synthetic RMAT graph (a, b, c, d = 0.57, 0.19, 0.19, 0.05,
edge factor 16), the shape of the paper's Graph500 inputs. `value` is raw input
pairs per second over whole steps; the count phase alone (the paper's tct) and
preprocessing (ppt) are reported beside it.

Roofline: every library launch in the timed steps is bracketed by HIP events
(tc_timer_attach) on the stream it runs on; the dominant kernel is the count
class with the most algorithmic bytes per launch (4 per probe + 4 per
hashed-row key + 12 per task + 32 per row of its class), and those bytes over
its average event time give `achieved`. (The light count classes run on a
side stream beside the heavy ones, so per-kernel event times overlap; the
count phase's own wall time, `count_ms`, comes from events around tc_count.) `count_median_ms` times tc_count alone on the resident graph
(2 warm-ups, median of 11).

Beside the step: one rank's block of the 13 x 13 grid (`block`), the
ablations of Section 7.3 and the per-rank tables of Section 7.2
(`ablation`), one step at RMAT scale 26 (`large`), per-edge
support in both modes on a resident RMAT scale-20 graph (`support`), the
batched form against the plain launch loop (`batched`) and the served form
against a plain FIFO (`served`); each is skipped with its --no-* flag.

cpu_baseline: the CPU oracle (plain C, list-based intersection) timed end to
end (its own preprocessing + count) on a bounded sample of the same input:
the first 1/8 of its raw pairs (--cpu-full adds the whole input).

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--scale 24]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact-count edges/s + HBM GB/s vs peak, RMAT scale 24; batched/served vs plain"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_count_rmat24.json")


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--scale", type=int, default=24)
    p.add_argument("--edge-factor", type=int, default=16)
    p.add_argument("--seed", type=int, default=1)
    p.add_argument("--cpu-sample", type=int, default=8,
                   help="cpu_baseline runs the oracle on the first 1/N of the input's raw pairs")
    p.add_argument("--cpu-full", action="store_true", help="also run the oracle on the whole input")
    p.add_argument("--cpu-threads", type=int, default=16,
                   help="oracle threads (the host cores allotted to one GPU)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run one plain 1 GiB device copy first (PMC byte-counter calibration)")
    p.add_argument("--gen-threads", type=int, default=16)
    p.add_argument("--tuning-file", default=None,
                   help="tuning table to load (default: paper_1907_09575_amd/tuning/<arch>_<CUs>cu.json if present)")
    p.add_argument("--no-tuning-file", action="store_true", help="run with the default thresholds")
    p.add_argument("--kernels-json", default=None, help="write the full per-kernel timer summary here")
    p.add_argument("--no-block", action="store_true", help="skip the 13x13 block grid of the graph")
    p.add_argument("--block-q", type=int, default=13)
    p.add_argument("--no-ablation", action="store_true", help="skip the ablations and per-rank tables")
    p.add_argument("--ablation-q", default="4,5,6,13", help="grid sizes of the per-rank tables")
    p.add_argument("--no-large", action="store_true", help="skip the RMAT scale 26 step")
    p.add_argument("--large-scale", type=int, default=26)
    p.add_argument("--no-support", action="store_true", help="skip the per-edge support leg")
    p.add_argument("--support-scale", type=int, default=20)
    p.add_argument("--no-batch", action="store_true", help="skip batched vs plain")
    p.add_argument("--batch-graphs", type=int, default=4096)
    p.add_argument("--batch-schedule", default=None,
                   help="tc_batch_create schedule JSON to use instead of autotuning (e.g. for profiles)")
    p.add_argument("--no-serve", action="store_true", help="skip served vs plain FIFO")
    p.add_argument("--serve-requests", type=int, default=10000)
    p.add_argument("--serve-warmup", type=int, default=1000)
    p.add_argument("--serve-slots", type=int, default=64)
    p.add_argument("--serve-prep-threads", type=int, default=8)
    p.add_argument("--serve-ticks", type=int, default=0, help="server ticks in flight (0: the library's default)")
    return p.parse_args()


def count_kernel_bytes(stats: dict, cls: str) -> int:
    """Algorithmic bytes of one launch of count:<cls>: every probe reads one
    int32 of U (4 B); every hashed row is read once to build its table (4 B per
    key) and its row bounds and task range once (32 B); every task reads its
    start (4 B) and its prefix entry (8 B)."""
    s = stats[cls]
    return 4 * s["probes"] + 4 * s["table_keys"] + 12 * s["tasks"] + 32 * s["rows"]


def preprocess_bytes(n: int, m_raw: int, m: int, tasks: int) -> int:
    """Algorithmic bytes of tc_preprocess (the paper's ppt): read the raw pairs
    once (8 per pair); an LSD radix sort moves 16 bytes per key per 8-bit
    pass (read + write of an 8-byte key) over ceil(2 log2 n / 8) passes: the
    dedup sort over the raw pairs and the orient sort over the simple edges;
    the rank sort over the n vertices takes ceil(log2 n / 8) passes; then the
    CSR (4 per edge, 8 per row pointer, 4 per rank-map entry) and the task
    lists (4 + 8 per task) are written once."""
    s = max(1, (n - 1).bit_length())
    p_edge = (2 * s + 7) // 8
    p_rank = (s + 7) // 8
    return (8 * m_raw + 16 * p_edge * m_raw + 16 * p_rank * n + 16 * p_edge * m
            + 4 * m + 8 * (n + 1) + 4 * n + 12 * tasks)


def measure_copy_gbs(dev, nbytes=1 << 31, reps=5):
    """On-box reference bandwidth: a plain device-to-device copy of nbytes
    (read + write bytes per second, GB/s, best of reps), reported beside the
    published peak."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.synchronize()
    return round(2 * nbytes / (best / 1e3) / 1e9, 1)


def load_traffic(kernel: str):
    """Fabric bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE: L2 misses,
    served by the Infinity Cache or HBM) from the committed PMC summary, if it
    was taken on the current count-kernel sources; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_1907_09575_amd.rocprof_summary import source_digest
    if t.get("kernel") != kernel or t.get("source_digest") != source_digest():
        return None
    return t.get("fabric_bytes_per_launch")


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(scale: int, edge_factor: int, seed: int, threads: int, frac: int, full: bool):
    """The CPU oracle (plain C: qsort preprocessing on one thread, list-based
    intersection on `threads` threads) end to end on a bounded sample of the
    benchmark's own input: the first 1/frac of the RMAT stream's raw pairs
    (the pairs are drawn independently, so a prefix is an RMAT sample on the
    same vertex space). With full=True the oracle also runs on the whole
    input (minutes)."""
    import graphgen
    import oracle

    src, dst = graphgen.rmat(scale, edge_factor=edge_factor, seed=seed, threads=threads)
    n = 1 << scale
    k = len(src) // frac
    ss, ds = src[:k].copy(), dst[:k].copy()

    def run(s, d, label):
        t0 = time.perf_counter()
        U = oracle.preprocess(s, d, n)
        t1 = time.perf_counter()
        print("cpu baseline %s: oracle preprocessing %.1f s" % (label, t1 - t0), file=sys.stderr, flush=True)
        T = oracle.count(U, threads=threads)
        t2 = time.perf_counter()
        print("cpu baseline %s: oracle count %.1f s" % (label, t2 - t1), file=sys.stderr, flush=True)
        return U, T, t1 - t0, t2 - t1

    U, T, tp, tc_ = run(ss, ds, "sample")
    out = {
        "value": k / (tp + tc_),
        "unit": "edges/s",
        "cores": threads,
        "kind": "oracle",
        "host_cpu": host_cpu_model(),
        "host_cpu_count": os.cpu_count(),
        "count_edges_per_s": U.m / tc_,
        "sample": "first 1/%d of the RMAT scale %d raw pairs (%d pairs, n = 2^%d; m = %d, T = %d): oracle "
                  "preprocessing %.2f s on one thread (qsort) + count %.2f s on %d threads; threads = the "
                  "host cores allotted to one GPU (%d of the %s this host reports)" % (
                      frac, scale, k, scale, U.m, T, tp, tc_, threads, threads, os.cpu_count()),
    }
    if full:
        del U
        U, T, tp, tc_ = run(src, dst, "full")
        out["full"] = {"pairs": len(src), "m": U.m, "triangles": T, "preprocess_s": round(tp, 2),
                       "count_s": round(tc_, 2), "edges_per_s": len(src) / (tp + tc_),
                       "count_edges_per_s": U.m / tc_}
    return out


def pct(vals, q):
    import numpy as np
    return float(np.percentile(np.asarray(vals, dtype=np.float64), q)) if len(vals) else None


def bench_block(tc, g, T, q):
    """One rank's block of the q x q cyclic grid at the graph's real shape:
    every rank once (their sum must be T, per-shift parts must sum to each
    block), then block (0, 0) and the slowest rank timed again."""
    import torch
    ps = torch.empty(q, dtype=torch.int64, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    total, times = 0, {}
    for x in range(q):
        for y in range(q):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tc.tc_block_count(g, q, x, y, cnt, ps)
            torch.cuda.synchronize()
            times[(x, y)] = time.perf_counter() - t0
            b = int(cnt.item())
            assert int(ps.sum().item()) == b, "per-shift parts do not sum to block (%d, %d)" % (x, y)
            total += b
    assert total == T, "blocks sum to %d, not T = %d" % (total, T)
    slow = max(times, key=times.get)
    out = {"q": q, "grid_sum_equals_T": True, "grid_wall_s": round(sum(times.values()), 3)}
    for name, (x, y) in (("block_0_0", (0, 0)), ("block_slowest", slow)):
        timer = tc.Timer(capacity=4096)
        reps = 3
        with timer:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                tc.tc_block_count(g, q, x, y, cnt, ps)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / reps
        k = timer.summary()
        timer.free()
        count_ms = sum(v["total_ms"] for kk, v in k.items() if kk.startswith("block:")) / reps
        st = tc.tc_block_stats(g, q, x, y).cpu().tolist()
        # algorithmic bytes of the rank's count kernels, a lower bound: 4 per
        # probe and 12 per task (its hashed rows' keys and bounds not counted)
        alg = 4 * st[1] + 12 * st[0]
        out[name] = {"x": x, "y": y, "count": int(cnt.item()), "per_shift": ps.cpu().tolist(),
                     "ms_total": round(wall * 1e3, 3), "count_kernel_ms": round(count_ms, 3),
                     "tasks": st[0], "probes": st[1], "alg_bytes_lb": alg,
                     "count_alg_GBps": round(alg / (count_ms / 1e3) / 1e9, 1) if count_ms > 0 else None,
                     "count_frac": round(alg / (count_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if count_ms > 0 else None}
    return out


def bench_ablation(tc, g, T, qs):
    """Section 7.3 and Section 7.2 on one GPU, on the benchmark's graph.
    Ablations: tc_count on the graph and on its variants without each of
    Section 5.2's optimizations (<i,j,k> enumeration instead of <j,i,k>, no
    doubly sparse traversal, multiplicative hashing instead of the direct
    AND), each one warm-up and the median of 5 (HIP events), with its probes,
    tasks and the count checked against T. Per-rank tables for every q: all
    q x q ranks' work (tc_block_stats): task imbalance (max / average over
    ranks, Section 7.2's task-count imbalance), per-shift imbalance (max /
    average of the probes of a (rank, shift) pair, the work behind Table
    "r_l_imb"), and the intersections performed when the shifts run one by
    one, summed over ranks and shifts (Table "opcount"), with its growth
    from the previous q."""
    import numpy as np
    import torch
    out = {}
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    base_ms = None
    for name, flags in (("jik", 0), ("ijk", tc.TC_VARIANT_IJK), ("no_dcsr", tc.TC_VARIANT_NO_DCSR),
                        ("mul_hash", tc.TC_VARIANT_MUL_HASH)):
        print("ablation %s ..." % name, file=sys.stderr, flush=True)
        V = g if flags == 0 else tc.tc_graph_variant(g, flags)
        runs = []
        for r in range(6):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            tc.tc_count(V, cnt)
            e1.record()
            e1.synchronize()
            assert int(cnt.item()) == T, "%s counts %d, not T = %d" % (name, int(cnt.item()), T)
            if r:
                runs.append(e0.elapsed_time(e1))
        info = V.info()
        med = float(np.median(runs))
        base_ms = med if base_ms is None else base_ms
        out[name] = {"count_ms": round(med, 3), "probes": info["probes"], "tasks": info["tasks"],
                     "time_vs_jik": round(med / base_ms, 3)}
        if flags:
            V.free()
    grid = {}
    prev = None
    for q in qs:
        print("rank tables q=%d ..." % q, file=sys.stderr, flush=True)
        rows = []
        for x in range(q):
            for y in range(q):
                rows.append(tc.tc_block_stats(g, q, x, y).cpu().numpy())
        a = np.stack(rows)
        tasks, probes = a[:, 0], a[:, 1]
        sp, stsk = a[:, 2:2 + q], a[:, 2 + q:]
        inter = int(stsk.sum())
        grid[str(q)] = {"ranks": q * q, "tasks_total": int(tasks.sum()), "probes_total": int(probes.sum()),
                        "task_imbalance": round(float(tasks.max() / tasks.mean()), 4),
                        "probe_imbalance": round(float(probes.max() / probes.mean()), 4),
                        "shift_probe_imbalance": round(float(sp.max() / sp.mean()), 4),
                        "intersections": inter,
                        "intersection_growth": round(inter / prev - 1, 4) if prev else None}
        prev = inter
    out["rank_tables"] = grid
    return out


def bench_large(tc, args):
    """RMAT scale 26 (2^30 raw pairs, the shape of the paper's g500-s26
    input): one warm-up, then one timed preprocess + count step, the count
    alone on the resident graph (median of 5, HIP events) and the dominant
    count kernel against the HBM roofline. T is checked against the value the
    oracle stored for this input (tests/golden)."""
    import numpy as np
    import torch
    import graphgen
    scale = args.large_scale
    n = 1 << scale
    print("large: generating RMAT scale %d ..." % scale, file=sys.stderr, flush=True)
    s, d = graphgen.rmat(scale, edge_factor=args.edge_factor, seed=args.seed, threads=args.gen_threads)
    m_raw = len(s)
    src, dst = torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()
    del s, d
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    g = tc.tc_preprocess(src, dst, n)
    tc.tc_count(g, out)
    torch.cuda.synchronize()
    g.free()
    print("large: timed step ...", file=sys.stderr, flush=True)
    timer = tc.Timer(capacity=4096)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    with timer:
        t0 = time.perf_counter()
        ev[0].record()
        g = tc.tc_preprocess(src, dst, n)
        ev[1].record()
        tc.tc_count(g, out)
        ev[2].record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    kern = timer.summary()
    timer.free()
    T = int(out.item())
    info = g.info()
    cstats = tc.tc_graph_class_stats(g)
    runs = []
    for r in range(7):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        tc.tc_count(g, out)
        e1.record()
        e1.synchronize()
        assert int(out.item()) == T
        if r >= 2:
            runs.append(e0.elapsed_time(e1))
    g.free()
    del src, dst
    torch.cuda.empty_cache()
    step_ms = (t1 - t0) * 1e3
    count_ms = ev[1].elapsed_time(ev[2])  # wall time of the count phase on the stream
    counts = {k: v for k, v in kern.items() if k.startswith("count:")}
    dom = max((k for k in counts if cstats[k.split(":", 1)[1]]["rows"]),
              key=lambda k: count_kernel_bytes(cstats, k.split(":", 1)[1]))
    cls = dom.split(":", 1)[1]
    achieved = count_kernel_bytes(cstats, cls) / (counts[dom]["avg_ms"] / 1e3) / 1e9
    res = {"workload": "rmat%d_ef%d_preprocess_count" % (scale, args.edge_factor), "n": n, "m_raw": m_raw,
           "m": info["m"], "triangles": T, "wedges_plus": info["wedges_plus"], "step_ms": round(step_ms, 3),
           "edges_per_s": m_raw / (step_ms / 1e3), "preprocess_ms": round(step_ms - count_ms, 3),
           "count_ms": round(count_ms, 3), "count_median_ms": round(float(np.median(runs)), 3),
           "count_median_edges_per_s": info["m"] / (float(np.median(runs)) / 1e3),
           "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "avg_launch_ms": round(counts[dom]["avg_ms"], 4),
                        "algorithmic_bytes_per_launch": count_kernel_bytes(cstats, cls)},
           "kernels_top": {k: {"total_ms": round(v["total_ms"], 3), "launches": v["launches"]}
                           for k, v in sorted(((k, v) for k, v in kern.items() if not k.startswith("_")),
                                              key=lambda kv: -kv[1]["total_ms"])[:10]}}
    fx = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                      "rmat%d_seed%d.json" % (scale, args.seed))
    if os.path.exists(fx) and args.edge_factor == 16:
        with open(fx) as f:
            want = json.load(f)
        res["oracle_triangles_equal"] = want["triangles"] == T and want["m"] == info["m"]
    return res


def bench_support(tc, args):
    """Per-edge support (Eq. 1) on a resident RMAT graph (default scale 20,
    the support workload): tc_count, then tc_edge_support in FULL and ORIENTED
    mode, each 2 warm-ups and the median of 5 (HIP events around the call on
    the current stream). Every run is checked: sum of FULL = 3T, sum of
    ORIENTED = T. Algorithmic bytes: the count's (count_kernel_bytes over the
    classes), plus 4m to clear the support array and 4m to write it back, plus
    for FULL the H_b edge ids read from the tables (4m) and two remote int32
    read-modify-writes per triangle (16 T)."""
    import numpy as np
    import torch

    import graphgen
    dev = torch.device("cuda", 0)
    scale = args.support_scale
    src_h, dst_h = graphgen.rmat(scale, edge_factor=args.edge_factor, seed=args.seed,
                                 threads=args.gen_threads)
    m_raw = len(src_h)
    src = torch.from_numpy(src_h).to(dev)
    dst = torch.from_numpy(dst_h).to(dev)
    del src_h, dst_h
    g = tc.tc_preprocess(src, dst, 1 << scale)
    del src, dst
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    tc.tc_count(g, cnt)
    torch.cuda.synchronize()
    T = int(cnt.item())
    m = g.info()["m"]
    cstats = tc.tc_graph_class_stats(g)
    b_count = sum(count_kernel_bytes(cstats, c) for c in cstats if cstats[c]["rows"])
    sup = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    out = {"workload": "rmat%d_ef%d_support" % (scale, args.edge_factor), "n": 1 << scale,
           "m_raw": m_raw, "m": m, "triangles": T}
    for name, mode, total, extra in (("full", tc.TC_SUPPORT_FULL, 3 * T, 12 * m + 16 * T),
                                     ("oriented", tc.TC_SUPPORT_ORIENTED, T, 8 * m)):
        runs = []
        timer = tc.Timer(capacity=4096)
        with timer:
            for r in range(7):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                tc.tc_edge_support(g, mode, support=sup)
                e1.record()
                e1.synchronize()
                s = int(sup[:m].sum(dtype=torch.int64).item())
                assert s == total, "%s support sums to %d, not %d" % (name, s, total)
                if r >= 2:
                    runs.append(e0.elapsed_time(e1))
        k = timer.summary()
        timer.free()
        kern_ms = sum(v["total_ms"] for kk, v in k.items() if kk.startswith("support_")) / 7
        med = float(np.median(runs))
        alg = b_count + extra
        out[name] = {"median_ms": round(med, 4), "kernel_ms": round(kern_ms, 4),
                     "edges_per_s": m / (med / 1e3), "raw_edges_per_s": m_raw / (med / 1e3),
                     "alg_bytes": alg, "alg_GBps": round(alg / (med / 1e3) / 1e9, 1),
                     "frac": round(alg / (med / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "sum_check": "3T" if name == "full" else "T"}
    # the plain count on the same resident graph, for comparison
    runs = []
    for r in range(7):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        tc.tc_count(g, cnt)
        e1.record()
        e1.synchronize()
        assert int(cnt.item()) == T
        if r >= 2:
            runs.append(e0.elapsed_time(e1))
    out["count_median_ms"] = round(float(np.median(runs)), 4)
    # the uses of the counts (Section 1) on the same graph: per-vertex counts
    # and clustering coefficients (checked: sum of t = 3T), trussness
    t0 = time.perf_counter()
    sums = torch.empty(2, dtype=torch.int64, device=dev)
    cc, _, _ = tc.tc_clustering(g, sums=sums)
    torch.cuda.synchronize()
    t_cc = time.perf_counter() - t0
    assert int(sums[0].item()) == 3 * T
    t0 = time.perf_counter()
    tau, kmax = tc.tc_truss(g)
    torch.cuda.synchronize()
    t_truss = time.perf_counter() - t0
    out["clustering"] = {"ms": round(t_cc * 1e3, 3), "transitivity": int(sums[0].item()) / int(sums[1].item()),
                         "avg_local": float(cc.mean().item())}
    out["truss"] = {"ms": round(t_truss * 1e3, 3), "kmax": kmax,
                    "edges_in_kmax_truss": int((tau == kmax).sum().item())}
    del cc, tau
    g.free()
    del sup
    torch.cuda.empty_cache()
    return out


def bench_batch(tc, args):
    """4096 uneven graphs: one persistent launch (autotuned schedule) against
    the plain loop of tc_count calls on one stream, both on preprocessed
    handles; counts must agree exactly."""
    import ctypes
    import numpy as np
    import torch
    import graphgen
    specs = graphgen.batch_specs(args.batch_graphs)
    print("batch: generating %d graphs ..." % len(specs), file=sys.stderr, flush=True)
    lists = graphgen.generate_many(specs, args.gen_threads)
    m_raw = sum(len(a) for a, _ in lists)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    graphs = []
    for sp, (a, b) in zip(specs, lists):
        graphs.append(tc.tc_preprocess(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), sp.n))
    torch.cuda.synchronize()
    pre_s = time.perf_counter() - t0
    del lists
    m_total = sum(g.m for g in graphs)
    n = len(graphs)
    stream = torch.cuda.current_stream()
    sptr = ctypes.c_void_p(stream.cuda_stream)
    plain = torch.empty(n, dtype=torch.int64, device="cuda")
    base = plain.data_ptr()
    handles = [g.handle for g in graphs]
    lib = tc._lib

    def plain_loop():
        for i in range(n):
            lib.tc_count(handles[i], ctypes.c_void_p(base + 8 * i), sptr)

    plain_loop()
    torch.cuda.synchronize()
    plain_times = []
    for _ in range(3):
        t0 = time.perf_counter()
        plain_loop()
        torch.cuda.synchronize()
        plain_times.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    if args.batch_schedule:
        tune = {"best": json.loads(args.batch_schedule), "candidates": []}
    else:
        tune = tc.tc_batch_autotune(graphs)
    tune_s = time.perf_counter() - t0
    plan = tc.tc_batch_create(graphs, tuning=tune["best"])
    desc = tc.tc_batch_describe(plan)
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    tc.tc_batch_count(plan, out)
    torch.cuda.synchronize()
    reps = 5
    timer = tc.Timer(capacity=64)
    with timer:
        t0 = time.perf_counter()
        for _ in range(reps):
            tc.tc_batch_count(plan, out)
        torch.cuda.synchronize()
        batch_s = (time.perf_counter() - t0) / reps
    k = timer.summary()
    timer.free()
    assert torch.equal(out, plain), "batched counts differ from the plain loop"
    kern_ms = k.get("batch:graph", {}).get("avg_ms")
    bytes_total = 0
    for g in graphs:
        cs = tc.tc_graph_class_stats(g)
        bytes_total += sum(count_kernel_bytes(cs, c) for c in cs if cs[c]["rows"])
    plain_s = min(plain_times)
    res = {
        "graphs": n, "m_raw": m_raw, "m": m_total, "triangles": int(out.sum().item()),
        "preprocess_s": round(pre_s, 3),
        "plain_loop_ms": round(plain_s * 1e3, 3), "batched_ms": round(batch_s * 1e3, 3),
        "plain_graphs_per_s": n / plain_s, "batched_graphs_per_s": n / batch_s,
        "plain_edges_per_s": m_total / plain_s, "batched_edges_per_s": m_total / batch_s,
        "speedup_vs_plain": plain_s / batch_s,
        "batched_kernel_ms": kern_ms,
        "batched_alg_GBps": bytes_total / (kern_ms / 1e3) / 1e9 if kern_ms else None,
        "batched_hbm_frac": bytes_total / (kern_ms / 1e3) / 1e9 / HBM_PEAK_GBS if kern_ms else None,
        "schedule": desc, "autotune_s": round(tune_s, 2), "autotune_candidates": len(tune["candidates"]),
        "counts_equal_plain": True,
    }
    plan.free()
    for g in graphs:
        g.free()
    return res


def bench_served(tc, args):
    """Serving: a Poisson trace of count/support requests (lognormal sizes,
    ER/RMAT, 30% re-queries). Capacity = closed-loop graphs/s of the server
    on the mix; then the trace arrives open-loop at 0.6 and at 0.8 x
    capacity, the latter against a plain FIFO (tc_preprocess + tc_count /
    tc_edge_support one at a time) on the same arrival times. Latency =
    result on host - arrival. (When the open loop sustains less than the
    closed loop, the 0.8 point sits near saturation and its latency grows
    over the trace; served_graphs_per_s below the arrival rate shows it.)"""
    import numpy as np
    import torch
    import graphgen
    total = args.serve_warmup + args.serve_requests
    reqs = graphgen.serving_trace(total, rate_per_s=1.0, seed=7)
    distinct = {}
    for r in reqs:
        distinct.setdefault(r.spec.seed, r.spec)
    print("serve: generating %d graphs for %d requests ..." % (len(distinct), total), file=sys.stderr,
          flush=True)
    keys = list(distinct)
    edges = dict(zip(keys, graphgen.generate_many([distinct[k] for k in keys], args.gen_threads)))
    warm, meas = reqs[:args.serve_warmup], reqs[args.serve_warmup:]
    budget = 96 << 30
    opts = {"prep_threads": args.serve_prep_threads}
    if args.serve_ticks:
        opts["ticks"] = args.serve_ticks

    def submit_all(srv, rs, arrivals=None):
        t0 = time.perf_counter()
        tickets = []
        for i, r in enumerate(rs):
            if arrivals is not None:
                dt = arrivals[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
            a, b = edges[r.spec.seed]
            tickets.append(srv.submit(r.op, a, b, r.spec.n, key=r.spec.seed))
        return [srv.poll(t) for t in tickets], t0

    # closed loop: everything queued at once
    with tc.Server(budget, max_slots=args.serve_slots, options=opts) as srv:
        submit_all(srv, warm)
        t0 = time.perf_counter()
        res, _ = submit_all(srv, meas)
        closed_s = time.perf_counter() - t0
        assert all(r["status"] == 0 for r in res), [r for r in res if r["status"]][:2]
        ref = [(r["count"], r.get("support")) for r in res]
    capacity = len(meas) / closed_s

    def open_loop(frac):
        # the trace's arrival times scaled to frac x capacity
        lam = frac * capacity
        arr = [r.arrival_s / lam for r in meas]
        arr = [a - arr[0] for a in arr]
        with tc.Server(budget, max_slots=args.serve_slots, options=opts) as srv:
            submit_all(srv, warm)
            res, _ = submit_all(srv, meas, arr)
            st = srv.stats()
        lat = [r["t_done"] - r["t_submit"] for r in res]
        span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
        for (c, sup), r in zip(ref, res):
            assert r["status"] == 0 and r["count"] == c
            if sup is not None:
                assert np.array_equal(sup, r["support"])
        return lam, arr, lat, span, st

    # open loop at 0.6 x capacity (a second point of the latency curve), then
    # at 0.8 x capacity (the headline point, with the FIFO on the same arrivals)
    lam6, _, lat6, span6, _ = open_loop(0.6)
    lam, arr, lat, span, st = open_loop(0.8)
    # plain FIFO on the same arrival times, one request at a time
    dev = torch.device("cuda")

    def plain_one(r):
        a, b = edges[r.spec.seed]
        g = tc.tc_preprocess(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), r.spec.n)
        if r.op == "count":
            c = int(tc.tc_count(g).item())
        else:
            cnt = torch.empty(1, dtype=torch.int64, device=dev)
            sup, _ = tc.tc_edge_support(g, tc.TC_SUPPORT_FULL, count=cnt)
            sup.cpu()
            c = int(cnt.item())
        g.free()
        return c

    for r in warm[:20]:
        plain_one(r)
    torch.cuda.synchronize()
    fifo_lat, fifo_counts = [], []
    t0 = time.perf_counter()
    for i, r in enumerate(meas):
        dt = arr[i] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        fifo_counts.append(plain_one(r))
        fifo_lat.append(time.perf_counter() - t0 - arr[i])
    fifo_span = time.perf_counter() - t0
    assert fifo_counts == [c for c, _ in ref], "FIFO counts differ from the served counts"
    return {
        "requests": len(meas), "warmup": len(warm), "distinct_graphs": len(distinct),
        "closed_loop_graphs_per_s": capacity, "arrival_rate_per_s": lam,
        "served_graphs_per_s": len(meas) / span, "served_p50_ms": pct(lat, 50) * 1e3,
        "served_p99_ms": pct(lat, 99) * 1e3,
        "load_0_6": {"arrival_rate_per_s": lam6, "served_graphs_per_s": len(meas) / span6,
                     "served_p50_ms": pct(lat6, 50) * 1e3, "served_p99_ms": pct(lat6, 99) * 1e3},
        "fifo_graphs_per_s": len(meas) / fifo_span, "fifo_p50_ms": pct(fifo_lat, 50) * 1e3,
        "fifo_p99_ms": pct(fifo_lat, 99) * 1e3,
        "p99_speedup_vs_fifo": pct(fifo_lat, 99) / pct(lat, 99),
        "results_equal_closed_open_fifo": True,
        "server": {k: st[k] for k in ("ticks", "tick_requests", "max_tick_requests", "cache_hits",
                                      "evicted", "peak_reserved_bytes", "prep_threads", "max_slots",
                                      "tick_slots")},
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the count "
              "would shard by replicating U on every GPU and splitting the tasks)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_1907_09575_amd as tc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    # the committed tuning table of this GPU type (thresholds per graph size,
    # the batch schedule), written by paper_1907_09575_amd/tune.py
    tuning_file = None
    if not args.no_tuning_file:
        tuning_file = args.tuning_file
        if tuning_file is None:
            arch, cus = tc.tc_tuning_key("graph", 1).split("/")[:2]
            tuning_file = os.path.join(ROOT, "paper_1907_09575_amd", "tuning", "%s_%s.json" % (arch, cus))
        if os.path.exists(tuning_file):
            tc.tc_tuning_load(tuning_file)
        else:
            tuning_file = None
    n = 1 << args.scale
    print("generating RMAT scale %d ..." % args.scale, file=sys.stderr, flush=True)
    src_h, dst_h = graphgen.rmat(args.scale, edge_factor=args.edge_factor, seed=args.seed,
                                 threads=args.gen_threads)
    m_raw = len(src_h)
    src = torch.from_numpy(src_h).to(dev)
    dst = torch.from_numpy(dst_h).to(dev)
    del src_h, dst_h
    out = torch.zeros(1, dtype=torch.int64, device=dev)

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # (not in calibration runs: their one 1 GiB copy scales the PMC byte counters)
    copy_gbs = None if args.copy_calibration else measure_copy_gbs(dev)

    phase_events = []

    def step(record=False):
        # (HIP events on the current stream, which both calls use, bracket
        # the two phases: the count's light classes run on a side stream the
        # count joins before it returns)
        if record:
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record()
        g = tc.tc_preprocess(src, dst, n)
        if record:
            ev[1].record()
        tc.tc_count(g, out)
        if record:
            ev[2].record()
            phase_events.append(ev)
        return g

    for i in range(args.warmup):
        g = step()
        torch.cuda.synchronize()
        print("warmup %d: T=%d" % (i, int(out.item())), file=sys.stderr, flush=True)
        info = g.info()
        cstats = tc.tc_graph_class_stats(g)
        g.free()

    timer = tc.Timer(capacity=16384)
    counts = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with timer:
        for i in range(args.steps):
            g = step(record=True)
            counts.append(out.clone())
            g.free()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = timer.summary()
    timer.free()
    if args.kernels_json:
        with open(args.kernels_json, "w") as f:
            json.dump(kern, f, indent=1)
    counts = [int(c.item()) for c in counts]
    assert len(set(counts)) == 1, "counts differ between steps: %s" % counts
    T = counts[0]
    if args.warmup == 0:
        g = step()
        torch.cuda.synchronize()
        info = g.info()
        cstats = tc.tc_graph_class_stats(g)
        g.free()

    step_s = (t1 - t0) / args.steps
    # per phase, wall time on the stream (mean over the timed steps)
    count_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in phase_events]))
    pre_event_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in phase_events]))
    count_kernel_sum_ms = sum(v["total_ms"] for k, v in kern.items() if k.startswith("count:")) / args.steps
    # count alone on the resident graph: 2 warm-ups, median of 11 (HIP events
    # around tc_count on the current stream)
    count_runs = []
    if not args.copy_calibration:
        g = tc.tc_preprocess(src, dst, n)
        for r in range(13):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            tc.tc_count(g, out)
            e1.record()
            e1.synchronize()
            assert int(out.item()) == T
            if r >= 2:
                count_runs.append(e0.elapsed_time(e1))
        g.free()
    count_median_ms = float(np.median(count_runs)) if count_runs else None
    pre_kernel_ms = sum(v["total_ms"] for k, v in kern.items()
                        if not k.startswith("count:") and not k.startswith("_") and k != "zero_i64") / args.steps
    pre_ms = step_s * 1e3 - count_ms  # wall time of the step outside the count phase
    launches = {k: v for k, v in kern.items() if not k.startswith("_")}
    # the dominant kernel: the count class with the most algorithmic bytes
    # (the light classes run on a side stream beside the heavy ones, so the
    # event-timed durations of kernels overlap and their sum exceeds the
    # phase's wall time)
    dom = max((k for k in launches if k.startswith("count:") and k.split(":", 1)[1] in cstats
               and cstats[k.split(":", 1)[1]]["rows"]),
              key=lambda k: count_kernel_bytes(cstats, k.split(":", 1)[1]))
    roofline = None
    if dom.startswith("count:"):
        cls = dom.split(":", 1)[1]
        bytes_per_launch = count_kernel_bytes(cstats, cls)
        avg_s = launches[dom]["avg_ms"] / 1e3
        achieved = bytes_per_launch / avg_s / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": load_traffic(dom), "traffic_kind": "fabric (L2 misses: Infinity Cache or HBM)",
                    "algorithmic_bytes_per_launch": bytes_per_launch,
                    "avg_launch_ms": round(launches[dom]["avg_ms"], 4),
                    "copy_GBps": copy_gbs,
                    "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None}
    else:
        roofline = {"bound": "hbm", "kernel": dom, "achieved": None, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": None, "traffic": None, "copy_GBps": copy_gbs,
                    "note": "dominant kernel is not a count kernel"}

    # whole count phase against the same roofline
    count_bytes = sum(count_kernel_bytes(cstats, c) for c in cstats if cstats[c]["rows"])
    result = {
        "metric": METRIC,
        "value": m_raw / step_s,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "rmat%d_ef%d_preprocess_count" % (args.scale, args.edge_factor),
                   "rmat_abcd": [0.57, 0.19, 0.19, 0.05], "n": n, "m_raw": m_raw, "seed": args.seed,
                   "parallelism": "single_gpu",
                   "tuning_file": os.path.relpath(tuning_file, ROOT) if tuning_file else None,
                   "work_params": tc.tc_tuning_get(tc.tc_tuning_key("graph", info["m"]))},
        "roofline": roofline,
        "triangles": T,
        "m": info["m"],
        "wedges_plus": info["wedges_plus"],
        "probes": info["probes"],
        "count_ms": count_ms,
        "count_kernel_sum_ms": round(count_kernel_sum_ms, 4),
        "preprocess_event_ms": round(pre_event_ms, 4),
        "count_median_ms": round(count_median_ms, 4) if count_median_ms else None,
        "count_median_edges_per_s": info["m"] / (count_median_ms / 1e3) if count_median_ms else None,
        "preprocess_ms": pre_ms,
        "preprocess_kernel_ms": pre_kernel_ms,
        "preprocess": {"ms": round(pre_ms, 3),
                       "alg_bytes": preprocess_bytes(n, m_raw, info["m"], info["tasks"]),
                       "alg_GBps": round(preprocess_bytes(n, m_raw, info["m"], info["tasks"]) / (pre_ms / 1e3) / 1e9, 1),
                       "frac": round(preprocess_bytes(n, m_raw, info["m"], info["tasks"]) / (pre_ms / 1e3) / 1e9
                                     / HBM_PEAK_GBS, 4)},
        "count_edges_per_s": info["m"] / (count_ms / 1e3) if count_ms > 0 else None,
        "count_raw_edges_per_s": m_raw / (count_ms / 1e3) if count_ms > 0 else None,
        "count_probes_per_s": info["probes"] / (count_ms / 1e3) if count_ms > 0 else None,
        "count_phase_alg_GBps": count_bytes / (count_ms / 1e3) / 1e9 if count_ms > 0 else None,
        "classes": {c: {"probes": v["probes"], "rows": v["rows"], "tasks": v["tasks"],
                        "workgroups": v["workgroups"], "table_slots": v["table_slots"]}
                    for c, v in cstats.items() if v["rows"]},
        "kernels_top": {k: {"avg_ms": round(v["avg_ms"], 4), "launches": v["launches"]}
                        for k, v in sorted(launches.items(), key=lambda kv: -kv[1]["total_ms"])[:6]},
    }
    if not args.no_block:
        print("block grid q=%d ..." % args.block_q, file=sys.stderr, flush=True)
        g = step()
        torch.cuda.synchronize()
        result["block"] = bench_block(tc, g, T, args.block_q)
        g.free()
    if not args.no_ablation:
        g = step()
        torch.cuda.synchronize()
        result["ablation"] = bench_ablation(tc, g, T, [int(v) for v in args.ablation_q.split(",") if v])
        g.free()
    del src, dst
    torch.cuda.empty_cache()
    if not args.no_large:
        result["large"] = bench_large(tc, args)
    if not args.no_support:
        print("support (RMAT scale %d) ..." % args.support_scale, file=sys.stderr, flush=True)
        result["support"] = bench_support(tc, args)
    if not args.no_batch:
        result["batched"] = bench_batch(tc, args)
        torch.cuda.empty_cache()
    if not args.no_serve:
        result["served"] = bench_served(tc, args)
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        threads = max(1, min(args.cpu_threads, os.cpu_count() or 1))
        result["cpu_baseline"] = cpu_baseline(args.scale, args.edge_factor, args.seed, threads,
                                              args.cpu_sample, args.cpu_full)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
