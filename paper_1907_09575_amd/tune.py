"""Tune the row-bucket thresholds and batch schedules on this GPU and save
the library's tuning table as JSON.

For each RMAT scale given, a seeded synthetic graph (edge factor 16, the
RMAT parameters of the benchmarks) is preprocessed and tc_graph_autotune
times tc_count under candidate thresholds; the best go into the table under
the "graph" key of that size. Then tc_batch_autotune tunes the schedule of
the 4096-graph batch (the benchmark's mix) under its "batch" key. The table
is written with tc_tuning_save; tc_tuning_load, or the TC_TUNING_FILE
environment variable, brings it back in a later process.

    python paper_1907_09575_amd/tune.py [--scales 20,22,24] [--batch-graphs 4096] [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--scales", default="20,22,24")
    p.add_argument("--batch-graphs", type=int, default=4096, help="0: skip the batch schedule")
    p.add_argument("--threads", type=int, default=16, help="generator threads")
    p.add_argument("--out", default=None, help="default: tuning/<arch>_<CUs>cu.json beside this file")
    a = p.parse_args(argv)

    import torch
    import graphgen
    import paper_1907_09575_amd as tc

    torch.cuda.set_device(0)
    report = {}
    for scale in [int(x) for x in a.scales.split(",") if x]:
        s, d = graphgen.rmat(scale, seed=1, threads=a.threads)
        g = tc.tc_preprocess(torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), 1 << scale)
        del s, d
        t0 = time.perf_counter()
        res = tc.tc_graph_autotune(g)
        print("scale %d: %s %.2f s -> %s" % (scale, res["key"], time.perf_counter() - t0, json.dumps(res["best"])),
              flush=True)
        report[res["key"]] = res["best"]
        g.free()
        torch.cuda.empty_cache()
    if a.batch_graphs > 0:
        specs = graphgen.batch_specs(a.batch_graphs)
        lists = graphgen.generate_many(specs, a.threads)
        graphs = [tc.tc_preprocess(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), sp.n)
                  for sp, (x, y) in zip(specs, lists)]
        del lists
        t0 = time.perf_counter()
        res = tc.tc_batch_autotune(graphs)
        print("batch of %d: %s %.2f s -> %s" % (len(graphs), res["key"], time.perf_counter() - t0,
                                                 json.dumps(res["best"])), flush=True)
        report[res["key"]] = res["best"]
        for g in graphs:
            g.free()
    out = a.out
    if out is None:
        arch, cus = next(iter(report)).split("/")[:2] if report else ("unknown", "0cu")
        out = os.path.join(HERE, "tuning", "%s_%s.json" % (arch, cus))
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    tc.tc_tuning_save(out)
    print("saved %d entries to %s" % (len(report), out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
