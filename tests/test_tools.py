"""Host logic of the measurement tools (CPU): the PMC traffic scaling, the
LDS / L2 ratio and launch-class summaries of rocprof_summary, and bench.py's
algorithmic-bytes formula, defaults and single-GPU refusal."""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_1907_09575_amd"))
sys.path.insert(0, ROOT)

import rocprof_summary as rs  # noqa: E402

FIELDS = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for name, grid, counter, value in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_scales_by_the_calibration_copy(tmp_path):
    # the 1 GiB copy reads 512 MiB of FETCH_SIZE (x2) and 1 GiB of WRITE_SIZE
    # (x1); the class launch is found by kernel name and grid = work-groups * 256
    kname = "void tc::(anonymous namespace)::k_count_items<0, false, 7, 4>(tc::Args, tc::CountItem const*)"
    write_counters(tmp_path / "f.csv", [
        ("__amd_rocclr_copyBuffer", 131072, "FETCH_SIZE", 524288.0),
        (kname, 2560, "FETCH_SIZE", 1000.0),
        (kname, 2560, "FETCH_SIZE", 3000.0),
        (kname, 512, "FETCH_SIZE", 99999.0),  # another class sharing the kernel
    ])
    write_counters(tmp_path / "w.csv", [
        ("__amd_rocclr_copyBuffer", 131072, "WRITE_SIZE", 1048576.0),
        (kname, 2560, "WRITE_SIZE", 10.0),
    ])
    bench = {"classes": {"wg_large": {"workgroups": 10}},
             "roofline": {"kernel": "count:wg_large", "algorithmic_bytes_per_launch": 4096000},
             "config": {"workload": "w", "seed": 1}}
    (tmp_path / "b.json").write_text(json.dumps(bench))
    res = rs.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "b.json"),
                     "count:wg_large", str(tmp_path / "out.json"), ["cmd"])
    assert res["calibration"]["fetch_scale"] == 2.0 and res["calibration"]["write_scale"] == 1.0
    assert res["fetch_kib_per_launch"] == 2000.0 and res["write_kib_per_launch"] == 10.0
    assert res["fabric_bytes_per_launch"] == 2000.0 * 1024 * 2 + 10.0 * 1024
    assert res["algorithmic_bytes_per_launch"] == 4096000
    assert json.loads((tmp_path / "out.json").read_text())["commands"] == ["cmd"]


def test_ratios(tmp_path):
    k = "void tc::k_rs_onesweep<unsigned long>(unsigned long const*)"
    write_counters(tmp_path / "l.csv", [
        (k, 1024, "SQ_LDS_BANK_CONFLICT", 30.0), (k, 1024, "SQ_LDS_IDX_ACTIVE", 100.0),
        (k, 1024, "TCC_HIT_sum", 70.0), (k, 1024, "TCC_MISS_sum", 30.0),
    ])
    out = rs.ratios(str(tmp_path / "l.csv")).splitlines()
    assert len(out) == 2
    cols = out[1].split()
    assert cols[-2:] == ["0.3000", "0.7000"]


def test_launches_group_by_kernel_and_grid(tmp_path):
    path = tmp_path / "t.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for grid, start, end in ((256, 0, 2000000), (256, 10, 1000010), (512, 0, 500000)):
            w.writerow({"Kernel_Name": "k_a", "Grid_Size_X": grid, "Start_Timestamp": start, "End_Timestamp": end})
    lines = rs.launches(str(path)).splitlines()
    first = lines[1].split()
    assert first[:3] == ["k_a", "256", "2"] and float(first[3]) == 3.0 and float(first[4]) == 1.5
    assert lines[2].split()[:3] == ["k_a", "512", "1"]


def test_count_kernel_bytes_formula():
    import bench
    stats = {"wg_large": {"probes": 10, "table_keys": 3, "tasks": 2, "rows": 1}}
    assert bench.count_kernel_bytes(stats, "wg_large") == 4 * 10 + 4 * 3 + 12 * 2 + 32 * 1


def test_bench_refuses_more_than_one_gpu():
    # exits with status 2 and a message before any device work
    import subprocess
    for argv, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})):
        e = dict(os.environ, **env)
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True,
                           text=True, env=e, timeout=120)
        assert r.returncode == 2
        assert "one GPU only" in r.stderr
        assert r.stdout == ""


def test_bench_defaults():
    import bench
    saved = sys.argv
    try:
        sys.argv = ["bench.py"]
        a = bench.parse()
    finally:
        sys.argv = saved
    assert (a.gpus, a.steps, a.warmup, a.scale, a.edge_factor) == (1, 5, 2, 24, 16)
    assert a.support_scale == 20 and a.block_q == 13 and a.batch_graphs == 4096
    assert not (a.no_block or a.no_support or a.no_batch or a.no_serve or a.no_cpu_baseline or a.no_large)
    assert a.large_scale == 26
