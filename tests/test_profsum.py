"""The rocprofv3 summaries behind the committed profiles (CPU only): per-kernel
statistics, dispatch durations by position in a repeating sequence, HBM
traffic scaled by the copy kernel's counter readings, and the source hash
that ties a traffic measurement to the code it was taken on."""
import argparse
import csv
import json

import pytest

from paper_2306_11686_amd import profsum


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_positions_groups_dispatches_by_their_place_in_the_period(tmp_path):
    """Two prologue dispatches, then 4 periods of 3 regions with known
    durations, interleaved with another kernel and written out of order."""
    rows, t = [], 1000
    for d in (50, 70):                                  # prologue
        rows.append({"Kernel_Name": "k_region<440u, 1, 1>", "Start_Timestamp": t, "End_Timestamp": t + d})
        t += d + 5
    for rep in range(4):
        for k, d in enumerate((100 + rep, 20, 7 + 2 * rep)):
            rows.append({"Kernel_Name": "k_region<440u, 1, 1>", "Start_Timestamp": t, "End_Timestamp": t + d * 1000})
            t += d * 1000 + 10
        rows.append({"Kernel_Name": "other", "Start_Timestamp": t, "End_Timestamp": t + 99999})
    rows.reverse()
    p = tmp_path / "trace.csv"
    _write(p, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    out = profsum.positions_table(str(p), "k_region<440u", 2, 3, 12, ["a", "b"])
    lines = out.splitlines()
    assert lines[2].startswith("| 0 | a | 101.5 | 101.5 |")   # median and mean of 100..103
    assert lines[3].startswith("| 1 | b | 20.0 | 20.0 |")
    assert lines[4].startswith("| 2 |  | 10.0 | 10.0 |")      # 7, 9, 11, 13
    total = sum(100 + r + 20 + 7 + 2 * r for r in range(4))
    assert f"Kernel time per period: {total / 4:.1f} us" in out
    with pytest.raises(SystemExit):
        profsum.positions_table(str(p), "k_region<440u", 2, 3, 13, [])


def test_stats_table_sorts_by_total_time(tmp_path):
    p = tmp_path / "stats.csv"
    fields = ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs", "Percentage"]
    _write(p, fields, [
        {"Name": "small", "Calls": 10, "TotalDurationNs": 1000, "AverageNs": 100, "MinNs": 90, "MaxNs": 110,
         "Percentage": 1.0},
        {"Name": "big", "Calls": 2, "TotalDurationNs": 99000, "AverageNs": 49500, "MinNs": 49000, "MaxNs": 50000,
         "Percentage": 99.0},
    ])
    lines = profsum.stats_table(str(p), 8).splitlines()
    assert lines[2] == "| `big` | 2 | 49.5 | 49.0 | 50.0 | 99.00% |"
    assert lines[3].startswith("| `small` | 10 | 0.1 |")


def test_traffic_scales_each_counter_by_the_copy_kernel(tmp_path):
    """The copy kernel reads and writes 1 GiB per dispatch. If FETCH_SIZE
    reads half of that and WRITE_SIZE all of it, the target kernel's
    readings scale by 2 and 1."""
    fields = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    gib_kib = (1 << 30) / 1024
    copy = "gf::k_copy_tiles(HIP_vector_type<double, 2u> const*, ...)"
    _write(tmp_path / "f.csv", fields, [
        {"Kernel_Name": copy, "Counter_Name": "FETCH_SIZE", "Counter_Value": gib_kib / 2},
        {"Kernel_Name": copy, "Counter_Name": "FETCH_SIZE", "Counter_Value": gib_kib / 2 + 8},
        {"Kernel_Name": copy, "Counter_Name": "FETCH_SIZE", "Counter_Value": gib_kib / 2 - 8},
        {"Kernel_Name": "void gf::k_persistent<132u>(...)", "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000.0},
    ])
    _write(tmp_path / "w.csv", fields, [
        {"Kernel_Name": copy, "Counter_Name": "WRITE_SIZE", "Counter_Value": gib_kib},
        {"Kernel_Name": "void gf::k_persistent<132u>(...)", "Counter_Name": "WRITE_SIZE", "Counter_Value": 300.0},
        {"Kernel_Name": "void gf::k_persistent<132u>(...)", "Counter_Name": "WRITE_SIZE", "Counter_Value": 500.0},
    ])
    db = tmp_path / "traffic.json"
    args = argparse.Namespace(fetch=str(tmp_path / "f.csv"), write=str(tmp_path / "w.csv"), kernel="k_persistent",
                              alg_bytes=123, copy_bytes=1 << 30, update=str(db), workload="w")
    e = profsum.traffic(args)
    assert e["fetch_scale"] == 2.0 and e["write_scale"] == 1.0
    assert e["fetch_bytes_per_launch"] == 2 * 1000 * 1024
    assert e["write_bytes_per_launch"] == 400 * 1024            # mean over the kernel's dispatches
    assert e["dispatches"] == [1, 2]
    assert json.loads(db.read_text())["w"]["bytes_per_launch"] == e["bytes_per_launch"]


def test_source_hash_ignores_comments_but_not_code():
    from paper_2306_11686_amd.build import _code_only
    a = "int f(int x) {\n    return x + 1;  // one more\n}\n/* note */\n"
    b = "int f(int x)\n{ /* changed\n comment */ return x + 1; }\n"
    c = "int f(int x) { return x + 2; }"
    assert _code_only(a) == _code_only(b) != _code_only(c)


def test_bench_reports_traffic_only_for_the_measured_code(tmp_path, monkeypatch):
    """bench.py's roofline.traffic comes from profiles/traffic.json only when
    the entry's source hash is that of the kernels as they are now."""
    import bench
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(
        {"w": {"source_hash": "abc", "bytes_per_launch": 42}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.load_traffic("w") == 42
    assert bench.load_traffic("other") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "def")
    assert bench.load_traffic("w") is None


def test_other_workloads_summary_from_measure_lines(tmp_path):
    """profsum other turns measure.py's JSON lines into one table per
    configuration, with the figures as printed."""
    from paper_2306_11686_amd import profsum
    lines = [
        {"config": "cg_27pt_128^3_f64_500iters", "rows": 2097152, "nnz": 55742968,
         "alg_bytes_per_iteration": 912185252,
         "persistent": {"ms_per_run": 133.6, "GBps": 3413.5, "regions_per_s": 22452.4},
         "per_region": {"ms_per_run": 120.4, "GBps": 3786.7, "regions_per_s": 24907.3}},
        {"config": "rpc_printf_1000_calls", "calls": 1000, "posted": {"us_per_call": 3.26},
         "blocking": {"us_per_call": 5.44}},
        {"config": "hist_u32_2^28_keys_65536_bins", "alg_bytes": 1074266112,
         "uniform_persistent": {"us_per_run": 293.8, "GBps": 3656.9}},
    ]
    p = tmp_path / "m.out"
    p.write_text("noise\n" + "\n".join(json.dumps(x) for x in lines) + "\n")
    md = profsum.other_workloads_md(str(p), "cmd")
    assert "| persistent | 133.6 | 3413.5 | 22452.4 |" in md
    assert "| per_region | 120.4 | 3786.7 | 24907.3 |" in md
    assert "Algorithmic bytes per iteration: 912,185,252." in md
    assert "posted 3.26 us per call, blocking 5.44 us per call" in md
    assert "| uniform | persistent | 293.8 | 3656.9 |" in md
    assert "    cmd" in md
