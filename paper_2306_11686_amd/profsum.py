"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2306_11686_amd.profsum stats KERNEL_STATS_CSV [--top 8]
    python -m paper_2306_11686_amd.profsum positions KERNEL_TRACE_CSV --kernel NAME --period P --count N \\
        [--skip S] [--labels a,b,...]
    python -m paper_2306_11686_amd.profsum traffic-positions --fetch COUNTER_CSV --write COUNTER_CSV \\
        --kernel NAME --period P --count N [--skip S] [--labels a,b,...] [--alg b0,b1,...]
    python -m paper_2306_11686_amd.profsum traffic --fetch COUNTER_CSV --write COUNTER_CSV \\
        --workload jacobi3d_512 --kernel k_persistent --alg-bytes N [--copy-bytes 1073741824] \\
        [--update profiles/traffic.json]

`stats` prints the kernel-trace statistics (``--kernel-trace --stats``) as a
markdown table. `positions` tabulates one kernel's dispatch durations by
their position in a repeating sequence (the regions of a program's loop). `traffic` turns two counter passes (FETCH_SIZE, WRITE_SIZE,
in KiB per dispatch) into HBM bytes per launch of the named kernel, each
scaled by what the same counter read for the copy kernel (`gf::k_copy_tiles`,
copy_bytes read and copy_bytes written per dispatch) in the same run, and
records them with the kernels' source hash (measurements lapse when the
kernels change).
"""
from __future__ import annotations

import argparse
import csv
import json
import statistics
import sys

from .build import kernel_source_hash


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def stats_table(path: str, top: int = 8) -> str:
    rows = _rows(path)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"] if len(r["Name"]) <= 100 else r["Name"][:97] + "..."
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f}% |")
    return "\n".join(out)


def counter_per_dispatch(path: str, counter: str, kernel: str):
    """(median over the copy-kernel dispatches, mean over the kernel's) in KiB."""
    copy, target = [], []
    for r in _rows(path):
        if r["Counter_Name"] != counter:
            continue
        v = float(r["Counter_Value"])
        if r["Kernel_Name"].startswith("gf::k_copy_tiles"):
            copy.append(v)
        elif kernel in r["Kernel_Name"]:
            target.append(v)
    if not copy or not target:
        raise SystemExit(f"{path}: no {counter} rows for the copy kernel or for {kernel}")
    return statistics.median(copy), sum(target) / len(target), len(target)


def traffic(args) -> dict:
    fc, fk, nf = counter_per_dispatch(args.fetch, "FETCH_SIZE", args.kernel)
    wc, wk, nw = counter_per_dispatch(args.write, "WRITE_SIZE", args.kernel)
    fs = args.copy_bytes / (fc * 1024.0)
    ws = args.copy_bytes / (wc * 1024.0)
    fb, wb = fk * 1024.0 * fs, wk * 1024.0 * ws
    entry = {"source_hash": kernel_source_hash(), "bytes_per_launch": int(round(fb + wb)),
             "fetch_bytes_per_launch": int(round(fb)), "write_bytes_per_launch": int(round(wb)),
             "alg_bytes_per_launch": args.alg_bytes, "fetch_scale": round(fs, 6), "write_scale": round(ws, 6),
             "fetch_kib_raw": round(fk, 1), "write_kib_raw": round(wk, 1), "dispatches": [nf, nw],
             "kernel": args.kernel}
    if args.update:
        try:
            with open(args.update) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
        db[args.workload] = entry
        with open(args.update, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
            f.write("\n")
    return entry


def _dispatch_values(path: str, counter: str, kernel: str):
    """(copy-kernel median, the kernel's values in dispatch order) in KiB."""
    copy, target = [], []
    for r in _rows(path):
        if r["Counter_Name"] != counter:
            continue
        v = float(r["Counter_Value"])
        if r["Kernel_Name"].startswith("gf::k_copy_tiles"):
            copy.append(v)
        elif kernel in r["Kernel_Name"]:
            target.append((int(r.get("Dispatch_Id", r.get("Correlation_Id", 0)) or 0), v))
    if not copy or not target:
        raise SystemExit(f"{path}: no {counter} rows for the copy kernel or for {kernel}")
    target.sort()
    return statistics.median(copy), [v for _, v in target]


def traffic_positions_table(fetch: str, write: str, kernel: str, skip: int, period: int, count: int, labels,
                            alg, copy_bytes: int = 1 << 30) -> str:
    """HBM bytes per dispatch of one kernel by position in a repeating
    sequence (the regions of a program's loop), each counter scaled by what
    it reads for the copy kernel in the same run, beside the algorithmic
    bytes of each position."""
    fc, fv = _dispatch_values(fetch, "FETCH_SIZE", kernel)
    wc, wv = _dispatch_values(write, "WRITE_SIZE", kernel)
    fs, ws = copy_bytes / (fc * 1024.0), copy_bytes / (wc * 1024.0)
    fv, wv = fv[skip:skip + count], wv[skip:skip + count]
    if len(fv) < count or len(wv) < count:
        raise SystemExit(f"only {min(len(fv), len(wv))} dispatches of {kernel!r} after skipping {skip}")
    out = ["| position | region | reads (MB) | writes (MB) | total (MB) | algorithmic (MB) | measured / algorithmic |",
           "|---|---|---|---|---|---|---|"]
    for k in range(period):
        rf = statistics.mean(fv[k::period]) * 1024.0 * fs
        rw = statistics.mean(wv[k::period]) * 1024.0 * ws
        a = alg[k] if k < len(alg) else 0
        ratio = f"{(rf + rw) / a:.3f}" if a else ""
        out.append(f"| {k} | {labels[k] if k < len(labels) else ''} | {rf / 1e6:.2f} | {rw / 1e6:.2f} | "
                   f"{(rf + rw) / 1e6:.2f} | {a / 1e6:.2f} | {ratio} |")
    out.append("")
    out.append(f"Scale factors from the 1 GiB copy in the same run: reads x{fs:.4f}, writes x{ws:.4f}.")
    return "\n".join(out)


def positions_table(path: str, kernel: str, skip: int, period: int, count: int, labels) -> str:
    """Durations of the dispatches of one kernel, taken in start order, by
    their position in a repeating sequence (a program's regions): the
    first `skip` dispatches are passed over, then `count` dispatches are
    grouped by index modulo `period`."""
    rows = sorted((r for r in _rows(path) if kernel in r["Kernel_Name"]), key=lambda r: int(r["Start_Timestamp"]))
    run = rows[skip:skip + count]
    if len(run) < count:
        raise SystemExit(f"only {len(run)} dispatches of {kernel!r} after skipping {skip}")
    by = [[] for _ in range(period)]
    for i, r in enumerate(run):
        by[i % period].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    span = (int(run[-1]["End_Timestamp"]) - int(run[0]["Start_Timestamp"])) / 1e3
    out = ["| position | region | median (us) | mean (us) | share of kernel time |", "|---|---|---|---|---|"]
    total = sum(sum(v) for v in by)
    for k, v in enumerate(by):
        name = labels[k] if k < len(labels) else ""
        out.append(f"| {k} | {name} | {statistics.median(v):.1f} | {statistics.mean(v):.1f} | "
                   f"{100 * sum(v) / total:.1f} % |")
    reps = count / period
    out.append("")
    out.append(f"Kernel time per period: {total / reps:.1f} us; wall span per period (first dispatch start to "
               f"last dispatch end, divided by {reps:g}): {span / reps:.1f} us.")
    return "\n".join(out)


def _row(cells) -> str:
    return "| " + " | ".join(str(c) for c in cells) + " |"


def other_workloads_md(path: str, command: str) -> str:
    """The JSON lines `measure.py` prints, as the markdown summary of the
    other workloads (one section per configuration it finds)."""
    recs = {}
    with open(path) as f:
        for line in f:
            if line.startswith("{"):
                d = json.loads(line)
                recs[d["config"].split("_")[0]] = d
    modes = ("persistent", "per_region", "per_region_graph", "kernel_split")
    out = ["# Other workloads: persistent, per-region, graph and kernel-split timings on one MI355X", "",
           "Command (from the repository root; launch shapes from `paper_2306_11686_amd/tuning_db.json`; "
           "the per-region modes of CG take the shape tuned in that mode):", "", "    " + command, "",
           "Times are HIP-event medians of the repetitions after a warm-up run. \"Algorithmic\" bytes are what "
           "the legacy loops must move (each input element read once, each output written once).", ""]
    d = recs.get("sync")
    if d:
        out += [f"## Cost of one trivial region (3D Jacobi on a 4^3 grid, {d['regions']} regions)", "",
                "| mode | us per region |", "|---|---|"]
        out += [_row([k[: -len("_us_per_region")], v]) for k, v in d.items() if k.endswith("_us_per_region")]
        one = {k[len("one_region_program_"): -len("_us")]: v for k, v in d.items()
               if k.startswith("one_region_program_")}
        if one:
            out += ["", "A program of one such region launched 200 times back to back (the fixed cost of one "
                    "launch):", "", "| mode | us per program |", "|---|---|"]
            out += [_row([k, v]) for k, v in one.items()]
        out.append("")
    d = recs.get("jacobi2d")
    if d:
        out += ["## 2D Jacobi 256^2, 100 sweeps, L2 residual, printf every 10 sweeps through the RPC", "",
                "| mode | ms per run | us per region | regions/s | printf cost (us each) |", "|---|---|---|---|---|"]
        for m in modes:
            if m in d:
                out.append(_row([m, d[m]["ms_per_run"], d[m]["us_per_region"], d[m]["regions_per_s"],
                                 d[m].get("printf_us_each", "")]))
        for m in modes:
            if m + "_no_printf" in d:
                e = d[m + "_no_printf"]
                out.append(_row([m + " (no printf)", e["ms_per_run"], e["us_per_region"], e["regions_per_s"], ""]))
        out.append("")
    for d in _all_lines(path):
        if d["config"].startswith("rpc_printf"):
            out += ["## RPC round trips (one wavefront calling 1,000 times; the library's server thread polls)", "",
                    f"printf with an int and a double as values: posted {d['posted']['us_per_call']} us per call, "
                    f"blocking {d['blocking']['us_per_call']} us per call.", ""]
    fp = [d for d in _all_lines(path) if d["config"].startswith("rpc_fprintf")]
    if fp:
        d = fp[-1]
        out += ["The paper's RPC benchmark shape: 1,000 blocking fprintf calls whose format string and 128-byte "
                "buffer are passed by reference (the buffer read-write when the callee's use is unknown, read-only "
                "when it is known).", "",
                "| buffer mode | us per call | device: args | copy in | wait | copy out | host: decode | call | "
                "reply | in flight |", "|---|---|---|---|---|---|---|---|---|---|"]
        for m in ("buffer_read_write", "buffer_read_only"):
            st = d[m]["stages_us"]
            out.append(_row([m[len("buffer_"):], d[m]["us_per_call"], st["dev_args_us"], st["dev_copy_in_us"],
                             st["dev_wait_us"], st["dev_copy_out_us"], st["host_decode_us"], st["host_call_us"],
                             st["host_reply_us"], st["transit_us"]]))
        out += ["", f"Stage times are averages over {d['buffer_read_write']['timed_calls']:,} timed calls.", ""]
    d = recs.get("phases")
    if d:
        out += ["## Manual worksharing with barriers: 2^22 doubles, 100 producer/consumer phases", "",
                f"Algorithmic bytes per phase {d['alg_bytes_per_phase']:,}.", "",
                "| mode | workgroups | ms per run | us per phase | algorithmic GB/s |", "|---|---|---|---|---|"]
        for k, v in d.items():
            if isinstance(v, dict):
                out.append(_row([k.rsplit("_wg", 1)[0], v["grid"], v["ms_per_run"], v["us_per_phase"], v["GBps"]]))
        out.append("")
    d = recs.get("cg")
    if d:
        out += [f"## CG on the 27-point matrix at 128^3 ({d['rows']:,} rows, {d['nnz']:,} nonzeros), 500 iterations",
                "", f"Algorithmic bytes per iteration: {d['alg_bytes_per_iteration']:,}.", "",
                "| mode | ms per run | algorithmic GB/s | regions/s |", "|---|---|---|---|"]
        out += [_row([m, d[m]["ms_per_run"], d[m]["GBps"], d[m]["regions_per_s"]]) for m in modes if m in d]
        out.append("")
    d = recs.get("hist")
    if d:
        out += ["## Histogram: 2^28 u32 keys into 65,536 bins", "",
                f"Algorithmic bytes: {d['alg_bytes']:,} (keys once, bins read and written once).", "",
                "| keys | mode | us per run | algorithmic GB/s |", "|---|---|---|---|"]
        for k, v in d.items():
            if isinstance(v, dict):
                keys, mode = k.split("_", 1)
                out.append(_row([keys, mode, v["us_per_run"], v["GBps"]]))
        out.append("")
    d = recs.get("batched")
    if d:
        out += ["## Batched: 256 uneven 2D Jacobi instances (sides 64..2047), 50 sweeps each", "",
                f"Sum of n^2 = {d['sum_n2']:,}; {d['regions_per_run']:,} regions per run; algorithmic bytes "
                f"{d['alg_bytes_per_run']:,}; a shape per instance from the batched autotuner: "
                f"{'yes' if d.get('per_instance_shapes') else 'no'}; workgroups off their group's XCD in the "
                f"persistent launch: {d.get('persistent_misplaced_workgroups', 'n/a')}.", "",
                "| mode | ms per run | algorithmic GB/s | regions/s |", "|---|---|---|---|"]
        out += [_row([m, d[m]["ms_per_run"], d[m]["GBps"], d[m]["regions_per_s"]]) for m in modes if m in d]
        out.append("")
    d = recs.get("heap")
    if d:
        out += ["## Allocator benchmark: every thread allocates, uses and frees 128 bytes in one kernel", "",
                "Balanced heap with 32 thread slots x 16 team slots (the paper's configuration) and with 64 x 32; "
                "HIP's device malloc with the same heap size.", "",
                "| teams | threads per team | balanced 32x16 (us) | balanced 64x32 (us) | HIP device malloc (us) | "
                "HIP / 64x32 |", "|---|---|---|---|---|---|"]
        for k, v in d.items():
            if isinstance(v, dict):
                t, th = k[len("teams"):].split("_threads")
                out.append(_row([t, th, v["balanced_us"], v["balanced64x32_us"], v["hip_malloc_us"],
                                 v["speedup64x32"]]))
        out.append("")
    return "\n".join(out)


def _all_lines(path: str):
    with open(path) as f:
        return [json.loads(line) for line in f if line.startswith("{")]


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=8)
    q = sub.add_parser("positions")
    q.add_argument("csv")
    q.add_argument("--kernel", required=True)
    q.add_argument("--skip", type=int, default=0)
    q.add_argument("--period", type=int, required=True)
    q.add_argument("--count", type=int, required=True)
    q.add_argument("--labels", default="")
    tp = sub.add_parser("traffic-positions")
    tp.add_argument("--fetch", required=True)
    tp.add_argument("--write", required=True)
    tp.add_argument("--kernel", required=True)
    tp.add_argument("--skip", type=int, default=0)
    tp.add_argument("--period", type=int, required=True)
    tp.add_argument("--count", type=int, required=True)
    tp.add_argument("--labels", default="")
    tp.add_argument("--alg", default="", help="comma list: algorithmic bytes of each position")
    tp.add_argument("--copy-bytes", type=int, default=1 << 30)
    o = sub.add_parser("other")
    o.add_argument("measure_out")
    o.add_argument("--command", default="python -m paper_2306_11686_amd.measure")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--alg-bytes", type=int, required=True)
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--update", default=None)
    args = ap.parse_args()
    if args.cmd == "other":
        print(other_workloads_md(args.measure_out, args.command))
        return
    if args.cmd == "stats":
        print(stats_table(args.csv, args.top))
        return
    if args.cmd == "traffic-positions":
        print(traffic_positions_table(args.fetch, args.write, args.kernel, args.skip, args.period, args.count,
                                      [x for x in args.labels.split(",") if x] if args.labels else [],
                                      [int(x) for x in args.alg.split(",") if x] if args.alg else [],
                                      args.copy_bytes))
        return
    if args.cmd == "positions":
        print(positions_table(args.csv, args.kernel, args.skip, args.period, args.count,
                              [x for x in args.labels.split(",") if x] if args.labels else []))
        return
    e = traffic(args)
    a = args.alg_bytes
    print("| quantity | per launch | vs algorithmic |\n|---|---|---|")
    print(f"| FETCH_SIZE raw | {e['fetch_kib_raw']:.0f} KiB | |")
    print(f"| WRITE_SIZE raw | {e['write_kib_raw']:.0f} KiB | |")
    print(f"| reads (scaled x{e['fetch_scale']:.4f}) | {e['fetch_bytes_per_launch'] / 1e9:.2f} GB | |")
    print(f"| writes (scaled x{e['write_scale']:.4f}) | {e['write_bytes_per_launch'] / 1e9:.2f} GB | |")
    print(f"| total | {e['bytes_per_launch'] / 1e9:.2f} GB | {e['bytes_per_launch'] / a:.3f} x of {a / 1e9:.2f} GB |")
    print(f"\nKernel source hash: {e['source_hash']}", file=sys.stdout)


if __name__ == "__main__":
    main()
