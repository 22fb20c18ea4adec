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
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--alg-bytes", type=int, required=True)
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--update", default=None)
    args = ap.parse_args()
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
