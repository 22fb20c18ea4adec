"""Tune the standard workloads with the library's autotuner and record the
winners in the tuning database.

    python -m paper_2306_11686_amd.tune_workloads [--db PATH] [--only jacobi3d_512,cg_128]

Every candidate runs the real program (shortened where the launch shape's
ranking does not depend on the run length: 40 of the 200 3D sweeps, 50 of
the 500 CG iterations); the batched workload is tuned per instance by the
batched autotuner (gf_tune_batched). Prints one JSON line per workload with the winner
and the spread of the candidates.
"""
from __future__ import annotations

import argparse
import json
import math
import sys

from . import tuner, workloads
from .binding import GF_EXEC_PER_REGION, GF_EXEC_PERSISTENT, Context


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--db", default=tuner.DEFAULT_DB)
    ap.add_argument("--only", default="jacobi3d_512,jacobi2d_256,cg_128,cg_128@per_region,hist_2^28,hist_2^28@per_region,batched_256,batched_256@per_region")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch
    ctx = Context(0, rpc_capture=True)
    builders = {
        "jacobi3d_512": lambda: workloads.jacobi3d(512, 40),
        "jacobi2d_256": lambda: workloads.jacobi2d(ctx, 256, 100),
        "cg_128": lambda: workloads.cg(128, 50),
        "cg_128@per_region": lambda: workloads.cg(128, 50),
        "hist_2^28": lambda: workloads.histogram(1 << 28),
        "hist_2^28@per_region": lambda: workloads.histogram(1 << 28),
        "batched_256": lambda: workloads.batched(256, 50),
        "batched_256@per_region": lambda: workloads.batched(256, 50),
    }
    for key in args.only.split(","):
        log(f"[tune] {key}")
        prog, inst, keep, _ = builders[key]()
        if key == "batched_256":
            launches, ms = tuner.tune_batched(ctx, prog, inst, key=key, reps=args.reps, path=args.db)
            print(json.dumps({"workload": key, "wg_size": int(launches[0].wg_size), "best_ms": round(ms, 4),
                              "rows_per_tile": sorted({int(l.tile_y) for l in launches})}), flush=True)
            del keep, inst
            torch.cuda.empty_cache()
            continue
        # a key ending in @per_region is tuned in that mode (its grid choices
        # differ: a per-region launch need not fit one resident round)
        mode = GF_EXEC_PER_REGION if key.endswith("@per_region") else GF_EXEC_PERSISTENT
        best, table = tuner.tune(ctx, prog, inst, key=key, mode=mode, reps=args.reps, path=args.db)
        ctx.take_output()
        ms = [m for _, m in table if math.isfinite(m)]
        print(json.dumps({"workload": key, "best": tuner.launch_to_dict(best), "best_ms": round(min(ms), 4),
                          "worst_ms": round(max(ms), 4), "runnable": len(ms), "candidates": len(table)}),
              flush=True)
        del keep, inst
        torch.cuda.empty_cache()
    ctx.close()


if __name__ == "__main__":
    main()
