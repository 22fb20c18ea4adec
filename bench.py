"""Benchmark: 3D 7-point Jacobi on a 512^3 FP64 grid, 200 sweeps, each sweep a
`parallel for` with a reduction(max) residual; one persistent kernel with
grid barriers between regions versus one launch per region.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

A step is one run of the whole program (200 sweeps). Prints one JSON line
(last line of stdout) with HBM GB/s (algorithmic bytes / time), regions/s,
the per-region comparison, the roofline of the persistent kernel and the
serial CPU oracle timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HBM GB/s + regions/s: persistent GPU-First vs per-region launch, Jacobi 512^3"
PEAK_GBPS = 8000.0  # MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def alg_bytes_per_sweep(n: int) -> int:
    """One read of every point the stencil touches (all but the 12 edges and
    8 corners) and one write of every interior point."""
    return 8 * (n ** 3 - 12 * (n - 2) - 8) + 8 * (n - 2) ** 3


def kernel_source_hash() -> str:
    from paper_2306_11686_amd.build import kernel_source_hash as h
    return h()


def load_traffic(workload: str):
    """HBM traffic per launch measured with rocprofv3 counters, if it was
    taken on the kernels as they are now (same source hash)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(workload)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def load_tuned(workload: str):
    path = os.path.join(ROOT, "paper_2306_11686_amd", "tuning_db.json")
    try:
        with open(path) as f:
            d = json.load(f)
        return d.get(workload)
    except (OSError, ValueError):
        return None


def time_mode(ctx, gf, torch, prog, inst, mode, launch, steps, warmup):
    for _ in range(warmup):
        ctx.run(prog, inst, mode=mode, launch=launch)
    torch.cuda.synchronize()
    ctx.sync()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    stats = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record()
        stats = ctx.run(prog, inst, mode=mode, launch=launch)
        ends[k].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync()
    ev_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return (t1 - t0) * 1e3 / steps, sum(ev_ms) / len(ev_ms), stats


def cpu_model() -> str:
    """The host CPU's model name (what lscpu prints), from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(u0, n, budget_s=15.0, max_sweeps=200, omp_budget_s=5.0):
    """The serial oracle on this host's cores (one thread) for a bounded
    number of sweeps of the same 512^3 workload; beside it, for context, the
    same loop built with OpenMP on all of the host's threads (the CPU build
    the paper compares each GPU region with)."""
    import oracle
    from oracle import omp

    u = u0.copy()
    w = u0.copy()
    # the serial oracle runs on one core: pin this thread to the first core it
    # may use, and restore the mask for the OpenMP leg afterwards
    mask = os.sched_getaffinity(0)
    core = min(mask)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        oracle.jacobi3d_inplace(u, w, 1)
        t1 = time.perf_counter() - t0
        k = int(max(1, min(max_sweeps, budget_s / max(t1, 1e-3))))
        t0 = time.perf_counter()
        oracle.jacobi3d_inplace(u, w, k)
        dt = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, mask)
    cpu = {
        "value": round(k * alg_bytes_per_sweep(n) / dt / 1e9, 3),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{k} sweeps of the {n}^3 grid (after 1 timed warm-up sweep), serial C oracle, 1 thread "
                  f"pinned to core {core}",
        "seconds": round(dt, 3),
        "pinned_core": core,
        "nproc": len(mask),
        "cpu_model": cpu_model(),
    }
    threads = omp.max_threads()
    t0 = time.perf_counter()
    omp.jacobi3d(u, w, 1)
    t1 = time.perf_counter() - t0
    k = int(max(1, min(max_sweeps, omp_budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    omp.jacobi3d(u, w, k)
    dt = time.perf_counter() - t0
    del u, w
    cpu_omp = {
        "value": round(k * alg_bytes_per_sweep(n) / dt / 1e9, 3),
        "unit": "GB/s",
        "threads": threads,
        "kind": "legacy loop built with OpenMP",
        "sample": f"{k} sweeps of the {n}^3 grid (after 1 timed warm-up sweep), {threads} OpenMP threads",
        "seconds": round(dt, 3),
    }
    return cpu, cpu_omp


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--sweeps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-region", action="store_true")
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--tile-z", type=int, default=0)
    ap.add_argument("--wg-size", type=int, default=0)
    ap.add_argument("--num-wg", type=int, default=0)
    ap.add_argument("--xcd-remap", type=int, default=-1)
    ap.add_argument("--prefetch", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the stencil would shard by z-slabs "
                                   "with halo exchange across GPUs, which is not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import gf_inputs as gi
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs

    n, sweeps = args.n, args.sweeps
    workload = f"jacobi3d_{n}"
    tuned = load_tuned(workload) or {}
    launch = gf.Launch.make(
        wg_size=args.wg_size or tuned.get("wg_size", 0),
        num_wg=args.num_wg or tuned.get("num_wg", 0),
        tile_y=args.tile_y or tuned.get("tile_y", 0),
        tile_z=args.tile_z or tuned.get("tile_z", 0),
        xcd_remap=args.xcd_remap if args.xcd_remap >= 0 else tuned.get("xcd_remap", 1),
        prefetch=args.prefetch or tuned.get("prefetch", 0),
    )

    log(f"[bench] generating {n}^3 grid")
    u0 = gi.grid3d(n, seed=1)
    ctx = gf.Context(0)
    u = torch.from_numpy(u0).to("cuda")
    w = u.clone()
    res = torch.zeros(sweeps, dtype=torch.float64, device="cuda")
    sc = torch.zeros(16, dtype=torch.float64, device="cuda")
    inst = gf.Instance.make({programs.J3_U: u, programs.J3_W: w, programs.J3_RES: res}, sc, ip=(n,))
    prog = programs.jacobi3d(sweeps)
    bps = alg_bytes_per_sweep(n)
    bytes_per_run = bps * sweeps

    # achievable ceiling: the copy kernel over 1 GiB
    cbytes = min(u.numel() * 8, 1 << 30)
    for _ in range(2):
        ctx.copy(w, u, cbytes, num_wg=0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        ctx.copy(w, u, cbytes, num_wg=0)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 5 * 2 * cbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9
    w.copy_(u)
    torch.cuda.synchronize()

    log(f"[bench] persistent: {args.warmup} warm-up + {args.steps} timed runs of {sweeps} sweeps")
    ms, kern_ms, stats = time_mode(ctx, gf, torch, prog, inst, gf.GF_EXEC_PERSISTENT, launch, args.steps,
                                   args.warmup)
    gbps = bytes_per_run / (ms * 1e-3) / 1e9
    achieved = bytes_per_run / (kern_ms * 1e-3) / 1e9
    log(f"[bench] persistent {ms:.2f} ms/run, kernel {kern_ms:.2f} ms, {gbps:.1f} GB/s")

    per_region = None
    if not args.no_per_region:
        out = {}
        for name, mode in (("per_region", gf.GF_EXEC_PER_REGION), ("per_region_graph", gf.GF_EXEC_PER_REGION_GRAPH),
                           ("kernel_split", gf.GF_EXEC_KERNEL_SPLIT)):
            log(f"[bench] {name}")
            pms, _, pst = time_mode(ctx, gf, torch, prog, inst, mode, launch, args.steps, args.warmup)
            out[name] = {"ms_per_step": round(pms, 3),
                         "GBps": round(bytes_per_run / (pms * 1e-3) / 1e9, 1),
                         "regions_per_s": round(sweeps / (pms * 1e-3), 1),
                         "launches_per_step": pst["launches"] if pst else None}
            log(f"[bench] {name} {pms:.2f} ms/run")
        per_region = out

    cpu = cpu_omp = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (serial oracle, then the OpenMP build)")
        cpu, cpu_omp = cpu_baseline(u0, n)
        log(f"[bench] cpu {cpu['value']} GB/s over {cpu['sample']}; OpenMP {cpu_omp['value']} GB/s")
        cpu_omp["gpu_speedup"] = round(gbps / cpu_omp["value"], 2)

    traffic = load_traffic(workload)
    line = {
        "metric": METRIC,
        "value": round(gbps, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"jacobi3d_7pt_{n}^3_f64_{sweeps}sweeps_maxres", "n": n, "sweeps": sweeps,
                   "mode": "persistent", "num_wg": stats["num_wg"] if stats else None,
                   "wg_size": stats["wg_size"] if stats else None,
                   "tile_y": launch.tile_y or 8, "tile_z": launch.tile_z or 64, "xcd_remap": launch.xcd_remap},
        "regions_per_s": round(sweeps / (ms * 1e-3), 1),
        "alg_bytes_per_sweep": bps,
        "per_region": per_region,
        "copy_ceiling_GBps": round(copy_gbps, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_GBPS, 4),
                     "traffic": traffic,
                     "kernel": "k_persistent (one launch = %d sweeps)" % sweeps,
                     "kernel_ms": round(kern_ms, 3)},
        "cpu_baseline": cpu,
        "cpu_openmp": cpu_omp,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
