"""Measure the legacy-loop workloads other than the benchmark's headline.

    python -m paper_2306_11686_amd.measure [--configs sync,2d,rpc,rpc_fprintf,phases,heap,cg,hist,batched]
                                           [--reps 3]

Each configuration prints one JSON line: time per run in the persistent,
per-region and per-region-graph modes, regions per second, and algorithmic
GB/s (bytes the sweep-at-a-time legacy loops must move; for the 2D grid the
working set is cache-resident, so its GB/s is labelled as such).
Launch shapes come from the tuning database when present.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import workloads

MODES = (("persistent", 1), ("per_region", 0), ("per_region_graph", 2), ("kernel_split", 3))
ONLY_MODES = None  # --modes: restrict every config to these execution modes


def modes(sel=MODES):
    return tuple(m for m in sel if ONLY_MODES is None or m[0] in ONLY_MODES)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _time(ctx, torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    ctx.sync()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ctx.sync()
    return float(np.median(ts))


def _launch(tuner, key, mode=1):
    """The tuned launch for `key`; the per-region modes (0, 2) take the one
    tuned in per-region mode when the database has it."""
    if mode in (0, 2):
        per_region = tuner.lookup(key + "@per_region")
        if per_region is not None:
            return per_region
    return tuner.lookup(key)


def measure_2d(ctx, gf, programs, tuner, torch, reps):
    n, sweeps = 256, 100
    bpsweep = 8 * (n * n - 4) + 8 * (n - 2) ** 2
    out = {"config": "jacobi2d_5pt_256^2_f64_100sweeps_l2res_printf10", "alg_bytes_per_sweep": bpsweep}
    launch = _launch(tuner, "jacobi2d_256")
    for pf in (True, False):
        prog, inst, keep, _ = workloads.jacobi2d(ctx, n, sweeps, printf=pf)
        for name, mode in modes():
            ms = _time(ctx, torch, lambda: ctx.run(prog, inst, mode=mode, launch=launch), reps)
            ctx.take_output()
            key = name + ("" if pf else "_no_printf")
            out[key] = {"ms_per_run": round(ms, 4), "us_per_region": round(ms * 1e3 / sweeps, 3),
                        "regions_per_s": round(sweeps / (ms * 1e-3), 1),
                        "GBps_cache_resident": round(bpsweep * sweeps / (ms * 1e-3) / 1e9, 1)}
    for name, _ in modes():
        out[name]["printf_us_each"] = round((out[name]["ms_per_run"] - out[name + "_no_printf"]["ms_per_run"])
                                            * 1e3 / 10, 3)
    return out


def measure_cg(ctx, gf, programs, tuner, torch, reps):
    m, iters = 128, 500
    prog, inst, keep, reset = workloads.cg(m, iters)
    N = m ** 3
    nnz = (3 * m - 2) ** 3
    spmv_b = 12 * nnz + 4 * (N + 1) + 8 * N + 8 * N
    # dot(p, q) reads two vectors, dot(r, r) one; each axpby reads two and writes one
    it_b = spmv_b + 16 * N + 8 * N + 3 * 24 * N
    out = {"config": f"cg_27pt_{m}^3_f64_{iters}iters", "rows": N, "nnz": nnz, "alg_bytes_per_iteration": it_b}
    for name, mode in modes():
        reset()
        launch = _launch(tuner, "cg_128", mode)
        ms = _time(ctx, torch, lambda: ctx.run(prog, inst, mode=mode, launch=launch), reps)
        out[name] = {"ms_per_run": round(ms, 3), "GBps": round(iters * it_b / (ms * 1e-3) / 1e9, 1),
                     "regions_per_s": round(6 * iters / (ms * 1e-3), 1)}
    return out


def measure_hist(ctx, gf, programs, tuner, torch, reps):
    n = 1 << 28
    out = {"config": "hist_u32_2^28_keys_65536_bins", "alg_bytes": 4 * n + 2 * 4 * 65536}
    for dist in ("uniform", "zipf"):
        prog, inst, keep, _ = workloads.histogram(n, 65536, dist)
        for name, mode in modes(MODES[:2]):
            launch = _launch(tuner, "hist_2^28", mode)
            ms = _time(ctx, torch, lambda: ctx.run(prog, inst, mode=mode, launch=launch), reps)
            out[f"{dist}_{name}"] = {"us_per_run": round(ms * 1e3, 1),
                                     "GBps": round(out["alg_bytes"] / (ms * 1e-3) / 1e9, 1)}
        del keep, inst
        torch.cuda.empty_cache()
    return out


def measure_batched(ctx, gf, programs, tuner, torch, reps):
    sweeps = 50
    prog, insts, keep, _ = workloads.batched(256, sweeps)
    sides = [int(i.ip[0]) for i in insts]
    bytes_per_sweepset = int(sum(8 * (n ** 2 - 4) + 8 * (n - 2) ** 2 for n in sides))
    out = {"config": "batched_256x_jacobi2d_sides_64_2048_50sweeps", "sum_n2": int(sum(n * n for n in sides)),
           "alg_bytes_per_run": bytes_per_sweepset * sweeps, "regions_per_run": 256 * sweeps}
    per = tuner.lookup_batched("batched_256")   # a shape per instance, from the batched autotuner
    out["per_instance_shapes"] = per is not None

    def run(mode):
        # the per-instance plan is the persistent launch's; the per-region
        # modes launch every instance with the shape tuned in that mode
        if per is not None and mode == 1:
            return ctx.run_batched(prog, insts, per, mode=mode)
        return ctx.run(prog, insts, mode=mode, launch=_launch(tuner, "batched_256", mode))

    for name, mode in modes(MODES[:3]):          # the kernel split runs one instance
        ms = _time(ctx, torch, lambda: run(mode), reps)
        if mode == 1:
            out["persistent_misplaced_workgroups"] = ctx.batch_misplaced()
        out[name] = {"ms_per_run": round(ms, 3), "GBps": round(out["alg_bytes_per_run"] / (ms * 1e-3) / 1e9, 1),
                     "regions_per_s": round(256 * sweeps / (ms * 1e-3), 1)}
    return out


def measure_sync(ctx, gf, programs, tuner, torch, reps):
    """Cost of one region of a trivial program (3D Jacobi on a 4^3 grid, one
    interior point): the grid barrier plus serial glue in the persistent mode,
    the launch gap in the per-region modes, at several grid sizes."""
    regions = 2000
    u = torch.zeros(64, dtype=torch.float64, device="cuda")
    w = u.clone()
    r = torch.zeros(regions, dtype=torch.float64, device="cuda")
    sc = torch.zeros(16, dtype=torch.float64, device="cuda")
    inst = gf.Instance.make({0: u, 1: w, 2: r}, sc, ip=(4,))
    prog = programs.jacobi3d(regions)
    out = {"config": "sync_cost_trivial_region", "regions": regions}
    launch = gf.Launch.make(tile_y=1)
    for nwg in (1, 64, 256, 512, 768):
        try:
            ms = _time(ctx, torch, lambda: ctx.run(prog, inst, mode=1, launch=gf.Launch.make(tile_y=1, num_wg=nwg)),
                       reps)
        except gf.GfError:          # beyond the co-resident capacity
            continue
        out[f"persistent_wg{nwg}_us_per_region"] = round(ms * 1e3 / regions, 3)
    for name, mode in MODES[1:]:
        ms = _time(ctx, torch, lambda: ctx.run(prog, inst, mode=mode, launch=launch), reps)
        out[f"{name}_us_per_region"] = round(ms * 1e3 / regions, 3)
    # a whole program of one region, launched 200 times back to back: the
    # fixed cost of a cooperative launch (persistent) against a plain one
    one = programs.jacobi3d(1)
    runs = 200

    def repeat(mode, l):
        for _ in range(runs):
            ctx.run(one, inst, mode=mode, launch=l)

    for name, mode, l in (("persistent_wg256", 1, gf.Launch.make(tile_y=1, num_wg=256)),
                          ("per_region", 0, launch)):
        ms = _time(ctx, torch, lambda: repeat(mode, l), reps)
        out[f"one_region_program_{name}_us"] = round(ms * 1e3 / runs, 3)
    return out


def measure_rpc(ctx, gf, programs, tuner, torch, reps):
    """RPC round trips: a persistent program whose body is one printf of an
    int and a double, run 1000 times by one workgroup, posted (the device
    continues at once) and blocking (the device waits until the host has
    printed and marked the slot done); a server thread polls the ring."""
    calls = 1000
    fmt = ctx.register_format("call %d value %.6e\n", "id")
    sc = torch.zeros(16, dtype=torch.float64, device="cuda")
    inst = gf.Instance.make({}, sc, ip=())
    out = {"config": "rpc_printf_1000_calls", "calls": calls}
    for name, flags in (("posted", 0), ("blocking", gf.GF_STEP_BLOCKING)):
        body = [gf.Step.make(gf.GF_S_SET, sc=(0,), c=3.25),
                gf.Step.make(gf.GF_S_PRINTF, sc=(0,), every=1, fmt_id=fmt, nargs=2, flags=flags)]
        prog = gf.Program.make([], body, calls)
        launch = gf.Launch.make(num_wg=1)
        ms = _time(ctx, torch, lambda: ctx.run(prog, inst, mode=gf.GF_EXEC_PERSISTENT, launch=launch), reps)
        text = ctx.take_output()
        out[name] = {"ms_per_run": round(ms, 3), "us_per_call": round(ms * 1e3 / calls, 2),
                     "lines_captured": text.count("\n")}
    return out


def measure_rpc_fprintf(ctx, gf, programs, tuner, torch, reps):
    """The paper's RPC benchmark shape (Section 5, "RPC Performance"): 1000
    blocking fprintf calls whose format string and 128-byte buffer are
    passed by reference. The buffer goes both ways when its access mode is
    unknown (read-write, the paper's case), and only to the host when it is
    known to be read-only. The stream is /dev/null without buffering, so
    every call makes one write system call, as fprintf to stderr does. The
    per-stage times are averages over all timed calls."""
    import ctypes
    calls = 1000
    libc = ctypes.CDLL(None)
    libc.fopen.restype = ctypes.c_void_p
    f = libc.fopen(b"/dev/null", b"w")
    if not f:
        return {"config": "rpc_fprintf_1000_calls_128B_buffer", "error": "cannot open /dev/null"}
    libc.setvbuf(ctypes.c_void_p(f), None, 2, 0)  # _IONBF
    fmt = b"buffer holds: %s\n\0"
    text = (b"legacy program output line " * 5)[:120] + b"\0"
    fmt_arr = torch.zeros(32, dtype=torch.uint8)
    fmt_arr[:len(fmt)] = torch.tensor(list(fmt), dtype=torch.uint8)
    buf = torch.zeros(128, dtype=torch.uint8)
    buf[:len(text)] = torch.tensor(list(text), dtype=torch.uint8)
    d_fmt, d_buf = fmt_arr.cuda(), buf.cuda()
    sc = torch.zeros(16, dtype=torch.float64, device="cuda")
    out = {"config": "rpc_fprintf_1000_calls_128B_buffer", "calls": calls}
    with gf.Context(0, rpc_thread=True) as c2:
        for name, bmode in (("buffer_read_write", gf.GF_REF_READWRITE), ("buffer_read_only", gf.GF_REF_READ)):
            cid = c2.register_call(gf.GF_CALLEE_FPRINTF, [
                gf.CallArg.const(f, "p"), gf.CallArg.ref(1, len(fmt), mode=gf.GF_REF_READ),
                gf.CallArg.ref(0, 128, mode=bmode)])
            body = [gf.Step.make(gf.GF_S_CALL, fmt_id=cid, every=1, flags=gf.GF_STEP_BLOCKING | gf.GF_STEP_TIMED)]
            prog = gf.Program.make([], body, calls)
            inst = gf.Instance.make({0: d_buf, 1: d_fmt}, sc)
            launch = gf.Launch.make(num_wg=1, wg_size=64)
            ms = _time(c2, torch, lambda: c2.run(prog, inst, mode=gf.GF_EXEC_PERSISTENT, launch=launch), reps)
            st = c2.call_stats(cid, reset=True)
            dev_total = st["dev_args_us"] + st["dev_copy_in_us"] + st["dev_wait_us"] + st["dev_copy_out_us"]
            out[name] = {"ms_per_run": round(ms, 3), "us_per_call": round(ms * 1e3 / calls, 3),
                         "stages_us": {k: round(v, 3) for k, v in st.items() if k != "calls"},
                         "device_stage_share": {k: round(st[k] / dev_total, 4) for k in
                                                ("dev_args_us", "dev_copy_in_us", "dev_wait_us",
                                                 "dev_copy_out_us")},
                         "timed_calls": st["calls"]}
    libc.fclose(ctypes.c_void_p(f))
    return out


def measure_phases(ctx, gf, programs, tuner, torch, reps):
    """A `parallel` region with manual worksharing: 2^22 doubles, 100
    producer/consumer phases separated by barriers across all workgroups
    (the persistent kernel's barrier, or the per-region kernel's own).
    Each thread walks its own contiguous block, as the legacy code does, so
    a wavefront's accesses are strided by the block length. Algorithmic
    bytes per phase: one read of the source and one write of the
    destination, 16 n."""
    n, P, shift = 1 << 22, 100, (1 << 22) // 3
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    sc = torch.zeros(16, dtype=torch.float64, device="cuda")
    inst = gf.Instance.make({0: a, 1: b}, sc, ip=(n,))
    prog = programs.phases(P, shift, owner=False)
    out = {"config": "phases_2^22_f64_100phases", "alg_bytes_per_phase": 16 * n}
    for name, mode in modes(MODES[:2]):
        for nwg in (256, 1024):
            launch = gf.Launch.make(wg_size=256, num_wg=nwg)
            try:
                ms = _time(ctx, torch, lambda: ctx.run(prog, inst, mode=mode, launch=launch), reps)
            except gf.GfError:
                continue
            st = ctx.run(prog, inst, mode=mode, launch=launch)
            ctx.sync()
            out[f"{name}_wg{nwg}"] = {"ms_per_run": round(ms, 3), "us_per_phase": round(ms * 1e3 / P, 2),
                                      "GBps": round(16 * n * P / (ms * 1e-3) / 1e9, 1), "grid": st["num_wg"]}
    return out


def measure_heap(ctx, gf, programs, tuner, torch, reps):
    """The allocator benchmark's shape (Section 5.1, "Allocator Performance"):
    every thread of every team allocates a block at the start of the kernel,
    uses it (writes and checks 128 bytes) and frees it. The balanced heap runs
    with 32 thread slots and 16 team slots (the configuration the paper
    measures) and with 64 x 32 (one thread slot per lane of a 64-wide
    wavefront), beside the HIP runtime's device malloc."""
    out = {"config": "heap_roundtrip_128B", "bytes": 128}
    heaps = {"balanced": gf.Heap(0, 1 << 28, 32, 16, 4), "balanced64x32": gf.Heap(0, 1 << 28, 64, 32, 4),
             "hip_malloc": gf.Heap(0, 1 << 28, vendor=True)}
    try:
        for teams in (1, 32, 64, 128, 256):
            for threads in (1, 32, 64, 128, 256):
                row = {}
                for name, h in heaps.items():
                    ms = _time(ctx, torch, lambda: h.bench(teams, threads, 128), reps)
                    row[name + "_us"] = round(ms * 1e3, 2)
                    c = h.counts(reset=True)
                    if any(c.values()):
                        row[name + "_errors"] = c
                row["speedup"] = round(row["hip_malloc_us"] / row["balanced_us"], 2)
                row["speedup64x32"] = round(row["hip_malloc_us"] / row["balanced64x32_us"], 2)
                out[f"teams{teams}_threads{threads}"] = row
    finally:
        for h in heaps.values():
            h.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", default="sync,2d,rpc,rpc_fprintf,phases,heap,cg,hist,batched")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--modes", default=None, help="comma list of execution modes to run (default: all)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy 1 GiB three times first (calibrates rocprofv3 byte counters per dispatch)")
    args = ap.parse_args()
    global ONLY_MODES
    if args.modes:
        ONLY_MODES = set(args.modes.split(","))
    import torch
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs, tuner
    ctx = gf.Context(0, rpc_capture=True, rpc_thread=True)
    if args.copy_probe:
        a = torch.zeros(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            ctx.copy(b, a, 1 << 30, num_wg=0)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    fns = {"sync": measure_sync, "2d": measure_2d, "rpc": measure_rpc, "rpc_fprintf": measure_rpc_fprintf,
           "phases": measure_phases, "heap": measure_heap, "cg": measure_cg, "hist": measure_hist,
           "batched": measure_batched}
    for c in args.configs.split(","):
        log(f"[measure] {c}")
        print(json.dumps(fns[c](ctx, gf, programs, tuner, torch, args.reps)), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
