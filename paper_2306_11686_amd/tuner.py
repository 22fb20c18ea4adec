"""Tuning database around the library's autotuner (gf_tune).

The autotuner itself (candidate decoding, timing with HIP events, argmin)
runs in libgf; this module keeps its results in a JSON database keyed by a
workload name so that later runs (the benchmark, gf_region_run callers) can
reuse the winning launch without timing again.
"""
from __future__ import annotations

import json
import math
import os

from .binding import GF_EXEC_PERSISTENT, Launch

DEFAULT_DB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_db.json")
_FIELDS = ("wg_size", "num_wg", "tile_y", "tile_z", "items", "xcd_remap", "prefetch")


def launch_to_dict(l: Launch) -> dict:
    return {f: int(getattr(l, f)) for f in _FIELDS}


def dict_to_launch(d: dict) -> Launch:
    return Launch.make(**{f: int(d.get(f, 0 if f != "xcd_remap" else 1)) for f in _FIELDS})


def load_db(path: str = DEFAULT_DB) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_db(db: dict, path: str = DEFAULT_DB) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(key: str, path: str = DEFAULT_DB):
    e = load_db(path).get(key)
    return dict_to_launch(e) if e else None


def tune(ctx, program, instances, key: str | None = None, mode: int = GF_EXEC_PERSISTENT, reps: int = 3,
         candidates=None, path: str = DEFAULT_DB):
    """Time the candidates on real runs, record the best under `key`.

    Returns (best Launch, list of (Launch, ms))."""
    cands = candidates if candidates is not None else ctx.tune_candidates(program, instances if not isinstance(
        instances, (list, tuple)) else instances[0])
    ms, best = ctx.tune(program, instances, mode=mode, candidates=cands, reps=reps)
    if best < 0:
        raise RuntimeError("no candidate launch could run")
    if key is not None:
        db = load_db(path)
        e = launch_to_dict(cands[best])
        e["ms"] = round(ms[best], 4)
        e["mode"] = int(mode)
        db[key] = e
        save_db(db, path)
    return cands[best], [(c, m) for c, m in zip(cands, ms)]


def ratio_to_best(ms) -> list:
    finite = [m for m in ms if math.isfinite(m)]
    b = min(finite)
    return [m / b if math.isfinite(m) else math.inf for m in ms]


def lookup_batched(key: str, path: str = DEFAULT_DB):
    """The per-instance launches a batched tuning recorded under `key`, or None."""
    e = load_db(path).get(key)
    if not e or "per_instance" not in e:
        return None
    return [Launch.make(wg_size=int(e.get("wg_size", 0)), tile_y=int(ty), num_wg=int(wt),
                        xcd_remap=int(e.get("xcd_remap", 1))) for ty, wt in e["per_instance"]]


def tune_batched(ctx, program, instances, key: str | None = None, reps: int = 3, path: str = DEFAULT_DB):
    """The library's batched autotuner (gf_tune_batched): a shape per instance;
    records (rows per tile, relative share) per instance under `key`.
    Returns (launches, median ms of the chosen plan)."""
    launches, ms = ctx.tune_batched(program, instances, reps=reps)
    if key is not None:
        db = load_db(path)
        db[key] = {"wg_size": int(launches[0].wg_size), "xcd_remap": int(launches[0].xcd_remap),
                   "per_instance": [[int(l.tile_y), int(l.num_wg)] for l in launches],
                   "ms": round(ms, 4), "mode": int(GF_EXEC_PERSISTENT)}
        save_db(db, path)
    return launches, ms
