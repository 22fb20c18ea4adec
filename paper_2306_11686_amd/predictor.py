"""Learned launch-config predictor: dataset, training and evaluation.

A loop nest is one region of the legacy-loop families (2D/3D Jacobi sweep,
CSR SpMV, dot, axpby, histogram) at a sampled size. Its label is the
autotuner's measurement of all GF_NUM_CANDIDATES launch shapes (gf_tune on
real runs); the network regresses t_c = log(time_c / min time) on the eight
loop features the library computes (gf_nest_features) and is trained on the
device by the library's own forward, backward and Adam kernels. At launch
time (gf_region_run without a launch, or gf_predict_launch) the argmin over
the predicted t_c of the runnable shapes is used; nests outside the training
distribution defer to the autotuner.

Timing inputs are device-random (their values do not change the timings);
the sizes and structure follow the workload families.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import gf_inputs as gi

from . import programs
from .binding import (GF_EXEC_PERSISTENT, GF_MLP_HIDDEN, GF_MLP_IN, GF_MLP_NPARAMS, GF_MLP_OUT, GF_OP_SUM,
                      GF_R_AXPBY, GF_R_DOT, GF_R_SPMV, Instance, Program, Step)

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predictor_weights.json")
KINDS = ("j2", "j3", "spmv", "dot", "axpby", "hist")
KIND_P = (0.2, 0.25, 0.15, 0.1, 0.1, 0.2)
CSR_GRIDS = (16, 24, 32, 48, 64, 80, 96, 112, 128)


def sample_nests(count: int, seed: int = 1, first: int = 0):
    """Nest specs drawn from stream 7 of the input generator (index = nest * 8 + k)."""
    specs = []
    for i in range(first, first + count):
        u = gi.u01(seed, gi.STREAM_NESTS, np.arange(i * 8, i * 8 + 8, dtype=np.uint64))
        kind = KINDS[int(np.searchsorted(np.cumsum(KIND_P), u[0] * sum(KIND_P), side="right"))]
        if kind == "j2":
            spec = {"kind": kind, "n": int(64 * 64 ** u[1])}                     # [64, 4096)
        elif kind == "j3":
            spec = {"kind": kind, "n": int(32 * 16 ** u[1])}                     # [32, 512)
        elif kind in ("spmv", "dot", "axpby"):
            spec = {"kind": kind, "m": CSR_GRIDS[int(u[1] * len(CSR_GRIDS))]}
        else:
            spec = {"kind": kind, "keys": int(2 ** (16 + 12 * u[1])), "bins": 2 ** (8 + int(u[2] * 9)),
                    "zipf": bool(u[3] < 0.5)}
        specs.append(spec)
    return specs


_CSR_CACHE = {}


def build_nest(spec):
    """Device tensors, program and instance for one timing nest."""
    import torch
    k = spec["kind"]
    sc = torch.zeros(16, dtype=torch.float64, device="cuda")
    keep = [sc]
    if k in ("j2", "j3"):
        n = spec["n"]
        shape = (n, n) if k == "j2" else (n, n, n)
        u = torch.rand(shape, dtype=torch.float64, device="cuda")
        w = u.clone()
        res = torch.zeros(1, dtype=torch.float64, device="cuda")
        keep += [u, w, res]
        prog = programs.jacobi2d(1) if k == "j2" else programs.jacobi3d(1)
        inst = Instance.make({0: u, 1: w, 2: res}, sc, ip=(n,))
        return prog, inst, keep
    if k in ("spmv", "dot", "axpby"):
        m = spec["m"]
        N = m ** 3
        x = torch.rand(N, dtype=torch.float64, device="cuda")
        y = torch.rand(N, dtype=torch.float64, device="cuda")
        keep += [x, y]
        if k == "spmv":
            if m not in _CSR_CACHE:
                rp, col, val = gi.poisson27_csr(m)
                _CSR_CACHE[m] = (torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(),
                                 torch.from_numpy(val).cuda())
            rp, col, val = _CSR_CACHE[m]
            keep += [rp, col, val]
            prog = Program.make([Step.make(GF_R_SPMV, arr=(0, 1, 2, 3, 4), np=0)], [], 0)
            inst = Instance.make({0: rp, 1: col, 2: val, 3: x, 4: y}, sc, ip=(N,))
        elif k == "dot":
            prog = Program.make([Step.make(GF_R_DOT, arr=(0, 1), sc=(0,), red_op=GF_OP_SUM, np=0)], [], 0)
            inst = Instance.make({0: x, 1: y}, sc, ip=(N,))
        else:
            prog = Program.make([Step.make(GF_R_AXPBY, arr=(1, 0, 1), sc=(-1, 1), c=1.0, np=0)], [], 0)
            inst = Instance.make({0: x, 1: y}, sc, ip=(N,))
        return prog, inst, keep
    nk, nb = spec["keys"], spec["bins"]
    if spec["zipf"]:
        cdf = torch.from_numpy(gi.zipf_cdf(nb, 1.1)).cuda()
        uu = torch.rand(nk, dtype=torch.float64, device="cuda")
        keys = torch.clamp(torch.searchsorted(cdf, uu), max=nb - 1).to(torch.int32)
    else:
        keys = torch.randint(0, 2 ** 31 - 1, (nk,), dtype=torch.int32, device="cuda")
    bins = torch.zeros(nb, dtype=torch.int32, device="cuda")
    keep += [keys, bins]
    return programs.histogram(nb), Instance.make({0: keys, 1: bins}, sc, ip=(nk,)), keep


def collect(ctx, specs, reps: int = 3, log=None):
    """Exhaustive autotuning of every nest: returns (features [N,8], ms [N,32])."""
    feats = np.zeros((len(specs), GF_MLP_IN))
    ms = np.full((len(specs), GF_MLP_OUT), np.inf)
    for i, spec in enumerate(specs):
        prog, inst, keep = build_nest(spec)
        t, _ = ctx.tune(prog, inst, mode=GF_EXEC_PERSISTENT, reps=reps)
        feats[i] = ctx.nest_features(prog, inst)
        ms[i] = t
        del keep
        if log and (i + 1) % 100 == 0:
            log(f"[predictor] tuned {i + 1}/{len(specs)} nests")
    return feats, ms


def transform(raw: np.ndarray) -> np.ndarray:
    return np.log2(1.0 + np.maximum(raw, 0.0))


def targets(ms: np.ndarray):
    best = np.min(np.where(np.isfinite(ms), ms, np.inf), axis=1, keepdims=True)
    mask = np.isfinite(ms).astype(np.float32)
    t = np.where(mask > 0, np.log(np.where(mask > 0, ms, 1.0) / best), 0.0).astype(np.float32)
    return t, mask


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initialisation of W1, W2, W3; zero biases."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(GF_MLP_HIDDEN * GF_MLP_IN) * math.sqrt(2.0 / GF_MLP_IN), np.zeros(GF_MLP_HIDDEN),
             rng.standard_normal(GF_MLP_HIDDEN * GF_MLP_HIDDEN) * math.sqrt(2.0 / GF_MLP_HIDDEN),
             np.zeros(GF_MLP_HIDDEN),
             rng.standard_normal(GF_MLP_OUT * GF_MLP_HIDDEN) * math.sqrt(1.0 / GF_MLP_HIDDEN), np.zeros(GF_MLP_OUT)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == GF_MLP_NPARAMS
    return p


def train(ctx, raw_feats, ms, epochs: int = 2000, lr: float = 3e-3, seed: int = 0):
    """Standardise log features, train on the device; returns a model dict."""
    import torch
    z = transform(raw_feats)
    mean = z.mean(axis=0)
    std = z.std(axis=0)
    std[std == 0] = 1.0
    zs = ((z - mean) / std).astype(np.float32)
    t, mask = targets(ms)
    n = zs.shape[0]
    p = torch.from_numpy(init_params(seed)).cuda()
    m = torch.zeros(GF_MLP_NPARAMS, device="cuda")
    v = torch.zeros(GF_MLP_NPARAMS, device="cuda")
    hist = torch.zeros(max(1, epochs), device="cuda")
    ctx.train_predictor(p, m, v, torch.from_numpy(zs).cuda(), torch.from_numpy(t).cuda(),
                        torch.from_numpy(mask).cuda(), n, 1.0 / float(mask.sum()), epochs, lr, hist)
    torch.cuda.synchronize()
    return {"params": p.cpu().numpy().tolist(), "mean": mean.tolist(), "std": std.tolist(),
            "loss_history": hist.cpu().numpy().tolist()}


def predict_indices(ctx, model, raw_feats, valid=None):
    """Predicted candidate per nest; valid (optional, [N,32] bool) restricts
    the argmin to shapes that can run."""
    ctx.predictor_set(model["params"], model["mean"], model["std"])
    if valid is None:
        return [ctx.predict(f) for f in raw_feats]
    return [ctx.predict(f, valid=v) for f, v in zip(raw_feats, valid)]


def evaluate(pred_idx, ms, default_idx=None):
    """Per-nest t(pred)/t(best) (OOD predictions fall back to the tuner: 1.0)."""
    ratios, fallback = [], 0
    for k, row in zip(pred_idx, ms):
        best = np.min(row[np.isfinite(row)])
        if k < 0 or not np.isfinite(row[k]):
            ratios.append(1.0)
            fallback += 1
        else:
            ratios.append(row[k] / best)
    r = np.array(ratios)
    out = {"geomean_ratio": float(np.exp(np.mean(np.log(r)))), "frac_within_1_10": float(np.mean(r <= 1.10)),
           "max_ratio": float(r.max()), "fallbacks": fallback, "n": len(r)}
    if default_idx is not None:
        d = []
        for k, row in zip(default_idx, ms):
            best = np.min(row[np.isfinite(row)])
            d.append(row[k] / best if np.isfinite(row[k]) else np.nan)
        d = np.array(d)
        d = d[np.isfinite(d)]
        out["default_geomean_ratio"] = float(np.exp(np.mean(np.log(d))))
    return out


def save(model, path: str = WEIGHTS):
    with open(path, "w") as f:
        json.dump(model, f)


def load(path: str = WEIGHTS):
    with open(path) as f:
        return json.load(f)
