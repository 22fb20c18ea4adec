"""Generate the predictor's dataset with the autotuner, train the MLP on the
device, evaluate on held-out nests and save the weights.

    python -m paper_2306_11686_amd.train_predictor [--train 2000] [--test 200]
           [--epochs 3000] [--reps 3] [--dataset PATH.npz] [--out paper_2306_11686_amd/predictor_weights.json]

With --dataset, the tuned timings are saved there (compressed numpy, no
pickles) or, if the file exists, loaded from it instead of tuning again, so
the weights can be rebuilt from a committed dataset. The weights record the
region kernels' source hash and the dataset's hash.

Prints one JSON line with the held-out quality: geometric mean of
t(predicted) / t(best) over the nests, the fraction within 1.10, and the same
ratio for the best single fixed launch shape (the method without the learned
part), plus tuning versus inference cost.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=None)
    ap.add_argument("--dataset", default=None, help="save/load the tuned dataset (.npz)")
    ap.add_argument("--recheck", action="store_true",
                    help="time the held-out nests again and score the predictor and the tuner's own choice "
                         "on the fresh timings (the tuner's re-measurement floor)")
    args = ap.parse_args()

    import torch  # noqa: F401
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import predictor

    ctx = gf.Context(0)
    specs_tr = predictor.sample_nests(args.train, seed=args.seed)
    specs_te = predictor.sample_nests(args.test, seed=args.seed, first=args.train)
    t0 = time.perf_counter()
    loaded = False
    if args.dataset:
        try:
            d = np.load(args.dataset)
            f_tr, ms_tr, f_te, ms_te = d["f_tr"], d["ms_tr"], d["f_te"], d["ms_te"]
            loaded = True
        except OSError:
            pass
    if not loaded:
        f_tr, ms_tr = predictor.collect(ctx, specs_tr, reps=args.reps, log=log)
        f_te, ms_te = predictor.collect(ctx, specs_te, reps=args.reps, log=log)
        if args.dataset:
            np.savez_compressed(args.dataset, f_tr=f_tr, ms_tr=ms_tr, f_te=f_te, ms_te=ms_te)
    tune_s = time.perf_counter() - t0
    log(f"[predictor] dataset ready in {tune_s:.1f} s")

    t0 = time.perf_counter()
    model = predictor.train(ctx, f_tr, ms_tr, epochs=args.epochs, lr=args.lr, seed=args.seed)
    train_s = time.perf_counter() - t0
    hist = model["loss_history"]
    log(f"[predictor] trained {args.epochs} epochs in {train_s:.2f} s, loss {hist[0]:.4f} -> {hist[-1]:.4f}")

    t0 = time.perf_counter()
    pred_te = predictor.predict_indices(ctx, model, f_te, valid=np.isfinite(ms_te))
    infer_us = (time.perf_counter() - t0) / max(1, len(f_te)) * 1e6
    pred_tr = predictor.predict_indices(ctx, model, f_tr, valid=np.isfinite(ms_tr))
    # best single fixed shape on the training set (per family shapes differ in
    # meaning, so the fixed baseline is chosen per kind)
    kinds_tr = [s["kind"] for s in specs_tr]
    kinds_te = [s["kind"] for s in specs_te]
    fixed = {}
    for k in set(kinds_tr):
        rows = ms_tr[[i for i, kk in enumerate(kinds_tr) if kk == k]]
        best = np.min(np.where(np.isfinite(rows), rows, np.inf), axis=1, keepdims=True)
        lr_ = np.where(np.isfinite(rows), np.log(rows / best), np.inf)
        fixed[k] = int(np.argmin(np.mean(np.where(np.isfinite(lr_), lr_, 10.0), axis=0)))
    fixed_te = [fixed.get(k, 0) for k in kinds_te]
    ev_te = predictor.evaluate(pred_te, ms_te, default_idx=fixed_te)
    ev_tr = predictor.evaluate(pred_tr, ms_tr)
    per_kind = {}
    for k in sorted(set(kinds_te)):
        idx = [i for i, kk in enumerate(kinds_te) if kk == k]
        e = predictor.evaluate([pred_te[i] for i in idx], ms_te[idx], default_idx=[fixed_te[i] for i in idx])
        per_kind[k] = {"n": e["n"], "geomean_ratio": round(e["geomean_ratio"], 4),
                       "fixed_geomean_ratio": round(e.get("default_geomean_ratio", float("nan")), 4)}
    recheck = None
    if args.recheck:
        _, ms_te2 = predictor.collect(ctx, specs_te, reps=args.reps, log=log)
        tuner_pick = [int(np.argmin(np.where(np.isfinite(r), r, np.inf))) for r in ms_te]
        ev_pred2 = predictor.evaluate(pred_te, ms_te2)
        ev_tuner2 = predictor.evaluate(tuner_pick, ms_te2)
        recheck = {"predictor_geomean_ratio": round(ev_pred2["geomean_ratio"], 4),
                   "predictor_frac_within_1_10": round(ev_pred2["frac_within_1_10"], 4),
                   "tuner_geomean_ratio": round(ev_tuner2["geomean_ratio"], 4),
                   "tuner_frac_within_1_10": round(ev_tuner2["frac_within_1_10"], 4)}
    tune_per_nest_ms = tune_s / max(1, len(specs_tr) + len(specs_te)) * 1e3
    import hashlib
    from .build import kernel_source_hash
    ds_hash = None
    if args.dataset:
        with open(args.dataset, "rb") as f:
            ds_hash = hashlib.sha256(f.read()).hexdigest()[:16]
    model.update({"kernel_source_hash": kernel_source_hash(), "dataset": args.dataset, "dataset_sha256": ds_hash,
                  "dataset_reused": loaded})
    model.update({"train_nests": args.train, "test_nests": args.test, "epochs": args.epochs, "lr": args.lr,
                  "heldout": ev_te, "train_fit": ev_tr, "per_kind": per_kind, "fixed_shapes": fixed,
                  "heldout_retimed": recheck})
    out = args.out or predictor.WEIGHTS
    predictor.save(model, out)
    line = {"metric": "launch-config predictor: geomean t(pred)/t(best) on held-out nests",
            "value": round(ev_te["geomean_ratio"], 4), "frac_within_1_10": round(ev_te["frac_within_1_10"], 4),
            "max_ratio": round(ev_te["max_ratio"], 3), "fallbacks_to_tuner": ev_te["fallbacks"],
            "fixed_best_shape_geomean_ratio": round(ev_te["default_geomean_ratio"], 4),
            "train_fit_geomean_ratio": round(ev_tr["geomean_ratio"], 4), "per_kind": per_kind,
            "train_nests": args.train, "test_nests": args.test, "epochs": args.epochs,
            "loss_first": round(hist[0], 5), "loss_last": round(hist[-1], 5),
            "train_seconds": round(train_s, 3), "inference_us_per_nest_host": round(infer_us, 2),
            "tuning_ms_per_nest": round(tune_per_nest_ms, 2)}
    if recheck:
        line["heldout_retimed"] = recheck
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
