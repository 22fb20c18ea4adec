"""CPU checks of the committed launch-shape predictor: its weights were
trained on the committed dataset (the dataset's hash is recorded in the
weights), and the held-out quality recorded with them is reproduced by the
FP64 oracle forward pass on that dataset (argmin over the runnable shapes,
out-of-distribution nests deferred to the tuner, as at launch time)."""
import hashlib
import json
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2306_11686_amd")


def _load():
    with open(os.path.join(PKG, "predictor_weights.json")) as f:
        model = json.load(f)
    path = os.path.join(PKG, "predictor_dataset.npz")
    d = np.load(path, allow_pickle=False)
    with open(path, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()[:16]
    return model, d, digest


def _params(flat, n_in=8, h=64, k=32):
    p = np.asarray(flat, dtype=np.float64)
    sizes = [("W1", (h, n_in)), ("b1", (h,)), ("W2", (h, h)), ("b2", (h,)), ("W3", (k, h)), ("b3", (k,))]
    out, o = {}, 0
    for name, shape in sizes:
        m = int(np.prod(shape))
        out[name] = p[o:o + m].reshape(shape)
        o += m
    assert o == p.size
    return out


def test_weights_name_the_committed_dataset():
    model, d, digest = _load()
    assert model["dataset_sha256"] == digest
    assert d["f_tr"].shape == (model["train_nests"], 8) and d["f_te"].shape == (model["test_nests"], 8)
    assert d["ms_tr"].shape[1] == 32 and d["ms_te"].shape[1] == 32
    assert len(model["params"]) == 64 * 8 + 64 + 64 * 64 + 64 + 32 * 64 + 32


def test_oracle_forward_reproduces_the_recorded_heldout_quality():
    import oracle
    model, d, _ = _load()
    z = np.log2(1.0 + np.maximum(d["f_te"], 0.0))
    zs = (z - np.asarray(model["mean"])) / np.asarray(model["std"])
    y, _ = oracle.mlp_forward(_params(model["params"]), zs)
    ms = d["ms_te"]
    ratios = []
    for row, yy, zz in zip(ms, y, zs):
        best = np.min(row[np.isfinite(row)])
        if np.any(np.abs(zz) > 4.0):
            ratios.append(1.0)            # out of distribution: the tuner decides
            continue
        k = int(np.argmin(np.where(np.isfinite(row), yy, np.inf)))
        ratios.append(row[k] / best)
    geo = float(np.exp(np.mean(np.log(ratios))))
    rec = model["heldout"]["geomean_ratio"]
    # FP32 device weights evaluated in FP64: near-ties may pick another shape
    assert abs(geo - rec) <= 0.005, (geo, rec)
    assert geo <= 1.10 and geo < model["heldout"]["default_geomean_ratio"]
