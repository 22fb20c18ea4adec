"""CPU checks of the autotuner's host logic: argmin over a known cost table
(the library's gf_tune_pick) and the tuning-database round trip."""
import math
import random

import pytest


def test_pick_is_exact_argmin_of_mock_cost_table():
    import paper_2306_11686_amd as gf
    rng = random.Random(7)
    for trial in range(50):
        n = rng.randint(1, 40)
        table = [rng.choice([math.inf, rng.uniform(0.1, 10.0)]) for _ in range(n)]
        finite = [i for i, v in enumerate(table) if math.isfinite(v)]
        want = min(finite, key=lambda i: (table[i], i)) if finite else -1
        # float32 rounding in the ABI: compare against the rounded table
        import numpy as np
        t32 = [float(np.float32(v)) for v in table]
        finite32 = [i for i, v in enumerate(t32) if math.isfinite(v)]
        want32 = min(finite32, key=lambda i: (t32[i], i)) if finite32 else -1
        assert gf.tune_pick(table) == want32
        assert want32 == want or t32[want32] == t32[want]


def test_pick_ties_and_nan():
    import paper_2306_11686_amd as gf
    assert gf.tune_pick([2.0, 1.0, 1.0]) == 1
    assert gf.tune_pick([math.nan, 3.0]) == 1
    assert gf.tune_pick([math.inf, math.nan]) == -1


def test_tuning_db_round_trip(tmp_path):
    from paper_2306_11686_amd import tuner
    import paper_2306_11686_amd as gf
    path = str(tmp_path / "db.json")
    l = gf.Launch.make(wg_size=128, num_wg=7, tile_y=4, tile_z=85, items=2, xcd_remap=0)
    db = tuner.load_db(path)
    db["k"] = tuner.launch_to_dict(l)
    tuner.save_db(db, path)
    back = tuner.lookup("k", path)
    assert tuner.launch_to_dict(back) == tuner.launch_to_dict(l)
    assert tuner.lookup("missing", path) is None
