"""CPU checks of the autotuner's host logic: argmin over a known cost table
(the library's gf_tune_pick), the tuning-database round trip, and the plan of
a batched launch (gf_batch_plan) against brute force."""
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


def _makespan(items, w, g):
    return max(math.ceil(it / gi) * (wi / it) for it, wi, gi in zip(items, w, g))


def _best_makespan(items, w, budget):
    """Brute force over every group-size vector with sum <= budget."""
    import itertools
    best = math.inf
    ranges = [range(1, min(it, budget) + 1) for it in items]
    for g in itertools.product(*ranges):
        if sum(g) <= budget:
            best = min(best, _makespan(items, w, g))
    return best


def test_batch_plan_group_sizes_reach_the_brute_force_makespan():
    """Without XCD packing the greedy's slowest group is as fast as the best
    possible split of the budget (exhaustive search on small cases)."""
    import paper_2306_11686_amd as gf
    rng = random.Random(3)
    for trial in range(60):
        n = rng.randint(1, 4)
        items = [rng.randint(1, 12) for _ in range(n)]
        w = [it * rng.choice([1.0, 0.5, 2.0, 3.0]) for it in items]
        budget = rng.randint(n, 16)
        grid, g, x = gf.batch_plan(items, w, budget=budget, align=False)
        assert all(v == -1 for v in x)
        assert all(1 <= gi <= it for gi, it in zip(g, items)) and sum(g) == grid <= budget
        assert _makespan(items, w, g) == pytest.approx(_best_makespan(items, w, budget))


def test_batch_plan_packs_groups_onto_xcds():
    """With packing every instance sits on one XCD, at most budget/8
    instances and workgroups per XCD, the grid is 8 x the fullest XCD, and
    the heaviest instances land on different XCDs."""
    import paper_2306_11686_amd as gf
    rng = random.Random(5)
    for trial in range(20):
        n = rng.randint(8, 200)
        items = [rng.randint(1, 2000) for _ in range(n)]
        budget = rng.choice([512, 1024, 4096])
        grid, g, x = gf.batch_plan(items, budget=budget)
        per = budget // 8
        assert all(0 <= xi < 8 for xi in x)
        used = [sum(gi for gi, xi in zip(g, x) if xi == k) for k in range(8)]
        counts = [sum(1 for xi in x if xi == k) for k in range(8)]
        assert max(used) <= per and max(counts) <= per and grid == 8 * max(used)
        top = sorted(range(n), key=lambda i: (-items[i], i))[:8]
        assert len({x[i] for i in top}) == 8
    # more instances than one XCD's share of slots: packing still fits them
    grid, g, x = gf.batch_plan([1] * 64, budget=64)
    assert all(0 <= xi < 8 for xi in x) and grid == 64
    # a budget below 8 cannot be split over the XCDs
    grid, g, x = gf.batch_plan([5, 5, 5], budget=7)
    assert x == [-1, -1, -1] and sum(g) == grid <= 7


def test_batch_plan_rejects_bad_arguments():
    import paper_2306_11686_amd as gf
    with pytest.raises(gf.GfError):
        gf.batch_plan([3, 0], budget=8)
    with pytest.raises(gf.GfError):
        gf.batch_plan([3, 3, 3], budget=2)

