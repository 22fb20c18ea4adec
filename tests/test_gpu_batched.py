"""GPU parity of the batched persistent launch: many uneven 2D Jacobi
instances in one cooperative launch, each on its own group of workgroups.
Every instance must equal the oracle on that instance (grid bit-exact,
residuals within 1e-12 of the compensated sum) and, bit for bit, the same
program run alone."""
import numpy as np
import pytest

import gf_inputs as gi
from tests.gpu_helpers import dev, host, run_jacobi2d

pytestmark = pytest.mark.gpu


def _batch(gf, programs, sides, sweeps, seed=1):
    import torch
    us, ws, rs, scs, insts = [], [], [], [], []
    for i, n in enumerate(sides):
        u = dev(gi.batched_grid(i, int(n), seed))
        w = u.clone()
        r = torch.zeros(sweeps, dtype=torch.float64, device="cuda")
        sc = torch.zeros(16, dtype=torch.float64, device="cuda")
        us.append(u); ws.append(w); rs.append(r); scs.append(sc)
        insts.append(gf.Instance.make({programs.J2_U: u, programs.J2_W: w, programs.J2_RES: r}, sc, ip=(int(n),)))
    return us, ws, rs, insts


@pytest.mark.parametrize("nwg", [0, 40, 300])
def test_batched_small_uneven_instances(gfx, oracle_lib, nwg):
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    sides = [3, 4, 5, 17, 64, 65, 100, 129, 200, 31, 9, 250]
    sweeps = 7
    us, ws, rs, insts = _batch(gf, programs, sides, sweeps)
    st = gfx.run(programs.jacobi2d(sweeps), insts, mode=gf.GF_EXEC_PERSISTENT,
                 launch=gf.Launch.make(num_wg=nwg) if nwg else None)
    gfx.sync()
    assert st["launches"] == 1 and st["num_wg"] >= len(sides)
    for i, n in enumerate(sides):
        g_ref, _, r_comp, _ = oracle_lib.jacobi2d(gi.batched_grid(i, n, 1), sweeps)
        g = host(us[i] if sweeps % 2 == 0 else ws[i])
        assert np.array_equal(g, g_ref), (i, n)
        r = host(rs[i])
        assert np.all(np.abs(r - r_comp) <= 1e-12 * r_comp + 1e-300), (i, n)


def test_batched_groups_laid_out_in_order(oracle_lib, monkeypatch):
    """GF_BATCH_ALIGN=0 (and a grid too small to split over the eight XCDs):
    groups laid out in order, whose members may sit on several XCDs, use the
    group barrier that writes each member's L2 back."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    sides, sweeps = [40, 71, 130, 9, 200], 6
    for env, nwg in (("0", 0), ("1", 7)):
        monkeypatch.setenv("GF_BATCH_ALIGN", env)
        with gf.Context(0) as ctx:
            us, ws, rs, insts = _batch(gf, programs, sides, sweeps, seed=2)
            ctx.run(programs.jacobi2d(sweeps), insts, mode=gf.GF_EXEC_PERSISTENT,
                    launch=gf.Launch.make(num_wg=nwg) if nwg else None)
            ctx.sync()
            for i, n in enumerate(sides):
                g_ref, _, r_comp, _ = oracle_lib.jacobi2d(gi.batched_grid(i, n, 2), sweeps)
                assert np.array_equal(host(us[i]), g_ref), (env, i, n)
                assert np.all(np.abs(host(rs[i]) - r_comp) <= 1e-12 * r_comp), (env, i, n)


def test_batched_placement_check_after_other_launches(gfx, oracle_lib):
    """Other launches first (odd grid sizes move the XCD that takes
    workgroup 0), then a batched launch whose groups are kept to one XCD:
    the placement check runs (a count, not -1) and the result equals the
    oracle."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    sides, sweeps = [40, 71, 130, 9, 200, 64, 33, 90, 17], 6
    for k, pre in enumerate((0, 3, 13)):
        for j in range(pre):
            run_jacobi2d(gfx, gi.batched_grid(j, 37 + 2 * j, 9), 2, gf.GF_EXEC_PERSISTENT,
                         launch=gf.Launch.make(num_wg=1 + 2 * j))
        us, ws, rs, insts = _batch(gf, programs, sides, sweeps, seed=3 + k)
        gfx.run(programs.jacobi2d(sweeps), insts, mode=gf.GF_EXEC_PERSISTENT, launch=gf.Launch.make(num_wg=64))
        gfx.sync()
        misplaced = gfx.batch_misplaced()
        print(f"placement check after {pre} launches: {misplaced} workgroups off their class's XCD", flush=True)
        assert misplaced >= 0
        for i, n in enumerate(sides):
            g_ref, _, r_comp, _ = oracle_lib.jacobi2d(gi.batched_grid(i, n, 3 + k), sweeps)
            assert np.array_equal(host(us[i]), g_ref), (pre, i, n)
            assert np.all(np.abs(host(rs[i]) - r_comp) <= 1e-12 * r_comp), (pre, i, n)


@pytest.mark.parametrize("mode", ["persistent", "per_region", "per_region_graph"])
def test_batched_shape_per_instance(gfx, oracle_lib, mode):
    """Every instance with its own rows per segment (shorter and longer than
    the register ring, longer than the grid) and its own share of the grid."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    sides = [3, 40, 71, 130, 9, 200, 257, 64, 1000, 33]
    segs = [1, 3, 7, 8, 2, 64, 13, 128, 32, 5000]
    weights = [0, 1, 5, 100, 0, 30, 2, 0, 1000, 7]
    sweeps = 5
    us, ws, rs, insts = _batch(gf, programs, sides, sweeps, seed=4)
    launches = [gf.Launch.make(wg_size=128, tile_y=sg, num_wg=wt) for sg, wt in zip(segs, weights)]
    m = {"persistent": gf.GF_EXEC_PERSISTENT, "per_region": gf.GF_EXEC_PER_REGION,
         "per_region_graph": gf.GF_EXEC_PER_REGION_GRAPH}[mode]
    st = gfx.run_batched(programs.jacobi2d(sweeps), insts, launches, mode=m)
    gfx.sync()
    if mode == "persistent":
        assert st["launches"] == 1
    for i, n in enumerate(sides):
        g_ref, _, r_comp, _ = oracle_lib.jacobi2d(gi.batched_grid(i, n, 4), sweeps)
        g = host(us[i] if sweeps % 2 == 0 else ws[i])
        assert np.array_equal(g, g_ref), (i, n)
        assert np.all(np.abs(host(rs[i]) - r_comp) <= 1e-12 * r_comp + 1e-300), (i, n)


def test_batched_tuner_plan_runs_and_matches_oracle(gfx, oracle_lib):
    """gf_tune_batched picks a shape per instance; a run with that plan
    equals the oracle on every instance (the tuner's own runs change the
    data, so the instances are reset first)."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    sides = [64, 70, 100, 130, 260, 300, 520, 700, 1100, 1500, 90, 2000]
    sweeps = 4
    us, ws, rs, insts = _batch(gf, programs, sides, sweeps, seed=5)
    prog = programs.jacobi2d(sweeps)
    launches, ms = gfx.tune_batched(prog, insts, reps=1)
    assert ms > 0 and len(launches) == len(sides)
    assert len({int(l.wg_size) for l in launches}) == 1 and all(int(l.tile_y) > 0 for l in launches)
    for i, n in enumerate(sides):
        us[i].copy_(dev(gi.batched_grid(i, n, 5)))
        ws[i].copy_(us[i])
    st = gfx.run_batched(prog, insts, launches)
    gfx.sync()
    assert st["launches"] == 1
    for i, n in enumerate(sides):
        g_ref, _, r_comp, _ = oracle_lib.jacobi2d(gi.batched_grid(i, n, 5), sweeps)
        assert np.array_equal(host(us[i]), g_ref), (i, n)
        assert np.all(np.abs(host(rs[i]) - r_comp) <= 1e-12 * r_comp), (i, n)


def test_batched_equals_single_instance_bitwise(gfx):
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    sides = [70, 300, 45, 1000, 129]
    sweeps = 6
    us, ws, rs, insts = _batch(gf, programs, sides, sweeps, seed=3)
    gfx.run(programs.jacobi2d(sweeps), insts, mode=gf.GF_EXEC_PERSISTENT)
    gfx.sync()
    for i, n in enumerate(sides):
        g1, r1, _ = run_jacobi2d(gfx, gi.batched_grid(i, n, 3), sweeps, gf.GF_EXEC_PERSISTENT)
        assert np.array_equal(host(us[i]), g1) and np.array_equal(host(rs[i]), r1)


_REF256 = {}


def _oracle_256(oracle_lib, sides, sweeps):
    """The oracle on every one of the 256 instances (serial C per instance,
    instances spread over host threads)."""
    from concurrent.futures import ThreadPoolExecutor
    key = (tuple(int(n) for n in sides), sweeps)
    if key not in _REF256:
        def one(i):
            g, _, r_comp, _ = oracle_lib.jacobi2d(gi.batched_grid(i, int(sides[i]), 1), sweeps)
            return g, r_comp
        with ThreadPoolExecutor(max_workers=8) as ex:
            _REF256.clear()
            _REF256[key] = list(ex.map(one, range(len(sides))))
    return _REF256[key]


@pytest.mark.parametrize("mode", ["persistent", "per_region"])
def test_batched_256_instances_config(gfx, oracle_lib, mode):
    """256 instances, sides floor(64 * 32^U) in [64, 2048], 50 sweeps with an
    L2 residual, in the measured launch shape (one launch in the persistent
    mode, a launch per region and instance otherwise). Every instance is
    compared with the oracle: grid bit-exact, residuals within 1e-12 of the
    compensated sum."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs, tuner
    sides = gi.batched_sides(256, seed=1)
    sweeps = 50
    print(f"batched 256 instances mode={mode}, sum n^2 = {int((sides.astype(np.int64) ** 2).sum())}", flush=True)
    us, ws, rs, insts = _batch(gf, programs, sides, sweeps)
    m = gf.GF_EXEC_PERSISTENT if mode == "persistent" else gf.GF_EXEC_PER_REGION
    per = tuner.lookup_batched("batched_256")
    if per is not None:
        st = gfx.run_batched(programs.jacobi2d(sweeps), insts, per, mode=m)
    else:
        st = gfx.run(programs.jacobi2d(sweeps), insts, mode=m, launch=tuner.lookup("batched_256"))
    gfx.sync()
    if mode == "persistent":
        assert st["launches"] == 1
    refs = _oracle_256(oracle_lib, sides, sweeps)
    for i in range(256):
        n = int(sides[i])
        g_ref, r_comp = refs[i]
        assert np.array_equal(host(us[i]), g_ref), (i, n)
        r = host(rs[i])
        assert np.all(np.abs(r - r_comp) <= 1e-12 * r_comp), (i, n)
        assert np.all(r > 0) and np.all(np.diff(r) <= 1e-12 * r[:-1])
