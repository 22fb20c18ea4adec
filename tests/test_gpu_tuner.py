"""GPU checks of the autotuner: candidate decoding per kernel family and that
the picked launch is the fastest of the timed ones and runs correctly."""
import math

import numpy as np
import pytest

import gf_inputs as gi
from tests.gpu_helpers import run_jacobi3d, scalars, dev

pytestmark = pytest.mark.gpu


def test_candidates_decode_per_family(gfx):
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    sc = scalars()
    u = dev(np.zeros((66, 66, 66)))
    inst = gf.Instance.make({0: u, 1: u, 2: sc}, sc, ip=(66,))
    c = gfx.tune_candidates(programs.jacobi3d(2), inst)
    assert len(c) == 32
    assert sorted({x.tile_y for x in c}) == [1, 2, 4, 8]
    assert sorted({x.tile_z for x in c}) == sorted({math.ceil(64 / k) for k in (2, 3, 4, 6)})
    keys = gf.Instance.make({0: u, 1: u}, sc, ip=(100,))
    h = gfx.tune_candidates(programs.histogram(65536), keys)
    assert sorted({x.wg_size for x in h}) == [256, 512, 768, 1024]


def test_tune_picks_fastest_and_result_is_correct(gfx, oracle_lib):
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    n = 130
    u0 = gi.grid3d(n, seed=1)
    u = dev(u0)
    w = u.clone()
    import torch
    res = torch.zeros(4, dtype=torch.float64, device="cuda")
    sc = scalars()
    inst = gf.Instance.make({0: u, 1: w, 2: res}, sc, ip=(n,))
    prog = programs.jacobi3d(4)
    ms, best = gfx.tune(prog, inst, mode=gf.GF_EXEC_PERSISTENT, reps=3)
    assert best >= 0 and ms[best] == min(m for m in ms if math.isfinite(m))
    assert sum(math.isfinite(m) for m in ms) >= 16
    cands = gfx.tune_candidates(prog, inst)
    g_ref, r_ref = oracle_lib.jacobi3d(u0, 4)
    g, r, _ = run_jacobi3d(gfx, u0, 4, gf.GF_EXEC_PERSISTENT, launch=cands[best])
    assert np.array_equal(g, g_ref) and np.array_equal(r, r_ref)
