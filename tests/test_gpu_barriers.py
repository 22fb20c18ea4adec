"""Both grid barriers — the XCD-aware one (the default: one L2 write-back
per XCD) and the tree barrier with per-workgroup publication
(GF_BARRIER=tree) — give results equal to the oracle's: grids bit-exact at
several grid sizes, persistent runs bit-identical to per-region runs for
programs with reductions (CG), exact histogram counts."""
import os

import numpy as np
import pytest

import gf_inputs as gi
from tests.gpu_helpers import run_jacobi2d, run_jacobi3d, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["xcd", "tree"])
def xctx(request):
    import paper_2306_11686_amd as gf
    old = os.environ.get("GF_BARRIER")
    os.environ["GF_BARRIER"] = request.param
    try:
        ctx = gf.Context(0, rpc_capture=True)
    finally:
        if old is None:
            del os.environ["GF_BARRIER"]
        else:
            os.environ["GF_BARRIER"] = old
    yield ctx
    ctx.close()


@pytest.mark.parametrize("nwg", [2, 7, 64, 255, 512])
def test_jacobi3d_barrier_grid_sizes(xctx, oracle_lib, nwg):
    import paper_2306_11686_amd as gf
    print(f"barrier jacobi3d n=66 sweeps=30 num_wg={nwg}", flush=True)
    u0 = gi.grid3d(66, seed=7)
    g_ref, r_ref = oracle_lib.jacobi3d(u0, 30)
    launch = gf.Launch.make(tile_y=1, tile_z=4, num_wg=nwg)
    g, r, st = run_jacobi3d(xctx, u0, 30, gf.GF_EXEC_PERSISTENT, launch=launch)
    assert st["num_wg"] == nwg
    assert np.array_equal(g, g_ref)
    assert np.array_equal(r, r_ref)


def test_jacobi2d_barrier_with_printf(xctx, oracle_lib):
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    print("barrier jacobi2d 256 printf", flush=True)
    fmt = xctx.register_format(programs.JACOBI2D_FORMAT, "id")
    u0 = gi.grid2d(256, seed=1)
    g_ref, _, r_comp, text = oracle_lib.jacobi2d(u0, 100, print_every=10)
    g, r, _ = run_jacobi2d(xctx, u0, 100, gf.GF_EXEC_PERSISTENT, fmt_id=fmt, print_every=10)
    out = xctx.take_output()
    assert np.array_equal(g, g_ref)
    assert np.all(np.abs(r - r_comp) <= 1e-12 * np.abs(r_comp))
    assert out.count("\n") == 10 and len(out.splitlines()) == len(text.splitlines())


def test_cg_barrier_matches_per_region(xctx):
    import torch
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import workloads
    print("barrier cg 24^3", flush=True)
    prog, inst, keep, reset = workloads.cg(24, 40)
    outs = []
    for mode in (gf.GF_EXEC_PER_REGION, gf.GF_EXEC_PERSISTENT):
        reset()
        xctx.run(prog, inst, mode=mode, launch=gf.Launch.make(num_wg=300) if mode else None)
        xctx.sync()
        outs.append([host(t).copy() for t in keep[3:8]])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_histogram_barrier_exact(xctx):
    import torch
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import workloads
    print("barrier histogram 2^22", flush=True)
    prog, inst, keep, reset = workloads.histogram(1 << 22, 65536, "zipf")
    keys = host(keep[0]).view(np.uint32)
    ref = np.bincount(keys & 0xFFFF, minlength=65536)
    reset()
    xctx.run(prog, inst, mode=gf.GF_EXEC_PERSISTENT)
    xctx.sync()
    assert np.array_equal(host(keep[1]).view(np.uint32).astype(np.int64), ref)


def test_barrier_stress_many_sweeps(xctx, oracle_lib):
    """40,000 barriers in one persistent launch with 1,024 work items over
    256 workgroups: every sweep reads planes other workgroups wrote in the
    previous one, so a barrier that let a workgroup through early would break
    bit-exactness against the serial oracle (the grid decays as
    cos(pi/33)^k and stays far from underflow)."""
    import paper_2306_11686_amd as gf
    n, sweeps = 34, 40000
    print(f"barrier stress jacobi3d n={n} sweeps={sweeps}", flush=True)
    u0 = gi.grid3d(n, seed=9)
    g_ref, r_ref = oracle_lib.jacobi3d(u0, sweeps)
    launch = gf.Launch.make(tile_y=1, tile_z=1, num_wg=256)
    g, r, st = run_jacobi3d(xctx, u0, sweeps, gf.GF_EXEC_PERSISTENT, launch=launch)
    assert st["num_wg"] == 256 and st["barriers"] == sweeps
    assert np.array_equal(r, r_ref)
    assert np.array_equal(g, g_ref)
