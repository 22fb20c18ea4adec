"""GPU parity of the stencil programs against the serial oracle.

Grids are compared bit for bit (both sides evaluate the same parenthesised
expression without contraction). The 3D residual is a max and must match
exactly; the 2D residual is a sum whose order differs, so it must lie within
1e-12 (relative, all terms are >= 0) of the oracle's compensated value.
"""
import numpy as np
import pytest

import gf_inputs as gi
from tests.gpu_helpers import run_jacobi2d, run_jacobi3d

pytestmark = pytest.mark.gpu

MODES = ["persistent", "per_region", "graph", "split"]


def _mode(gf, name):
    return {"persistent": gf.GF_EXEC_PERSISTENT, "per_region": gf.GF_EXEC_PER_REGION,
            "graph": gf.GF_EXEC_PER_REGION_GRAPH, "split": gf.GF_EXEC_KERNEL_SPLIT}[name]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,sweeps", [(3, 2), (5, 3), (13, 4), (37, 5), (66, 3)])
def test_jacobi3d_small_odd_shapes(gfx, oracle_lib, mode, n, sweeps):
    import paper_2306_11686_amd as gf
    print(f"jacobi3d n={n} sweeps={sweeps} mode={mode}", flush=True)
    u0 = gi.grid3d(n, seed=1)
    g_ref, r_ref = oracle_lib.jacobi3d(u0, sweeps)
    g, r, _ = run_jacobi3d(gfx, u0, sweeps, _mode(gf, mode))
    assert np.array_equal(g, g_ref)
    assert np.array_equal(r, r_ref)


_TILINGS = [(1, 1, 64, 0), (2, 7, 128, 1), (4, 16, 192, 0), (8, 64, 256, 1), (16, 5, 256, 1), (8, 300, 64, 1)]


@pytest.mark.parametrize("n,ty,tz,wg,remap", [(n,) + t for n in (41, 64) for t in _TILINGS]
                         + [(300, 8, 300, 64, 1)])
@pytest.mark.parametrize("mode", ["persistent", "per_region"])
def test_jacobi3d_tilings(gfx, oracle_lib, n, ty, tz, wg, remap, mode):
    """Odd n runs the one-value-per-thread tile, even n the x-pair tile with
    lane shifts; n = 300 with 64-thread workgroups spans several row chunks
    per tile row."""
    import paper_2306_11686_amd as gf
    print(f"jacobi3d tiling n={n} ty={ty} tz={tz} wg={wg} remap={remap} mode={mode}", flush=True)
    u0 = gi.grid3d(n, seed=2)
    g_ref, r_ref = oracle_lib.jacobi3d(u0, 3)
    launch = gf.Launch.make(wg_size=wg, tile_y=ty, tile_z=tz, xcd_remap=remap)
    g, r, _ = run_jacobi3d(gfx, u0, 3, _mode(gf, mode), launch=launch)
    assert np.array_equal(g, g_ref)
    assert np.array_equal(r, r_ref)


@pytest.mark.parametrize("ty,tz", [(1, 3), (2, 9), (4, 1), (8, 40)])
@pytest.mark.parametrize("mode", ["persistent", "per_region"])
@pytest.mark.parametrize("n", [41, 64])
def test_jacobi3d_prefetch2(gfx, oracle_lib, ty, tz, mode, n):
    """Two planes requested ahead: segments shorter than, equal to and longer
    than the prefetch depth."""
    import paper_2306_11686_amd as gf
    print(f"jacobi3d prefetch2 n={n} ty={ty} tz={tz} mode={mode}", flush=True)
    u0 = gi.grid3d(n, seed=4)
    g_ref, r_ref = oracle_lib.jacobi3d(u0, 3)
    launch = gf.Launch.make(wg_size=64 if n == 41 else 256, tile_y=ty, tile_z=tz, prefetch=2)
    g, r, _ = run_jacobi3d(gfx, u0, 3, _mode(gf, mode), launch=launch)
    assert np.array_equal(g, g_ref)
    assert np.array_equal(r, r_ref)


def test_jacobi3d_persistent_small_grid_count(gfx, oracle_lib):
    import paper_2306_11686_amd as gf
    u0 = gi.grid3d(30, seed=3)
    g_ref, r_ref = oracle_lib.jacobi3d(u0, 6)
    for nwg in (1, 3, 8, 37):
        print(f"jacobi3d persistent num_wg={nwg}", flush=True)
        g, r, st = run_jacobi3d(gfx, u0, 6, gf.GF_EXEC_PERSISTENT, launch=gf.Launch.make(num_wg=nwg))
        assert st["num_wg"] == nwg and st["launches"] == 1
        assert np.array_equal(g, g_ref) and np.array_equal(r, r_ref)


def test_jacobi3d_eigenmode_and_determinism(gfx, oracle_lib):
    import paper_2306_11686_amd as gf
    n, k = 48, 10
    u0 = gi.eigenmode3d(n, 1, 2, 3)
    g_ref, r_ref = oracle_lib.jacobi3d(u0, k)
    g1, r1, _ = run_jacobi3d(gfx, u0, k, gf.GF_EXEC_PERSISTENT)
    g2, r2, _ = run_jacobi3d(gfx, u0, k, gf.GF_EXEC_PERSISTENT)
    g3, r3, _ = run_jacobi3d(gfx, u0, k, gf.GF_EXEC_PER_REGION)
    assert np.array_equal(g1, g_ref) and np.array_equal(g1, g2) and np.array_equal(g1, g3)
    assert np.array_equal(r1, r_ref) and np.array_equal(r1, r2) and np.array_equal(r1, r3)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,sweeps", [(3, 1), (4, 2), (9, 5), (130, 7), (257, 3)])
def test_jacobi2d_small_shapes(gfx, oracle_lib, mode, n, sweeps):
    import paper_2306_11686_amd as gf
    print(f"jacobi2d n={n} sweeps={sweeps} mode={mode}", flush=True)
    u0 = gi.grid2d(n, seed=1)
    g_ref, r_naive, r_comp, _ = oracle_lib.jacobi2d(u0, sweeps)
    g, r, _ = run_jacobi2d(gfx, u0, sweeps, _mode(gf, mode))
    assert np.array_equal(g, g_ref)
    assert np.all(np.abs(r - r_comp) <= 1e-12 * r_comp + 1e-300)


@pytest.mark.parametrize("n", [75, 76, 129, 300, 301])
@pytest.mark.parametrize("seg,wg", [(1, 64), (2, 64), (6, 64), (7, 128), (8, 64), (15, 192), (64, 256), (1000, 64)])
def test_jacobi2d_tilings(gfx, oracle_lib, n, seg, wg):
    """Row segments of every length against the ring of seven rows (shorter,
    equal, longer, ragged, longer than the grid), even n and odd n (rows on
    8-byte boundaries; the last column n-1 held alone by one thread, at
    n = 129 with 64-thread workgroups the only column of its chunk), one or
    several column chunks per row."""
    import paper_2306_11686_amd as gf
    print(f"jacobi2d tiling n={n} seg={seg} wg={wg}", flush=True)
    u0 = gi.grid2d(n, seed=4)
    g_ref, _, r_comp, _ = oracle_lib.jacobi2d(u0, 5)
    for mode in (gf.GF_EXEC_PERSISTENT, gf.GF_EXEC_PER_REGION):
        g, r, _ = run_jacobi2d(gfx, u0, 5, mode, launch=gf.Launch.make(tile_y=seg, wg_size=wg))
        assert np.array_equal(g, g_ref)
        assert np.all(np.abs(r - r_comp) <= 1e-12 * r_comp)


@pytest.mark.parametrize("mode", MODES)
def test_jacobi2d_256_with_printf_rpc(gfx, oracle_lib, mode):
    """The 2D program at its full size: 256^2, 100 sweeps, printf every 10
    sweeps forwarded to the host by RPC."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    print(f"jacobi2d 256 printf mode={mode}", flush=True)
    fmt = gfx.register_format(programs.JACOBI2D_FORMAT, "id")
    gfx.take_output()
    u0 = gi.grid2d(256, seed=1)
    g_ref, _, r_comp, text_ref = oracle_lib.jacobi2d(u0, 100, print_every=10)
    g, r, st = run_jacobi2d(gfx, u0, 100, _mode(gf, mode), fmt_id=fmt, print_every=10)
    text = gfx.take_output()
    assert np.array_equal(g, g_ref)
    assert np.all(np.abs(r - r_comp) <= 1e-12 * r_comp)
    lines = text.splitlines()
    assert len(lines) == 10
    # the text is the host's own formatting of the doubles the device sent
    assert lines == [programs.JACOBI2D_FORMAT.strip() % (s, r[s - 1]) for s in range(10, 101, 10)]
    ref_lines = text_ref.splitlines()
    for a, b in zip(lines, ref_lines):
        assert a.split()[1] == b.split()[1]
        assert abs(float(a.split()[3]) - float(b.split()[3])) <= 1e-9 * abs(float(b.split()[3]))


def test_jacobi2d_blocking_printf_with_server_thread(oracle_lib):
    import torch
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    with gf.Context(0, rpc_capture=True, rpc_thread=True, rpc_slots=8) as ctx:
        fmt = ctx.register_format(programs.JACOBI2D_FORMAT, "id")
        u0 = gi.grid2d(64, seed=2)
        _, r_naive, r_comp, _ = oracle_lib.jacobi2d(u0, 40, print_every=2)
        g, r, _ = run_jacobi2d(ctx, u0, 40, gf.GF_EXEC_PERSISTENT, fmt_id=fmt, print_every=2, blocking=True)
        text = ctx.take_output()
        assert len(text.splitlines()) == 20
        assert np.all(np.abs(r - r_comp) <= 1e-12 * r_comp)
        torch.cuda.synchronize()


def test_rpc_ring_wraps_with_server_thread():
    """More posted printf calls than ring slots: the device waits for freed
    slots while the library's server thread drains them, in FIFO order."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    with gf.Context(0, rpc_capture=True, rpc_thread=True, rpc_slots=8) as ctx:
        fmt = ctx.register_format(programs.JACOBI2D_FORMAT, "id")
        u0 = gi.grid2d(32, seed=3)
        _, r, _ = run_jacobi2d(ctx, u0, 50, gf.GF_EXEC_PER_REGION, fmt_id=fmt, print_every=1)
        lines = ctx.take_output().splitlines()
        assert [int(l.split()[1]) for l in lines] == list(range(1, 51))
        assert lines == [programs.JACOBI2D_FORMAT.strip() % (s, r[s - 1]) for s in range(1, 51)]


def test_rpc_blocking_without_server_times_out_cleanly():
    """A blocking RPC with nobody polling ends in the device watchdog and a
    GF_ETIMEOUT from gf_sync, not a hang."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    with gf.Context(0, rpc_capture=True, rpc_timeout_us=20000) as ctx:
        fmt = ctx.register_format(programs.JACOBI2D_FORMAT, "id")
        u0 = gi.grid2d(16, seed=1)
        prog = programs.jacobi2d(3, fmt_id=fmt, print_every=1, blocking=True)
        import torch
        u = torch.from_numpy(u0).cuda(); w = u.clone()
        res = torch.zeros(3, dtype=torch.float64, device="cuda")
        sc = torch.zeros(16, dtype=torch.float64, device="cuda")
        inst = gf.Instance.make({0: u, 1: w, 2: res}, sc, ip=(16,))
        ctx.run(prog, inst, mode=gf.GF_EXEC_PER_REGION)
        torch.cuda.synchronize()
        with pytest.raises(gf.GfError) as ei:
            ctx.sync()
        assert ei.value.status == gf.binding.GF_ETIMEOUT


@pytest.mark.parametrize("mode", ["persistent", "per_region"])
def test_rpc_ring_recovers_after_a_timeout(mode):
    """Posted printfs overrun an 8-slot ring that nobody drains: a client
    gives up waiting for a free slot (the 20 ms watchdog, forced from the
    host by polling nothing) and gf_sync reports GF_ETIMEOUT. gf_sync then
    re-synchronises the ring, so later runs on the same context (six posted
    printfs each, drained by gf_sync, wrapping the ring) print every line in
    order."""
    import torch
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    m = _mode(gf, mode)
    with gf.Context(0, rpc_capture=True, rpc_slots=8, rpc_timeout_us=20000) as ctx:
        fmt = ctx.register_format(programs.JACOBI2D_FORMAT, "id")
        u0 = gi.grid2d(24, seed=5)
        u = torch.from_numpy(u0).cuda(); w = u.clone()
        res = torch.zeros(20, dtype=torch.float64, device="cuda")
        sc = torch.zeros(16, dtype=torch.float64, device="cuda")
        inst = gf.Instance.make({0: u, 1: w, 2: res}, sc, ip=(24,))
        ctx.run(programs.jacobi2d(20, fmt_id=fmt, print_every=1), inst, mode=m)
        torch.cuda.synchronize()
        with pytest.raises(gf.GfError) as ei:
            ctx.sync()
        assert ei.value.status == gf.binding.GF_ETIMEOUT
        ctx.take_output()
        for rnd in range(3):
            _, r, _ = run_jacobi2d(ctx, u0, 6, m, fmt_id=fmt, print_every=1)
            lines = ctx.take_output().splitlines()
            assert lines == [programs.JACOBI2D_FORMAT.strip() % (k, r[k - 1]) for k in range(1, 7)], rnd


def _bench_launch(gf):
    import bench
    tuned = bench.load_tuned("jacobi3d_512") or {}
    return gf.Launch.make(wg_size=tuned.get("wg_size", 0), num_wg=tuned.get("num_wg", 0),
                          tile_y=tuned.get("tile_y", 0), tile_z=tuned.get("tile_z", 0),
                          xcd_remap=tuned.get("xcd_remap", 1), prefetch=tuned.get("prefetch", 0))


_REF512 = {}


@pytest.mark.parametrize("mode", MODES)
def test_jacobi3d_512_full_size_first_sweeps(gfx, oracle_lib, mode):
    """512^3 in the launch configuration the benchmark times, in every mode
    it times: the first two sweeps compared element by element with the
    oracle."""
    import paper_2306_11686_amd as gf
    print(f"jacobi3d 512 full mode={mode}", flush=True)
    u0 = gi.grid3d(512, seed=1)
    if not _REF512:
        _REF512["ref"] = oracle_lib.jacobi3d(u0, 2)
    g_ref, r_ref = _REF512["ref"]
    g, r, _ = run_jacobi3d(gfx, u0, 2, _mode(gf, mode), launch=_bench_launch(gf))
    assert np.array_equal(r, r_ref)
    assert np.array_equal(g, g_ref)


def test_jacobi3d_512_lockstep_after_200_sweeps(gfx, oracle_lib):
    """After the benchmark's 200 persistent sweeps, one more GPU sweep must
    equal one oracle sweep from the GPU's own state (grid bit-exact, max
    residual exact); the residual history must decay monotonically."""
    import torch
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    from tests.gpu_helpers import host, scalars
    print("jacobi3d 512 lockstep", flush=True)
    n = 512
    u0 = gi.grid3d(n, seed=1)
    u = torch.from_numpy(u0).cuda()
    w = u.clone()
    res = torch.zeros(200, dtype=torch.float64, device="cuda")
    sc = scalars()
    inst = gf.Instance.make({0: u, 1: w, 2: res}, sc, ip=(n,))
    gfx.run(programs.jacobi3d(200), inst, mode=gf.GF_EXEC_PERSISTENT, launch=_bench_launch(gf))
    gfx.sync()
    r200 = host(res)
    assert np.all(np.diff(r200) <= 0.0)
    state = host(u)
    del u0
    res1 = torch.zeros(1, dtype=torch.float64, device="cuda")
    inst1 = gf.Instance.make({0: u, 1: w, 2: res1}, sc, ip=(n,))
    gfx.run(programs.jacobi3d(1), inst1, mode=gf.GF_EXEC_PERSISTENT, launch=_bench_launch(gf))
    gfx.sync()
    g_gpu = host(w)
    g_ref, r_ref = oracle_lib.jacobi3d(state, 1)
    assert host(res1)[0] == r_ref[0]
    assert np.array_equal(g_gpu, g_ref)
