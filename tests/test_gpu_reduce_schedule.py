"""GPU parity of gf_reduce (reduction regions) and of the static worksharing
schedule with continuous global thread ids."""
import math

import numpy as np
import pytest

import gf_inputs as gi
from tests.gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 63, 64, 65, 1000, 4097, 1 << 20, (1 << 22) + 17]


def _reduce(ctx, op, dt, a):
    import torch
    import paper_2306_11686_amd as gf
    x = dev(a)
    out_dt = torch.float64 if dt == gf.GF_F64 else torch.int64
    out = torch.zeros(1, dtype=out_dt, device="cuda")
    ctx.reduce(op, dt, x, a.shape[0], out)
    v = host(out)[0]
    if dt in (gf.GF_U32, gf.GF_U64):
        v = int(np.uint64(np.int64(v)))
    return v


@pytest.mark.parametrize("n", SIZES)
def test_reduce_f64_sum_and_max(gfx, oracle_lib, n):
    import paper_2306_11686_amd as gf
    print(f"reduce f64 n={n}", flush=True)
    a = gi.um11(1, 11, np.arange(n, dtype=np.uint64))
    s = _reduce(gfx, gf.GF_OP_SUM, gf.GF_F64, a)
    ref = oracle_lib.reduce("sum", a, compensated=True)
    assert abs(s - ref) <= 1e-12 * float(np.sum(np.abs(a))) or (n == 0 and s == 0.0)
    m = _reduce(gfx, gf.GF_OP_MAX, gf.GF_F64, a)
    assert m == oracle_lib.reduce("max", a) if n else m == -math.inf
    # integer-valued doubles: exact in any order
    b = (np.arange(n) % 1024).astype(np.float64)
    assert _reduce(gfx, gf.GF_OP_SUM, gf.GF_F64, b) == oracle_lib.reduce("sum", b)


@pytest.mark.parametrize("n", SIZES)
def test_reduce_integers_exact(gfx, oracle_lib, n):
    import paper_2306_11686_amd as gf
    h = gi.hash_u64(2, 12, np.arange(n, dtype=np.uint64))
    u32 = (h >> np.uint64(32)).astype(np.uint32)
    assert _reduce(gfx, gf.GF_OP_SUM, gf.GF_U32, u32) == oracle_lib.reduce("sum", u32)
    assert _reduce(gfx, gf.GF_OP_MAX, gf.GF_U32, u32) == (oracle_lib.reduce("max", u32) if n else 0)
    assert _reduce(gfx, gf.GF_OP_SUM, gf.GF_U64, h) == oracle_lib.reduce("sum", h)
    assert _reduce(gfx, gf.GF_OP_MAX, gf.GF_U64, h) == (oracle_lib.reduce("max", h) if n else 0)
    i64 = h.view(np.int64)
    assert _reduce(gfx, gf.GF_OP_SUM, gf.GF_I64, i64) == oracle_lib.reduce("sum", i64)
    if n:
        assert _reduce(gfx, gf.GF_OP_MAX, gf.GF_I64, i64) == oracle_lib.reduce("max", i64)


def test_reduce_is_deterministic(gfx):
    import paper_2306_11686_amd as gf
    a = gi.um11(3, 11, np.arange(3 << 20, dtype=np.uint64))
    vals = {_reduce(gfx, gf.GF_OP_SUM, gf.GF_F64, a) for _ in range(4)}
    assert len(vals) == 1


@pytest.mark.parametrize("mode_name", ["persistent", "per_region"])
@pytest.mark.parametrize("n,chunk,nwg,wg", [(1000, 0, 3, 64), (100003, 0, 37, 256), (5, 0, 2, 128),
                                             (99991, 7, 11, 192), (4096, 1, 4, 64), (0, 0, 2, 64)])
def test_static_schedule_owner_map(gfx, oracle_lib, mode_name, n, chunk, nwg, wg):
    """Every iteration is executed by the thread the static-schedule formula
    names, with ids continuous across workgroups (bit-exact)."""
    import torch
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    mode = gf.GF_EXEC_PERSISTENT if mode_name == "persistent" else gf.GF_EXEC_PER_REGION
    owner = torch.full((max(1, n),), -1, dtype=torch.int32, device="cuda")
    sc = torch.zeros(16, dtype=torch.float64, device="cuda")
    inst = gf.Instance.make({0: owner}, sc, ip=(n,))
    gfx.run(programs.owner_map(chunk), inst, mode=mode, launch=gf.Launch.make(wg_size=wg, num_wg=nwg))
    gfx.sync()
    got = host(owner)[:n]
    ref = oracle_lib.static_owner(n, nwg * wg, chunk)
    assert np.array_equal(got, ref)


def test_copy_kernel(gfx):
    import torch
    a = torch.arange(1 << 20, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    gfx.copy(b, a, a.numel() * 8)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("num_wg", [4096, 1021])
def test_per_region_reduction_sees_every_workgroup(gfx, oracle_lib, num_wg):
    """One launch per region over thousands of workgroups on all XCDs: the
    workgroup that finishes last reads every other one's partial, which was
    stored at agent scope without an L2 write-back. Ten launches over fresh
    data, each checked against the oracle."""
    import torch
    import paper_2306_11686_amd as gf
    from tests.gpu_helpers import scalars
    print(f"per-region dot num_wg={num_wg}", flush=True)
    n = (1 << 22) + 5
    idx = np.arange(n, dtype=np.uint64)
    ta = torch.empty(n, dtype=torch.float64, device="cuda")
    tb = torch.empty(n, dtype=torch.float64, device="cuda")
    sc = scalars()
    prog = gf.Program.make([gf.Step.make(gf.GF_R_DOT, arr=(0, 1), sc=(1,), red_op=gf.GF_OP_SUM, np=0)], [], 0)
    inst = gf.Instance.make({0: ta, 1: tb}, sc, ip=(n,))
    for rep in range(10):
        a = gi.um11(40 + rep, 11, idx)
        b = gi.um11(80 + rep, 11, idx)
        ta.copy_(torch.from_numpy(a))
        tb.copy_(torch.from_numpy(b))
        sc.zero_()
        st = gfx.run(prog, inst, mode=gf.GF_EXEC_PER_REGION, launch=gf.Launch.make(items=1, num_wg=num_wg))
        gfx.sync()
        assert st["num_wg"] == num_wg
        d, s = oracle_lib.dot_compensated(a, b)
        got = host(sc)[1]
        assert abs(got - d) <= 1e-12 * s, (rep, got, d)


@pytest.mark.parametrize("num_wg", [1, 2, 3, 7, 8, 9, 17, 1000])
def test_per_region_finalize_counts_every_grid_size(gfx, oracle_lib, num_wg):
    """The finishing workgroup is found through eight sub-counters (workgroup
    b on counter b mod 8) and a top counter; grids smaller than eight or not
    a multiple of it leave sub-counters short or empty. Three launches in a
    row (the counters must be back at zero after each) of a dot whose glue
    divides two scalars: the glue runs exactly once per launch."""
    import torch
    import paper_2306_11686_amd as gf
    from tests.gpu_helpers import scalars
    print(f"per-region finalize num_wg={num_wg}", flush=True)
    n = 300007
    idx = np.arange(n, dtype=np.uint64)
    a = gi.um11(5, 11, idx)
    b = gi.um11(6, 11, idx)
    ta, tb = dev(a), dev(b)
    prog = gf.Program.make([
        gf.Step.make(gf.GF_R_DOT, arr=(0, 1), sc=(1,), red_op=gf.GF_OP_SUM, np=0),
        gf.Step.make(gf.GF_S_DIV, sc=(2, 3, 1)),
        gf.Step.make(gf.GF_S_SET, sc=(4,), c=7.0),
    ], [], 0)
    d, s = oracle_lib.dot_compensated(a, b)
    for rep in range(3):
        sc = scalars({3: 2.0 + rep})
        inst = gf.Instance.make({0: ta, 1: tb}, sc, ip=(n,))
        st = gfx.run(prog, inst, mode=gf.GF_EXEC_PER_REGION, launch=gf.Launch.make(items=1, num_wg=num_wg))
        gfx.sync()
        assert st["launches"] == 1 and st["num_wg"] == num_wg
        h = host(sc)
        assert abs(h[1] - d) <= 1e-12 * s
        assert h[2] == (2.0 + rep) / h[1] and h[4] == 7.0
