"""GPU parity of a `parallel` region with manual worksharing and barriers
across all workgroups (GF_R_PHASES, Section 3.3): both buffers bit-exact
against the serial oracle after every phase count, and the owner map equal
to the balanced block split over the global thread count."""
import numpy as np
import pytest

import gf_inputs as gi
from tests.gpu_helpers import dev, host, scalars

pytestmark = pytest.mark.gpu

MODES = ["persistent", "per_region", "graph", "split"]


def _mode(gf, name):
    return {"persistent": gf.GF_EXEC_PERSISTENT, "per_region": gf.GF_EXEC_PER_REGION,
            "graph": gf.GF_EXEC_PER_REGION_GRAPH, "split": gf.GF_EXEC_KERNEL_SPLIT}[name]


def _run_phases(ctx, gf, a0, n_phases, shift, mode, launch, owner=True):
    import torch
    from paper_2306_11686_amd import programs
    n = a0.size
    a = dev(a0 if n else np.zeros(1))
    b = torch.zeros_like(a)
    own = torch.full((max(1, n),), -1, dtype=torch.int32, device="cuda")
    sc = scalars()
    inst = gf.Instance.make({0: a, 1: b, 2: own}, sc, ip=(n,))
    stats = ctx.run(programs.phases(n_phases, shift, owner=owner), inst, mode=mode, launch=launch)
    ctx.sync()
    return host(a)[:n], host(b)[:n], host(own)[:n], stats


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,phases,shift,nwg,wg", [(1000, 3, 17, 3, 64), (100003, 5, 50001, 37, 256),
                                                   (5, 4, 3, 2, 128), (99991, 7, 1, 11, 192),
                                                   (4096, 2, 4095, 4, 64), (0, 3, 0, 2, 64),
                                                   (30011, 6, 15000, 255, 256), (777, 1, 400, 1, 64)])
def test_phases_parity(gfx, oracle_lib, mode, n, phases, shift, nwg, wg):
    import paper_2306_11686_amd as gf
    print(f"phases mode={mode} n={n} P={phases} s={shift} nwg={nwg} wg={wg}", flush=True)
    a0 = gi.um11(7, 21, np.arange(n, dtype=np.uint64)) if n else np.zeros(0)
    ga, gb, own, st = _run_phases(gfx, gf, a0, phases, shift, _mode(gf, mode),
                                  gf.Launch.make(wg_size=wg, num_wg=nwg))
    ra, rb = oracle_lib.phases(a0, phases, shift)
    assert np.array_equal(ga, ra)
    assert np.array_equal(gb, rb)
    T = st["num_wg"] * wg
    assert st["num_wg"] >= 1 and (mode != "persistent" or st["num_wg"] == nwg)
    assert np.array_equal(own, oracle_lib.static_owner(n, T))


def test_phases_without_owner_map_and_default_launch(gfx, oracle_lib):
    import paper_2306_11686_amd as gf
    a0 = gi.um11(8, 21, np.arange(65537, dtype=np.uint64))
    for mode in (gf.GF_EXEC_PERSISTENT, gf.GF_EXEC_PER_REGION):
        ga, gb, own, _ = _run_phases(gfx, gf, a0, 9, 12345, mode, None, owner=False)
        ra, rb = oracle_lib.phases(a0, 9, 12345)
        assert np.array_equal(ga, ra) and np.array_equal(gb, rb)
        assert np.all(own == -1)


@pytest.mark.parametrize("mode", ["persistent", "per_region"])
def test_phases_feed_the_next_region(gfx, oracle_lib, mode):
    """The region's end barrier publishes the last phase to the next region:
    a dot product of the result with itself on every workgroup."""
    import torch
    import paper_2306_11686_amd as gf
    n, P, s = 200_003, 4, 77_777
    a0 = gi.um11(9, 21, np.arange(n, dtype=np.uint64))
    a, b = dev(a0), torch.zeros(n, dtype=torch.float64, device="cuda")
    sc = scalars()
    pro = [gf.Step.make(gf.GF_R_PHASES, arr=(0, 1, -1), np=0, chunk=P, mask=s),
           gf.Step.make(gf.GF_S_SET, sc=(0,), c=0.0),
           gf.Step.make(gf.GF_R_DOT, arr=(0, 0), sc=(0,), red_op=gf.GF_OP_SUM, np=0)]
    gfx.run(gf.Program.make(pro, [], 0), gf.Instance.make({0: a, 1: b}, sc, ip=(n,)), mode=_mode(gf, mode),
            launch=gf.Launch.make(wg_size=256, num_wg=300))
    gfx.sync()
    ra, _ = oracle_lib.phases(a0, P, s)
    assert np.array_equal(host(a), ra)
    ref, mag = oracle_lib.dot_compensated(ra, ra)
    assert abs(host(sc)[0] - ref) <= 1e-12 * mag


def test_phases_batched_instances(gfx, oracle_lib):
    """Several instances in one persistent launch: each group's barrier and
    thread count are its own."""
    import torch
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    sizes = [17, 5000, 123457, 999]
    keep, insts, a0s = [], [], []
    for i, n in enumerate(sizes):
        a0 = gi.um11(10 + i, 21, np.arange(n, dtype=np.uint64))
        a, b = dev(a0), torch.zeros(n, dtype=torch.float64, device="cuda")
        own = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        sc = scalars()
        keep.append((a, b, own, sc))
        a0s.append(a0)
        insts.append(gf.Instance.make({0: a, 1: b, 2: own}, sc, ip=(n,)))
    gfx.run(programs.phases(5, 3), insts, mode=gf.GF_EXEC_PERSISTENT, launch=gf.Launch.make(wg_size=128, num_wg=64))
    gfx.sync()
    for (a, b, own, _), a0 in zip(keep, a0s):
        ra, rb = oracle_lib.phases(a0, 5, 3)
        assert np.array_equal(host(a), ra) and np.array_equal(host(b), rb)
        # the group's thread count is some number of whole 128-thread workgroups
        o = host(own)
        assert any(np.array_equal(o, oracle_lib.static_owner(o.size, g * 128)) for g in range(1, 65))


def test_phases_argument_errors(gfx):
    import torch
    import paper_2306_11686_amd as gf
    a = torch.zeros(10, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    sc = scalars()
    inst = gf.Instance.make({0: a, 1: b}, sc, ip=(10,))
    bad = [gf.Step.make(gf.GF_R_PHASES, arr=(0, 1, -1), np=0, chunk=0, mask=1),     # no phases
           gf.Step.make(gf.GF_R_PHASES, arr=(0, 0, -1), np=0, chunk=2, mask=1),     # one buffer twice
           gf.Step.make(gf.GF_R_PHASES, arr=(0, 1, -1), np=0, chunk=2, mask=10),    # shift not below n
           gf.Step.make(gf.GF_R_PHASES, arr=(0, 1, 3), np=0, chunk=2, mask=1),      # unbound owner slot
           gf.Step.make(gf.GF_R_PHASES, arr=(0, 1, -1), np=0, chunk=2, mask=1, red_op=gf.GF_OP_SUM)]
    for st in bad:
        with pytest.raises(gf.GfError):
            gfx.run(gf.Program.make([st], [], 0), inst)
    gfx.sync()
