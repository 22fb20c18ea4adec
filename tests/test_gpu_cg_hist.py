"""GPU parity of the legacy-loop mix: CG on the 27-point matrix (SpMV, dot and
axpy each a separate region) and the u32 histogram.

SpMV and axpy are elementwise-exact (same products, same order, no
contraction); dots are sums whose order differs, held to 1e-12 of the sum of
|terms| around the oracle's compensated value. CG trajectories are checked by
lock-step replay: one GPU iteration from a snapshot of the GPU's own state is
compared region by region with the oracle, the axpys bit-exact given the
GPU's alpha and beta. Histograms are bit-exact.
"""
import math

import numpy as np
import pytest

import gf_inputs as gi
from tests.gpu_helpers import dev, host, scalars

pytestmark = pytest.mark.gpu


def _mode(gf, name):
    return {"persistent": gf.GF_EXEC_PERSISTENT, "per_region": gf.GF_EXEC_PER_REGION,
            "graph": gf.GF_EXEC_PER_REGION_GRAPH, "split": gf.GF_EXEC_KERNEL_SPLIT}[name]


_MATS = {}


def _matrix(m):
    if m not in _MATS:
        _MATS[m] = gi.poisson27_csr(m)
    return _MATS[m]


def _cg_instance(gf, programs, m, b, x=None, r=None, p=None, rho_hist_len=1):
    import torch
    rowptr, col, val = _matrix(m)
    n = m ** 3
    t = {programs.CG_ROWPTR: dev(rowptr), programs.CG_COL: dev(col), programs.CG_VAL: dev(val),
         programs.CG_X: dev(np.zeros(n) if x is None else x), programs.CG_R: dev(b if r is None else r),
         programs.CG_P: dev(b if p is None else p), programs.CG_Q: torch.zeros(n, dtype=torch.float64, device="cuda"),
         programs.CG_RHO: torch.zeros(max(1, rho_hist_len), dtype=torch.float64, device="cuda")}
    sc = scalars()
    inst = gf.Instance.make(t, sc, ip=(n,))
    return inst, t, sc


@pytest.mark.parametrize("mode", ["persistent", "per_region"])
@pytest.mark.parametrize("m", [3, 5, 8, 13])
def test_spmv_region_bit_exact(gfx, oracle_lib, mode, m):
    import paper_2306_11686_amd as gf
    print(f"spmv m={m} mode={mode}", flush=True)
    rowptr, col, val = _matrix(m)
    n = m ** 3
    x = gi.cg_rhs(n, seed=7)
    y = np.zeros(n)
    prog = gf.Program.make([gf.Step.make(gf.GF_R_SPMV, arr=(0, 1, 2, 3, 4), np=0)], [], 0)
    ty = dev(y)
    inst = gf.Instance.make({0: dev(rowptr), 1: dev(col), 2: dev(val), 3: dev(x), 4: ty}, scalars(), ip=(n,))
    gfx.run(prog, inst, mode=_mode(gf, mode))
    gfx.sync()
    assert np.array_equal(host(ty), oracle_lib.spmv(rowptr, col, val, x))


def test_spmv_fallback_path_for_dense_rows(gfx, oracle_lib):
    """Rows too long for the LDS product tile take the one-thread-per-row
    path; both paths are bit-exact."""
    import paper_2306_11686_amd as gf
    rng = np.random.default_rng(5)
    n = 700
    lens = np.where(np.arange(n) % 97 == 0, 3000, rng.integers(0, 40, n))
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(lens)
    col = rng.integers(0, n, int(rowptr[-1])).astype(np.int32)
    val = rng.standard_normal(int(rowptr[-1]))
    x = rng.standard_normal(n)
    ty = dev(np.zeros(n))
    prog = gf.Program.make([gf.Step.make(gf.GF_R_SPMV, arr=(0, 1, 2, 3, 4), np=0)], [], 0)
    inst = gf.Instance.make({0: dev(rowptr), 1: dev(col), 2: dev(val), 3: dev(x), 4: ty}, scalars(), ip=(n,))
    for mode in (gf.GF_EXEC_PERSISTENT, gf.GF_EXEC_PER_REGION):
        gfx.run(prog, inst, mode=mode)
        gfx.sync()
        assert np.array_equal(host(ty), oracle_lib.spmv(rowptr, col, val, x))


@pytest.mark.parametrize("per_row", [29, 30, 31, 32])
def test_spmv_slices_around_the_lds_tile_size(gfx, oracle_lib, per_row):
    """32-row slices of 29..32 nonzeros per row: 928..1,024 products per
    slice, on both sides of the wavefront's 960 LDS product slots (LDS path
    below, row loop above); both are bit-exact."""
    import paper_2306_11686_amd as gf
    rng = np.random.default_rng(per_row)
    n = 64 * 37 + 5
    rowptr = np.arange(n + 1, dtype=np.int64) * per_row
    rowptr = rowptr.astype(np.int32)
    col = rng.integers(0, n, int(rowptr[-1])).astype(np.int32)
    val = rng.standard_normal(int(rowptr[-1]))
    x = rng.standard_normal(n)
    ty = dev(np.zeros(n))
    prog = gf.Program.make([gf.Step.make(gf.GF_R_SPMV, arr=(0, 1, 2, 3, 4), np=0)], [], 0)
    inst = gf.Instance.make({0: dev(rowptr), 1: dev(col), 2: dev(val), 3: dev(x), 4: ty}, scalars(), ip=(n,))
    for mode in (gf.GF_EXEC_PERSISTENT, gf.GF_EXEC_PER_REGION):
        gfx.run(prog, inst, mode=mode)
        gfx.sync()
        assert np.array_equal(host(ty), oracle_lib.spmv(rowptr, col, val, x)), mode


@pytest.mark.parametrize("n", [1, 257, 100003, 2097152])
@pytest.mark.parametrize("items", [1, 4, 16])
def test_dot_and_axpby_regions(gfx, oracle_lib, n, items):
    import paper_2306_11686_amd as gf
    a = gi.cg_rhs(n, seed=3)
    b = gi.cg_rhs(n, seed=4)
    ta, tb, tout = dev(a), dev(b), dev(np.zeros(n))
    sc = scalars({1: 0.0, 2: 0.8125})
    prog = gf.Program.make([
        gf.Step.make(gf.GF_R_DOT, arr=(0, 1), sc=(1,), red_op=gf.GF_OP_SUM, np=0),
        gf.Step.make(gf.GF_R_AXPBY, arr=(2, 0, 1), sc=(-1, 2), c=-1.0, np=0),
    ], [], 0)
    inst = gf.Instance.make({0: ta, 1: tb, 2: tout}, sc, ip=(n,))
    for mode in (gf.GF_EXEC_PERSISTENT, gf.GF_EXEC_PER_REGION):
        sc[1] = 0.0
        gfx.run(prog, inst, mode=mode, launch=gf.Launch.make(items=items))
        gfx.sync()
        d, s = oracle_lib.dot_compensated(a, b)
        assert abs(host(sc)[1] - d) <= 1e-12 * s
        assert np.array_equal(host(tout), oracle_lib.axpby(a, -0.8125, b))


@pytest.mark.parametrize("mode", ["persistent", "per_region", "graph", "split"])
@pytest.mark.parametrize("m,iters", [(3, 20), (6, 40), (11, 30)])
def test_cg_small_systems(gfx, oracle_lib, mode, m, iters):
    """Whole CG runs on small systems: the GPU rho history stays within the
    envelope set by the oracle's own naive-vs-compensated divergence."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    print(f"cg m={m} iters={iters} mode={mode}", flush=True)
    rowptr, col, val = _matrix(m)
    n = m ** 3
    b = gi.cg_rhs(n, seed=1)
    inst, t, sc = _cg_instance(gf, programs, m, b, rho_hist_len=iters)
    gfx.run(programs.cg(iters), inst, mode=_mode(gf, mode))
    gfx.sync()
    x_n, rh_n, _, _, k_n = oracle_lib.cg(rowptr, col, val, b, iters)
    x_c, rh_c, _, _, k_c = oracle_lib.cg(rowptr, col, val, b, iters, compensated=True)
    k = min(k_n, k_c)
    rh = host(t[programs.CG_RHO])[:k]
    rh_n, rh_c = rh_n[:k], rh_c[:k]
    # the envelope: the largest relative gap so far between two legitimate
    # summation orders (the oracle's naive and compensated dots), at least
    # the 1e-12 dot tolerance, times 4, relative to rho_k itself
    assert np.all(rh_c > 0)
    gap = np.maximum.accumulate(np.abs(rh_n - rh_c) / rh_c)
    env = 4.0 * np.maximum(gap, 1e-12) * rh_c
    assert np.all(np.abs(rh - rh_c) <= env), (np.abs(rh - rh_c) / rh_c, gap)
    xg = host(t[programs.CG_X])
    scale = max(1.0, float(np.max(np.abs(x_c))))
    assert np.max(np.abs(xg - x_c)) <= max(8 * np.max(np.abs(x_n - x_c)), 1e-11 * scale)


def test_cg_persistent_equals_per_region_bitwise(gfx):
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    m, iters = 9, 25
    b = gi.cg_rhs(m ** 3, seed=2)
    outs = []
    for mode in (gf.GF_EXEC_PERSISTENT, gf.GF_EXEC_PER_REGION):
        inst, t, sc = _cg_instance(gf, programs, m, b, rho_hist_len=iters)
        gfx.run(programs.cg(iters), inst, mode=mode)
        gfx.sync()
        outs.append((host(t[programs.CG_X]), host(t[programs.CG_RHO])))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("m,iters", [(9, 25), (64, 12)])
def test_cg_nowait_equals_every_barrier_bitwise(gfx, m, iters):
    """The two axpby loops marked nowait drop two of the six barriers per
    iteration in the persistent kernel. The results are the same bits as
    with every barrier kept (same schedule, same summation order), and the
    run reports two fewer barriers per iteration."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    print(f"cg nowait m={m} iters={iters}", flush=True)
    b = gi.cg_rhs(m ** 3, seed=3)
    outs, bars = [], []
    for nowait in (False, True):
        inst, t, sc = _cg_instance(gf, programs, m, b, rho_hist_len=iters)
        st = gfx.run(programs.cg(iters, nowait=nowait), inst, mode=gf.GF_EXEC_PERSISTENT)
        gfx.sync()
        outs.append([host(t[k]) for k in (programs.CG_X, programs.CG_R, programs.CG_P, programs.CG_RHO)])
        bars.append(st["barriers"])
    assert bars[0] - bars[1] == 2 * iters
    for a, c in zip(*outs):
        assert np.array_equal(a, c)


def test_cg_nowait_in_a_batched_launch(gfx):
    """Three CG instances of different sizes in one persistent launch (group
    barriers per instance): with the nowait axpbys the results are the same
    bits as with every barrier kept, and as each instance run alone."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    sides, iters = (5, 9, 13), 15
    print(f"cg batched nowait sides={sides}", flush=True)
    runs = []
    for nowait in (False, True):
        made = [_cg_instance(gf, programs, m, gi.cg_rhs(m ** 3, seed=10 + m), rho_hist_len=iters) for m in sides]
        gfx.run(programs.cg(iters, nowait=nowait), [i for i, _, _ in made], mode=gf.GF_EXEC_PERSISTENT)
        gfx.sync()
        runs.append([[host(t[k]) for k in (programs.CG_X, programs.CG_RHO)] for _, t, _ in made])
    for m, a, b in zip(sides, *runs):
        inst, t, _ = _cg_instance(gf, programs, m, gi.cg_rhs(m ** 3, seed=10 + m), rho_hist_len=iters)
        gfx.run(programs.cg(iters), inst, mode=gf.GF_EXEC_PERSISTENT)
        gfx.sync()
        alone = [host(t[k]) for k in (programs.CG_X, programs.CG_RHO)]
        for u, v, w in zip(a, b, alone):
            assert np.array_equal(u, v) and np.array_equal(v, w), m


def test_nowait_misuse_is_rejected(gfx):
    """nowait is refused where the barrier it drops is needed: after a
    reduction, on regions with barriers inside them, and before a host call
    that would copy in arrays other workgroups may still write."""
    import torch
    import paper_2306_11686_amd as gf
    from oracle import hostcall as hc
    S = gf.Step
    n = 1024
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    sc = scalars()
    inst = gf.Instance.make({0: a, 1: a, 2: a}, sc, ip=(n,))
    nw = gf.GF_STEP_NOWAIT
    axpby = S.make(gf.GF_R_AXPBY, arr=(2, 0, 1), sc=(-1, 2), c=1.0, np=0, flags=nw)
    bad = [
        [S.make(gf.GF_R_DOT, arr=(0, 1), sc=(1,), red_op=gf.GF_OP_SUM, np=0, flags=nw)],
        [S.make(gf.GF_R_HIST, arr=(0, 1), np=0, mask=255, flags=nw)],
        [S.make(gf.GF_R_PHASES, arr=(0, 1, -1), np=0, chunk=2, mask=1, flags=nw)],
        [S.make(gf.GF_R_AXPBY, arr=(2, 0, 1), sc=(-1, 2), c=1.0, np=0, flags=gf.GF_STEP_BLOCKING)],
    ]
    for steps in bad:
        with pytest.raises(gf.GfError) as ei:
            gfx.run(gf.Program.make(steps, [], 0), inst)
        assert ei.value.status == gf.binding.GF_EINVAL
    cid = gfx.register_call(gf.GF_CALLEE_FWRITE, [gf.CallArg.ref(0, 8, mode=gf.GF_REF_READ), gf.CallArg.const(8),
                                                  gf.CallArg.const(1), gf.CallArg.const(hc.STDOUT, "p")])
    call = S.make(gf.GF_S_CALL, fmt_id=cid, every=1)
    setv = S.make(gf.GF_S_SET, sc=(3,), c=1.0)
    plain = S.make(gf.GF_R_AXPBY, arr=(2, 0, 1), sc=(-1, 2), c=1.0, np=0)
    for pro, body, iters in (([axpby, setv, call], [], 0),       # directly after, past a serial step
                             ([], [call, axpby], 2),              # the body wraps around to the call
                             ([axpby], [setv, call, plain], 1)):  # the prologue runs into the body
        with pytest.raises(gf.GfError) as ei:
            gfx.run(gf.Program.make(pro, body, iters), inst)
        assert ei.value.status == gf.binding.GF_EINVAL
    # a region between them restores the barrier, and the last region's
    # nowait is accepted
    gfx.run(gf.Program.make([axpby, setv, plain, call, axpby], [], 0), inst)
    gfx.sync()


def _tuned(key):
    """The launch shape the measurements of this workload use (tuning
    database), or None for the library's defaults."""
    from paper_2306_11686_amd import tuner
    return tuner.lookup(key)


@pytest.mark.parametrize("mode,k", [("persistent", 1), ("persistent", 10), ("persistent", 100),
                                    ("persistent", 499), ("per_region", 1), ("per_region", 499),
                                    ("graph", 1), ("graph", 499)])
def test_cg_128_lockstep_replay(gfx, oracle_lib, mode, k):
    """128^3 (2,097,152 rows, 55,742,968 nonzeros), the measured size and
    launch shape: run k GPU iterations, snapshot (x, r, p, rho), run one more
    GPU iteration and replay it on the oracle region by region."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    print(f"cg 128 lockstep mode={mode} k={k}", flush=True)
    m = 128
    rowptr, col, val = _matrix(m)
    n = m ** 3
    assert col.size == 55742968
    b = gi.cg_rhs(n, seed=1)
    launch = _tuned("cg_128")
    inst, t, sc = _cg_instance(gf, programs, m, b, rho_hist_len=k + 1)
    gfx.run(programs.cg(k), inst, mode=_mode(gf, mode), launch=launch)
    gfx.sync()
    x0, r0, p0 = host(t[programs.CG_X]), host(t[programs.CG_R]), host(t[programs.CG_P])
    s0 = host(sc)
    rho0 = s0[programs.CG_S_RHO]
    gfx.run(programs.cg_iterations_only(1), inst, mode=_mode(gf, mode), launch=launch)
    gfx.sync()
    s1 = host(sc)
    q = host(t[programs.CG_Q])
    assert np.array_equal(q, oracle_lib.spmv(rowptr, col, val, p0))
    pq_ref, pq_abs = oracle_lib.dot_compensated(p0, q)
    assert abs(s1[programs.CG_S_PQ] - pq_ref) <= 1e-12 * pq_abs
    alpha = s1[programs.CG_S_ALPHA]
    assert alpha == rho0 / s1[programs.CG_S_PQ]
    x1 = host(t[programs.CG_X])
    r1 = host(t[programs.CG_R])
    assert np.array_equal(x1, oracle_lib.axpby(x0, alpha, p0))
    assert np.array_equal(r1, oracle_lib.axpby(r0, -alpha, q))
    rn_ref, rn_abs = oracle_lib.dot_compensated(r1, r1)
    assert abs(s1[programs.CG_S_RHO] - rn_ref) <= 1e-12 * rn_abs
    beta = s1[programs.CG_S_BETA]
    assert beta == s1[programs.CG_S_RHO] / rho0
    assert np.array_equal(host(t[programs.CG_P]), oracle_lib.axpby(r1, beta, p0))


def _envelope_golden():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cg128_envelope.txt")
    meta = {}
    rows = []
    with open(path) as f:
        for line in f:
            if line.startswith("# true_residual_"):
                k, v = line[2:].split()
                meta[k] = float(v)
            elif not line.startswith("#"):
                rows.append([float(v) for v in line.split()[1:]])
    a = np.array(rows)
    return a[:, 0], a[:, 1], meta


@pytest.mark.parametrize("mode", ["persistent", "per_region"])
def test_cg_128_end_to_end_envelope(gfx, oracle_lib, mode):
    """500 GPU iterations at 128^3 in the measured launch shape against the
    oracle's own sensitivity to summation order: the oracle ran once with
    naive and once with compensated dots (tests/golden/cg128_envelope.txt,
    written from the oracle alone). At every k the GPU's rho_k may differ
    from the compensated run's by at most 4x the largest relative gap
    between the two oracle runs so far (at least the 1e-12 dot tolerance);
    the final true residual ||b - A x|| / ||b|| must agree within 2x."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    print(f"cg 128 envelope mode={mode}", flush=True)
    rho_n, rho_c, meta = _envelope_golden()
    iters = rho_c.size
    assert iters == 500
    m = 128
    rowptr, col, val = _matrix(m)
    b = gi.cg_rhs(m ** 3, seed=1)
    inst, t, sc = _cg_instance(gf, programs, m, b, rho_hist_len=iters)
    gfx.run(programs.cg(iters), inst, mode=_mode(gf, mode), launch=_tuned("cg_128"))
    gfx.sync()
    rho_g = host(t[programs.CG_RHO])
    gap = np.maximum.accumulate(np.abs(rho_n - rho_c) / rho_c)
    env = 4.0 * np.maximum(gap, 1e-12)
    bad = np.nonzero(np.abs(rho_g - rho_c) > env * rho_c)[0]
    assert bad.size == 0, (bad[:5], rho_g[bad[:5]], rho_c[bad[:5]], env[bad[:5]])
    x = host(t[programs.CG_X])
    true_res = float(np.linalg.norm(b - oracle_lib.spmv(rowptr, col, val, x)) / np.linalg.norm(b))
    ref = meta["true_residual_compensated"]
    assert ref / 2 <= true_res <= 2 * ref, (true_res, ref)


# ----------------------------------------------------------------------------
# Histogram
# ----------------------------------------------------------------------------

def _hist_run(gfx, keys, nbins, mode, launch=None, init=None):
    import torch
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    tk = dev(keys) if keys.size else torch.zeros(4, dtype=torch.int32, device="cuda")
    bins = dev(np.zeros(nbins, dtype=np.uint32) if init is None else init)
    inst = gf.Instance.make({0: tk, 1: bins}, scalars(), ip=(keys.size,))
    gfx.run(programs.histogram(nbins), inst, mode=mode, launch=launch)
    gfx.sync()
    return host(bins)


@pytest.mark.parametrize("mode", ["persistent", "per_region", "graph", "split"])
@pytest.mark.parametrize("n,nbins", [(0, 65536), (1, 65536), (13, 256), (100003, 65536), (1 << 20, 1024),
                                      ((1 << 20) + 7, 65536), (3 << 18, 1 << 20), (1001, 1), (1001, 2), (5, 4)])
def test_hist_uniform_bit_exact(gfx, oracle_lib, mode, n, nbins):
    import paper_2306_11686_amd as gf
    print(f"hist n={n} nbins={nbins} mode={mode}", flush=True)
    keys = gi.hist_keys_uniform(n, seed=2)
    init = (np.arange(nbins) % 5).astype(np.uint32)
    got = _hist_run(gfx, keys, nbins, _mode(gf, mode), init=init)
    ref = oracle_lib.hist_u32(keys, nbins, bins=init.copy())
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("wg,items,nwg", [(64, 1, 2), (256, 2, 6), (1024, 4, 0), (512, 8, 64)])
def test_hist_launch_configs(gfx, oracle_lib, wg, items, nwg):
    import paper_2306_11686_amd as gf
    keys = gi.hist_keys_zipf(300007, seed=3)
    ref = oracle_lib.hist_u32(keys, 65536)
    for mode in (gf.GF_EXEC_PERSISTENT, gf.GF_EXEC_PER_REGION):
        got = _hist_run(gfx, keys, 65536, mode, launch=gf.Launch.make(wg_size=wg, items=items, num_wg=nwg))
        assert np.array_equal(got, ref)


def test_hist_invariants_on_gpu(gfx):
    import paper_2306_11686_amd as gf
    n = 1 << 22
    got = _hist_run(gfx, np.arange(n, dtype=np.uint32), 65536, gf.GF_EXEC_PERSISTENT)
    assert np.all(got == n // 65536)
    got = _hist_run(gfx, np.full(n, 0xABCD1234, dtype=np.uint32), 65536, gf.GF_EXEC_PERSISTENT)
    assert got[0x1234] == n and int(got.sum()) == n


_HIST_KEYS = {}


@pytest.mark.parametrize("mode", ["persistent", "per_region"])
@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_hist_full_size_2_28(gfx, oracle_lib, dist, mode):
    """2^28 keys into 65,536 bins (the measured size and launch shape),
    bit-exact."""
    import paper_2306_11686_amd as gf
    print(f"hist 2^28 {dist} mode={mode}", flush=True)
    n = 1 << 28
    if dist not in _HIST_KEYS:
        _HIST_KEYS.clear()
        keys = gi.hist_keys_uniform(n, seed=1) if dist == "uniform" else gi.hist_keys_zipf(n, seed=1)
        _HIST_KEYS[dist] = (keys, oracle_lib.hist_u32(keys, 65536))
    keys, ref = _HIST_KEYS[dist]
    got = _hist_run(gfx, keys, 65536, _mode(gf, mode), launch=_tuned("hist_2^28"))
    assert int(got.sum()) == n
    assert np.array_equal(got, ref)
