"""gf_reduce_noalloc (the reduction on a static device array, for callers
that cannot allocate) against gf_reduce on the same inputs: the same grid
and summation order, so the same result bits, on two calls in a row, the
second with a smaller input; and against the oracle (compensated sum within
the relative 1e-12 of sum |a_i|, exact integers and maxima)."""
import math

import numpy as np
import pytest

import gf_inputs as gi
from tests.gpu_helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2306_11686_amd as gf
    c = gf.Context(0)
    yield c
    c.close()


def _both(ctx, op, dt, a, stream=None):
    """(gf_reduce_noalloc, gf_reduce) of a; u64 results as Python ints."""
    import torch
    import paper_2306_11686_amd as gf
    x = dev(a)
    out_dt = torch.float64 if dt == gf.GF_F64 else torch.int64
    o1 = torch.full((1,), 7, dtype=out_dt, device="cuda")
    o2 = torch.full((1,), 7, dtype=out_dt, device="cuda")
    ctx.reduce_noalloc(op, dt, x, a.shape[0], o1, stream=stream)
    ctx.reduce(op, dt, x, a.shape[0], o2, stream=stream)
    if stream is not None:
        stream.synchronize()
    ctx.sync()
    v1, v2 = host(o1)[0], host(o2)[0]
    if dt in (gf.GF_U32, gf.GF_U64):
        v1, v2 = int(np.uint64(np.int64(v1))), int(np.uint64(np.int64(v2)))
    return v1, v2


def _bits(v):
    return np.float64(v).view(np.uint64) if isinstance(v, (float, np.floating)) else v


@pytest.mark.parametrize("sizes", [((1 << 22) + 17, 4097), ((1 << 20), 63), (100000, 0)])
def test_f64_matches_gf_reduce_and_oracle(ctx, oracle_lib, sizes):
    import paper_2306_11686_amd as gf
    for k, n in enumerate(sizes):
        print(f"noalloc f64 n={n} call={k}", flush=True)
        a = gi.um11(1, 21 + k, np.arange(n, dtype=np.uint64))
        s1, s2 = _both(ctx, gf.GF_OP_SUM, gf.GF_F64, a)
        assert _bits(s1) == _bits(s2)
        if n:
            ref = oracle_lib.reduce("sum", a, compensated=True)
            assert abs(s1 - ref) <= 1e-12 * float(np.sum(np.abs(a)))
        else:
            assert s1 == 0.0
        m1, m2 = _both(ctx, gf.GF_OP_MAX, gf.GF_F64, a)
        assert _bits(m1) == _bits(m2)
        assert m1 == (oracle_lib.reduce("max", a) if n else -math.inf)


@pytest.mark.parametrize("sizes", [((1 << 21) + 5, 1000)])
def test_integers_match_gf_reduce_and_oracle(ctx, oracle_lib, sizes):
    import paper_2306_11686_amd as gf
    for k, n in enumerate(sizes):
        print(f"noalloc int n={n} call={k}", flush=True)
        h = gi.hash_u64(3, 22 + k, np.arange(n, dtype=np.uint64))
        u32 = (h >> np.uint64(32)).astype(np.uint32)
        i64 = h.view(np.int64)
        for op, dt, a, name in ((gf.GF_OP_SUM, gf.GF_U32, u32, "sum"), (gf.GF_OP_MAX, gf.GF_U32, u32, "max"),
                                (gf.GF_OP_SUM, gf.GF_U64, h, "sum"), (gf.GF_OP_MAX, gf.GF_U64, h, "max"),
                                (gf.GF_OP_SUM, gf.GF_I64, i64, "sum"), (gf.GF_OP_MAX, gf.GF_I64, i64, "max")):
            v1, v2 = _both(ctx, op, dt, a)
            assert v1 == v2 == oracle_lib.reduce(name, a)


def test_on_a_side_stream_and_argument_errors(ctx, oracle_lib):
    import torch
    import paper_2306_11686_amd as gf
    s = torch.cuda.Stream()
    for n in (300000, 5):
        a = (np.arange(n) % 1024).astype(np.float64)  # integer-valued: exact in any order
        v1, v2 = _both(ctx, gf.GF_OP_SUM, gf.GF_F64, a, stream=s)
        assert v1 == v2 == oracle_lib.reduce("sum", a)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(gf.GfError):
        ctx.reduce_noalloc(7, gf.GF_F64, out, 1, out)
    with pytest.raises(gf.GfError):
        ctx.reduce_noalloc(gf.GF_OP_SUM, 9, out, 1, out)
    with pytest.raises(gf.GfError):
        ctx.reduce_noalloc(gf.GF_OP_SUM, gf.GF_F64, out, -1, out)
