"""GPU parity of the balanced heap allocator (include/gf_heap.h, Section 3.4).

A script of malloc/free/find operations run by one device thread must return
exactly the offsets, sizes and watermarks of the sequential model
(oracle/heap.py). Concurrent use by many threads must never hand out
overlapping blocks: every thread fills its block, all blocks stay live, then
every thread checks its own. It must also leave every chunk empty after all
frees."""
import numpy as np
import pytest

from oracle.heap import BalancedHeap

pytestmark = pytest.mark.gpu


def _script(rng, n_ops, n_ids, n_teams, max_bytes):
    """Random operations on live allocations only (no double free)."""
    ops, live, mallocs = [], [], []
    for i in range(n_ops):
        r = rng.random()
        if r < 0.6 or not mallocs:
            ops.append((1, int(rng.integers(0, max_bytes + 1)),
                        int(rng.integers(0, n_ids)) | (int(rng.integers(0, n_teams)) << 32)))
            live.append(i)
            mallocs.append(i)
        elif r < 0.9 and live:
            j = live.pop(int(rng.integers(0, len(live))))
            ops.append((2, j, 0))
        else:
            j = mallocs[int(rng.integers(0, len(mallocs)))]
            ops.append((3, j, int(rng.integers(0, max_bytes + 48))))
    return ops


def _oracle_run(heap, ops):
    res, offs = [], []
    for op, a, b in ops:
        if op == 1:
            o = heap.malloc(b & 0xFFFFFFFF, b >> 32, a)
            offs.append(o)
            res.append((-1 if o is None else o, 0))
        elif op == 2:
            heap.free(res[a][0] if res[a][0] >= 0 else None)
            offs.append(None)
            res.append((0, 0))
        else:
            base = res[a][0]
            f = heap.find(base + b) if base >= 0 else None
            offs.append(None)
            res.append((-1, 0) if f is None else f)
    return res


@pytest.mark.parametrize("nbytes,N,M,ratio,seed", [(32 * 1024, 4, 2, 3, 1), (8 * 1024, 1, 1, 1, 2),
                                                   (64 * 1024, 8, 4, 5, 3), (48 * 1024, 3, 5, 2, 4)])
def test_heap_script_matches_the_model(nbytes, N, M, ratio, seed):
    import torch
    import paper_2306_11686_amd as gf
    print(f"heap script bytes={nbytes} N={N} M={M} ratio={ratio} seed={seed}", flush=True)
    rng = np.random.default_rng(seed)
    ops = _script(rng, 600, 2 * N + 1, 2 * M + 1, 700)
    want = _oracle_run(model := BalancedHeap(nbytes, N, M, ratio), ops)
    assert any(r[0] == -1 for (o, _, _), r in zip(ops, want) if o == 1), "the script should exhaust a chunk"
    with gf.Heap(0, nbytes, N, M, ratio) as h:
        d_ops = torch.tensor(np.array(ops, dtype=np.int64).reshape(-1), device="cuda")
        d_res = torch.full((2 * len(ops),), -7, dtype=torch.int64, device="cuda")
        h.script(d_ops, len(ops), d_res)
        got = d_res.cpu().numpy().reshape(-1, 2)
        assert [tuple(int(v) for v in r) for r in got] == [tuple(r) for r in want]
        assert h.tops() == model.tops()
        assert h.counts() == {"null": 0, "corrupt": 0, "timeouts": 0, "bad_frees": 0}


@pytest.mark.parametrize("teams,threads,nbytes,N,M", [(256, 256, 64, 32, 16), (37, 100, 200, 7, 3),
                                                       (64, 1024, 8, 32, 16), (16, 64, 24, 1, 1)])
def test_concurrent_blocks_never_overlap(teams, threads, nbytes, N, M):
    """All threads hold their blocks at once, then check them: overwritten
    words would show an overlap. Afterwards every chunk is empty."""
    import torch
    import paper_2306_11686_amd as gf
    print(f"heap hold/release teams={teams} threads={threads} bytes={nbytes} N={N} M={M}", flush=True)
    with gf.Heap(0, 1 << 26, N, M, 4) as h:
        ptrs = torch.zeros(teams * threads, dtype=torch.int64, device="cuda")
        h.bench(teams, threads, nbytes, gf.GF_HEAP_BENCH_HOLD, ptrs)
        torch.cuda.synchronize()
        p = ptrs.cpu().numpy()
        assert np.all(p != 0)
        assert np.unique(p).size == p.size
        h.bench(teams, threads, nbytes, gf.GF_HEAP_BENCH_RELEASE, ptrs)
        assert h.counts() == {"null": 0, "corrupt": 0, "timeouts": 0, "bad_frees": 0}
        assert h.tops() == [0] * (N * M)


@pytest.mark.parametrize("teams,threads,N,M", [(1, 1, 32, 16), (32, 64, 32, 16), (256, 256, 32, 16),
                                               (128, 32, 32, 16), (256, 256, 64, 32), (256, 1, 64, 32)])
def test_roundtrip_benchmark_shape(teams, threads, N, M):
    """The allocation benchmark's shape: allocate, use, free in one kernel.
    After every round each chunk's watermark is back at its start: a free
    that read a stale in-use mark below the top would leave it raised."""
    import paper_2306_11686_amd as gf
    print(f"heap roundtrip teams={teams} threads={threads} N={N} M={M}", flush=True)
    with gf.Heap(0, 1 << 26, N, M, 4) as h:
        for _ in range(10):
            h.bench(teams, threads, 128, gf.GF_HEAP_BENCH_ROUNDTRIP)
            assert h.tops() == [0] * (N * M)
        assert h.counts() == {"null": 0, "corrupt": 0, "timeouts": 0, "bad_frees": 0}


def test_one_chunk_shared_by_every_thread():
    """N = M = 1: every lane of every wavefront contends for one lock."""
    import paper_2306_11686_amd as gf
    print("heap single chunk", flush=True)
    with gf.Heap(0, 1 << 24, 1, 1, 1) as h:
        h.bench(64, 256, 32, gf.GF_HEAP_BENCH_ROUNDTRIP)
        assert h.counts() == {"null": 0, "corrupt": 0, "timeouts": 0, "bad_frees": 0}
        assert h.tops() == [0]


def test_full_heap_returns_null_and_recovers():
    import torch
    import paper_2306_11686_amd as gf
    print("heap exhaustion", flush=True)
    with gf.Heap(0, 32 * 1024, 4, 2, 1) as h:       # 8 chunks of 256 units (4 KiB)
        ptrs = torch.zeros(2 * 64, dtype=torch.int64, device="cuda")
        # each chunk serves 16 threads of one workgroup; 17 units each: 15 fit
        h.bench(2, 64, 256, gf.GF_HEAP_BENCH_HOLD, ptrs)
        c = h.counts(reset=True)
        assert c["null"] == 8 * (16 - 15) and c["corrupt"] == 0
        h.bench(2, 64, 256, gf.GF_HEAP_BENCH_RELEASE, ptrs)
        assert h.counts() == {"null": 0, "corrupt": 0, "timeouts": 0, "bad_frees": 0}
        assert h.tops() == [0] * 8


def test_vendor_device_malloc_roundtrip():
    import paper_2306_11686_amd as gf
    print("vendor device malloc", flush=True)
    with gf.Heap(0, 1 << 26, vendor=True) as h:
        h.bench(64, 64, 128, gf.GF_HEAP_BENCH_ROUNDTRIP)
        assert h.counts() == {"null": 0, "corrupt": 0, "timeouts": 0, "bad_frees": 0}


def test_heap_argument_errors():
    import torch
    import paper_2306_11686_amd as gf
    for kw in ({"nbytes": 8}, {"thread_slots": 0}, {"first_ratio": 0}, {"nbytes": 256, "thread_slots": 16}):
        with pytest.raises(gf.GfError):
            gf.Heap(0, **kw)
    with gf.Heap(0, 1 << 20, 2, 2, 2) as h:
        bad = torch.tensor([1, 16, 0, 2, 3, 0], dtype=torch.int64, device="cuda")   # frees a later operation
        res = torch.zeros(4, dtype=torch.int64, device="cuda")
        with pytest.raises(gf.GfError):
            h.script(bad, 2, res)
        with pytest.raises(gf.GfError):
            h.bench(1, 2048, 64)
        with pytest.raises(gf.GfError):
            h.bench(1, 64, 12)
    with gf.Heap(0, 1 << 20, vendor=True) as v:
        with pytest.raises(gf.GfError):
            v.tops()
