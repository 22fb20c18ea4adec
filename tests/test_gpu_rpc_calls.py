"""GPU parity of general host calls (GF_S_CALL, Section 3.2): value and
reference arguments, objects copied to the host and back by access mode,
landing pads chosen by argument types. Each test runs a small program on the
device and the same calls through the oracle (oracle/hostcall.py: the libc
call on host copies of the objects); objects, return values and the text
sent to stdout must agree byte for byte."""
import ctypes

import numpy as np
import pytest

from oracle import hostcall as hc
from tests.gpu_helpers import dev, host, scalars

pytestmark = pytest.mark.gpu

MODES = ["persistent", "per_region", "graph", "split"]


def _mode(gf, name):
    return {"persistent": gf.GF_EXEC_PERSISTENT, "per_region": gf.GF_EXEC_PER_REGION,
            "graph": gf.GF_EXEC_PER_REGION_GRAPH, "split": gf.GF_EXEC_KERNEL_SPLIT}[name]


def _cstr(s: bytes, size: int) -> np.ndarray:
    a = np.zeros(size, dtype=np.uint8)
    a[:len(s)] = np.frombuffer(s, dtype=np.uint8)
    return a


def _gf_args(gf, args):
    """Oracle argument descriptors -> gf.CallArg records."""
    out = []
    for a in args:
        if a[0] == "const":
            out.append(gf.CallArg.const(a[2], a[1]))
        elif a[0] == "scalar":
            out.append(gf.CallArg.scalar(a[2], a[1]))
        elif a[0] == "iter":
            out.append(gf.CallArg.iteration())
        else:
            _, slot, start, size, offset, mode = a
            m = {"r": gf.GF_REF_READ, "w": gf.GF_REF_WRITE, "rw": gf.GF_REF_READWRITE}[mode]
            out.append(gf.CallArg.ref(slot, size, start=start, offset=offset, mode=m))
    return out


@pytest.fixture(scope="module")
def cctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2306_11686_amd as gf
    ctx = gf.Context(0, rpc_capture=True, rpc_thread=True, rpc_slots=16)
    yield ctx
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_snprintf_into_a_device_buffer_every_iteration(cctx, mode):
    """A write-only object filled by snprintf from the iteration number and
    a scalar that changes every iteration; the return value goes to a scalar
    and is recorded."""
    import paper_2306_11686_amd as gf
    print(f"call snprintf mode={mode}", flush=True)
    iters = 6
    buf0 = np.full(256, 0x5A, dtype=np.uint8)
    fmt = _cstr(b"it %lld x %.17g", 32)
    args = [("ref", 0, 32, 64, 0, "w"), ("const", "i", 64), ("ref", 1, 0, 32, 0, "r"), ("iter",),
            ("scalar", "d", 3)]
    cid = cctx.register_call(gf.GF_CALLEE_SNPRINTF, _gf_args(gf, args))
    d_buf, d_fmt = dev(buf0), dev(fmt)
    import torch
    rec = torch.zeros(iters, dtype=torch.float64, device="cuda")
    sc = scalars()
    pro = [gf.Step.make(gf.GF_S_SET, sc=(3,), c=1.0), gf.Step.make(gf.GF_S_SET, sc=(4,), c=3.0)]
    body = [gf.Step.make(gf.GF_S_DIV, sc=(3, 3, 4)),
            gf.Step.make(gf.GF_S_CALL, fmt_id=cid, every=1, flags=gf.GF_STEP_BLOCKING, sc=(5,)),
            gf.Step.make(gf.GF_S_RECORD, arr=(2,), sc=(5,))]
    prog = gf.Program.make(pro, body, iters)
    inst = gf.Instance.make({0: d_buf, 1: d_fmt, 2: rec}, sc)
    cctx.run(prog, inst, mode=_mode(gf, mode))
    cctx.sync()

    buf, scal, rec_ref = buf0.copy(), np.zeros(16), np.zeros(iters)
    scal[3], scal[4] = 1.0, 3.0
    for it in range(iters):
        scal[3] = scal[3] / scal[4]
        ret, _ = hc.call("snprintf", args, {0: buf, 1: fmt.copy()}, scal, it)
        scal[5] = ret
        rec_ref[it] = ret
    assert np.array_equal(host(d_buf), buf)
    assert np.array_equal(host(d_fmt), fmt)
    assert np.array_equal(host(rec), rec_ref)
    assert host(sc)[5] == scal[5]


@pytest.mark.parametrize("mode", MODES)
def test_sscanf_writes_reach_every_workgroup(cctx, mode):
    """sscanf writes through two references (one element of a large array,
    one 8-byte field at an offset into a small object); the region after the
    call reads the large array on every workgroup."""
    import paper_2306_11686_amd as gf
    import torch
    print(f"call sscanf mode={mode}", flush=True)
    n, k = 1 << 17, 100_003
    text, fmt = _cstr(b"12345 6.25e-3", 32), _cstr(b"%lld %lf", 16)
    x0 = np.zeros(n)
    ints0 = np.arange(4, dtype=np.int64) + 7
    args = [("ref", 0, 0, 32, 0, "r"), ("ref", 1, 0, 16, 0, "r"), ("ref", 3, 0, 32, 16, "rw"),
            ("ref", 2, 8 * k, 8, 0, "w")]
    cid = cctx.register_call(gf.GF_CALLEE_SSCANF, _gf_args(gf, args))
    d_x, d_ints = dev(x0), dev(ints0)
    ones = torch.ones(n, dtype=torch.float64, device="cuda")
    sc = scalars()
    pro = [gf.Step.make(gf.GF_S_CALL, fmt_id=cid, every=1, flags=gf.GF_STEP_BLOCKING, sc=(1,)),
           gf.Step.make(gf.GF_R_DOT, arr=(2, 4), sc=(0,), red_op=gf.GF_OP_SUM, np=0)]
    prog = gf.Program.make(pro, [], 0)
    d_text, d_fmt = dev(text), dev(fmt)      # kept alive until the run has completed
    inst = gf.Instance.make({0: d_text, 1: d_fmt, 2: d_x, 3: d_ints, 4: ones}, sc, ip=(n,))
    cctx.run(prog, inst, mode=_mode(gf, mode), launch=gf.Launch.make(num_wg=200, wg_size=256, items=1))
    cctx.sync()

    x, ints = x0.copy(), ints0.copy()
    ret, _ = hc.call("sscanf", args, {0: text, 1: fmt, 2: x, 3: ints})
    assert ret == 2 and ints[2] == 12345 and x[k] == 6.25e-3
    assert np.array_equal(host(d_x), x)
    assert np.array_equal(host(d_ints), ints)
    s = host(sc)
    assert s[1] == ret
    assert s[0] == 6.25e-3


@pytest.mark.parametrize("mode", MODES)
def test_fprintf_of_a_read_write_buffer_and_posted_fwrite(cctx, mode):
    """The paper's RPC benchmark call shape: fprintf with the format and a
    128-byte buffer passed by reference (read-write, since the callee's use
    is unknown), then a posted fwrite of part of the buffer. The buffer,
    including bytes after its string, comes back unchanged."""
    import paper_2306_11686_amd as gf
    print(f"call fprintf/fwrite mode={mode}", flush=True)
    rng = np.random.default_rng(5)
    buf = rng.integers(1, 256, 128, dtype=np.uint8)
    buf[:13] = np.frombuffer(b"device text\n\0", dtype=np.uint8)
    fmt = _cstr(b"buffer: %s (call %lld)\n", 48)
    a_pr = [("const", "p", hc.STDOUT), ("ref", 1, 0, 48, 0, "r"), ("ref", 0, 0, 128, 0, "rw"), ("iter",)]
    a_wr = [("ref", 0, 0, 16, 0, "r"), ("const", "i", 1), ("const", "i", 12), ("const", "p", hc.STDOUT)]
    c_pr = cctx.register_call(gf.GF_CALLEE_FPRINTF, _gf_args(gf, a_pr))
    c_wr = cctx.register_call(gf.GF_CALLEE_FWRITE, _gf_args(gf, a_wr))
    d_buf, d_fmt = dev(buf), dev(fmt)
    sc = scalars()
    body = [gf.Step.make(gf.GF_S_CALL, fmt_id=c_pr, every=1, flags=gf.GF_STEP_BLOCKING, sc=(2,)),
            gf.Step.make(gf.GF_S_CALL, fmt_id=c_wr, every=2)]
    prog = gf.Program.make([], body, 5)
    cctx.take_output()
    cctx.run(prog, gf.Instance.make({0: d_buf, 1: d_fmt}, sc), mode=_mode(gf, mode))
    cctx.sync()
    text = cctx.take_output().encode()

    want, arrays = b"", {0: buf.copy(), 1: fmt}
    for it in range(5):
        ret, out = hc.call("fprintf", a_pr, arrays, None, it)
        want += out
        if (it + 1) % 2 == 0:
            want += hc.call("fwrite", a_wr, arrays, None, it)[1]
    assert text == want
    assert np.array_equal(host(d_buf), buf)
    assert host(sc)[2] == ret


@pytest.mark.parametrize("mode", ["persistent", "per_region", "split"])
def test_unaligned_objects(cctx, mode):
    """Objects that start or end off a 16-byte boundary are copied byte by
    byte: a read-write object keeps the bytes the callee does not write, a
    write-only one comes back zero-filled."""
    import paper_2306_11686_amd as gf
    print(f"call unaligned mode={mode}", flush=True)
    area = np.full(100, 0xEE, dtype=np.uint8)
    fmt = _cstr(b"[%lld:%.3e]", 16)
    a1 = [("ref", 0, 3, 37, 5, "rw"), ("const", "i", 20), ("ref", 1, 0, 16, 0, "r"), ("iter",), ("scalar", "d", 2)]
    a2 = [("ref", 0, 45, 19, 0, "w"), ("const", "i", 19), ("ref", 1, 0, 16, 0, "r"), ("const", "i", -9),
          ("const", "d", 0.5)]
    c1 = cctx.register_call(gf.GF_CALLEE_SNPRINTF, _gf_args(gf, a1))
    c2 = cctx.register_call(gf.GF_CALLEE_SNPRINTF, _gf_args(gf, a2))
    d_area, d_fmt = dev(area), dev(fmt)
    sc = scalars({2: -1234.5})
    body = [gf.Step.make(gf.GF_S_CALL, fmt_id=c1, every=1, flags=gf.GF_STEP_BLOCKING),
            gf.Step.make(gf.GF_S_CALL, fmt_id=c2, every=3, flags=gf.GF_STEP_BLOCKING)]
    cctx.run(gf.Program.make([], body, 4), gf.Instance.make({0: d_area, 1: d_fmt}, sc), mode=_mode(gf, mode))
    cctx.sync()
    want, scal = area.copy(), np.zeros(16)
    scal[2] = -1234.5
    for it in range(4):
        hc.call("snprintf", a1, {0: want, 1: fmt}, scal, it)
        if (it + 1) % 3 == 0:
            hc.call("snprintf", a2, {0: want, 1: fmt}, scal, it)
    assert np.array_equal(host(d_area), want)


def test_fread_reads_successive_chunks_of_a_host_file(cctx, tmp_path):
    """fread into a write-only device object: the host file position moves
    on between iterations, as in the serial program."""
    import paper_2306_11686_amd as gf
    import torch
    print("call fread", flush=True)
    data = bytes((7 * i + 3) % 256 for i in range(200))
    path = tmp_path / "chunks.bin"
    path.write_bytes(data)
    libc = ctypes.CDLL(None)
    libc.fopen.restype = ctypes.c_void_p
    f_dev, f_ref = libc.fopen(str(path).encode(), b"rb"), libc.fopen(str(path).encode(), b"rb")
    assert f_dev and f_ref
    try:
        args = [("ref", 0, 0, 48, 0, "w"), ("const", "i", 1), ("const", "i", 48), ("const", "p", f_dev)]
        cid = cctx.register_call(gf.GF_CALLEE_FREAD, _gf_args(gf, args))
        d_obj = dev(np.full(48, 1, dtype=np.uint8))
        rec = torch.zeros(5, dtype=torch.float64, device="cuda")
        sc = scalars()
        body = [gf.Step.make(gf.GF_S_CALL, fmt_id=cid, every=1, flags=gf.GF_STEP_BLOCKING, sc=(0,)),
                gf.Step.make(gf.GF_S_RECORD, arr=(1,), sc=(0,))]
        cctx.run(gf.Program.make([], body, 5), gf.Instance.make({0: d_obj, 1: rec}, sc), mode=gf.GF_EXEC_PERSISTENT)
        cctx.sync()
        obj, rets = np.full(48, 1, dtype=np.uint8), []
        args_ref = args[:3] + [("const", "p", f_ref)]
        for it in range(5):
            rets.append(hc.call("fread", args_ref, {0: obj}, None, it)[0])
    finally:
        libc.fclose(ctypes.c_void_p(f_dev))
        libc.fclose(ctypes.c_void_p(f_ref))
    assert rets == [48, 48, 48, 48, 8]
    assert host(rec).tolist() == [float(r) for r in rets]
    assert np.array_equal(host(d_obj), obj)


@pytest.mark.parametrize("mode", ["persistent", "per_region"])
def test_many_instances_share_a_small_ring(mode):
    """24 instances make blocking calls that copy objects back through a
    ring of 8 slots: a slot is reused only after its caller has finished
    copying its payload back."""
    import paper_2306_11686_amd as gf
    import torch
    print(f"call ring reuse mode={mode}", flush=True)
    n_inst, iters = 24, 10
    fmt = _cstr(b"inst %.1f it %lld %s", 32)
    args = [("ref", 0, 0, 96, 0, "rw"), ("const", "i", 96), ("ref", 1, 0, 32, 0, "r"), ("scalar", "d", 0),
            ("iter",), ("ref", 2, 0, 64, 0, "r")]
    with gf.Context(0, rpc_capture=True, rpc_thread=True, rpc_slots=8) as ctx:
        cid = ctx.register_call(gf.GF_CALLEE_SNPRINTF, _gf_args(gf, args))
        body = [gf.Step.make(gf.GF_S_CALL, fmt_id=cid, every=1, flags=gf.GF_STEP_BLOCKING, sc=(1,)),
                gf.Step.make(gf.GF_S_RECORD, arr=(3,), sc=(1,))]
        prog = gf.Program.make([], body, iters)
        d_fmt = dev(fmt)
        bufs, tags, d_tags, recs, scs, insts = [], [], [], [], [], []
        for i in range(n_inst):
            tag = _cstr(b"x" * (i % 50) + b"#", 64)
            tags.append(tag)
            d_tags.append(dev(tag))
            bufs.append(dev(np.full(96, i, dtype=np.uint8)))
            recs.append(torch.zeros(iters, dtype=torch.float64, device="cuda"))
            scs.append(scalars({0: float(i)}))
            insts.append(gf.Instance.make({0: bufs[i], 1: d_fmt, 2: d_tags[i], 3: recs[i]}, scs[i]))
        ctx.run(prog, insts, mode=_mode(gf, mode))
        ctx.sync()
        for i in range(n_inst):
            buf, scal, rets = np.full(96, i, dtype=np.uint8), np.zeros(16), []
            scal[0] = float(i)
            for it in range(iters):
                rets.append(hc.call("snprintf", args, {0: buf, 1: fmt, 2: tags[i]}, scal, it)[0])
            assert np.array_equal(host(bufs[i]), buf), i
            assert host(recs[i]).tolist() == [float(r) for r in rets], i


def test_posted_calls_wrap_the_ring_in_order(cctx):
    """Posted calls with read-only objects: more calls than slots, text in
    ticket order."""
    import paper_2306_11686_amd as gf
    print("call posted ring wrap", flush=True)
    fmt = _cstr(b"%lld:%s\n", 16)
    word = _cstr(b"abc", 16)
    args = [("const", "p", hc.STDERR), ("ref", 0, 0, 16, 0, "r"), ("iter",), ("ref", 1, 0, 16, 0, "r")]
    cid = cctx.register_call(gf.GF_CALLEE_FPRINTF, _gf_args(gf, args))
    body = [gf.Step.make(gf.GF_S_CALL, fmt_id=cid, every=1)]
    cctx.take_output()
    d_fmt, d_word, sc = dev(fmt), dev(word), scalars()
    cctx.run(gf.Program.make([], body, 40), gf.Instance.make({0: d_fmt, 1: d_word}, sc),
             mode=gf.GF_EXEC_PERSISTENT)
    cctx.sync()
    assert cctx.take_output() == "".join(f"{i}:abc\n" for i in range(1, 41))


def test_call_stage_times_are_collected(cctx):
    import paper_2306_11686_amd as gf
    print("call stats", flush=True)
    buf = _cstr(b"stats", 128)
    fmt = _cstr(b"%s\n", 8)
    args = [("const", "p", hc.STDOUT), ("ref", 1, 0, 8, 0, "r"), ("ref", 0, 0, 128, 0, "rw")]
    cid = cctx.register_call(gf.GF_CALLEE_FPRINTF, _gf_args(gf, args))
    body = [gf.Step.make(gf.GF_S_CALL, fmt_id=cid, every=1, flags=gf.GF_STEP_BLOCKING | gf.GF_STEP_TIMED)]
    d_buf, d_fmt, sc = dev(buf), dev(fmt), scalars()
    cctx.run(gf.Program.make([], body, 50), gf.Instance.make({0: d_buf, 1: d_fmt}, sc),
             mode=gf.GF_EXEC_PERSISTENT)
    cctx.sync()
    assert cctx.take_output() == "stats\n" * 50
    st = cctx.call_stats(cid, reset=True)
    assert st["calls"] == 50
    for key in ("dev_args_us", "dev_copy_in_us", "dev_copy_out_us", "host_decode_us", "host_reply_us"):
        assert st[key] >= 0.0, key
    assert st["dev_wait_us"] > 0.0 and st["host_call_us"] > 0.0
    assert st["dev_wait_us"] > st["host_call_us"]
    assert cctx.call_stats(cid)["calls"] == 0


def test_call_site_and_step_errors(cctx):
    """Argument errors are reported before anything is enqueued."""
    import paper_2306_11686_amd as gf
    A = gf.CallArg
    with pytest.raises(gf.GfError) as ei:     # fprintf needs (FILE *, format) first
        cctx.register_call(gf.GF_CALLEE_FPRINTF, [A.const(1, "i"), A.ref(0, 8, mode=gf.GF_REF_READ)])
    assert ei.value.status == gf.binding.GF_EUNSUPPORTED
    with pytest.raises(gf.GfError):           # five references
        cctx.register_call(gf.GF_CALLEE_SSCANF, [A.ref(0, 8, mode=gf.GF_REF_READ)] * 2 +
                           [A.ref(1, 8, mode=gf.GF_REF_WRITE)] * 3)
    with pytest.raises(gf.GfError):           # objects larger than the slot payload (1024 bytes)
        cctx.register_call(gf.GF_CALLEE_FWRITE, [A.ref(0, 2048, mode=gf.GF_REF_READ), A.const(1), A.const(1),
                                                 A.const(hc.STDOUT, "p")])
    with pytest.raises(gf.GfError):           # offset beyond the object
        cctx.register_call(gf.GF_CALLEE_FWRITE, [A.ref(0, 8, offset=9, mode=gf.GF_REF_READ), A.const(1),
                                                 A.const(1), A.const(hc.STDOUT, "p")])
    with pytest.raises(gf.GfError):           # a scalar cannot pass as a pointer
        cctx.register_call(gf.GF_CALLEE_FPRINTF, [A.const(hc.STDOUT, "p"), A.ref(0, 8, mode=gf.GF_REF_READ),
                                                  A.scalar(0, "p")])
    cid = cctx.register_call(gf.GF_CALLEE_SNPRINTF, [A.ref(0, 16, mode=gf.GF_REF_WRITE), A.const(16),
                                                     A.ref(1, 8, mode=gf.GF_REF_READ)])
    sc = scalars()
    d0, d1 = dev(np.zeros(16, np.uint8)), dev(_cstr(b"x", 8))
    inst = gf.Instance.make({0: d0, 1: d1}, sc)
    with pytest.raises(gf.GfError) as ei:     # copies back, so it must be blocking
        cctx.run(gf.Program.make([], [gf.Step.make(gf.GF_S_CALL, fmt_id=cid, every=1)], 1), inst)
    assert ei.value.status == gf.binding.GF_EINVAL
    with pytest.raises(gf.GfError):           # unregistered call site
        cctx.run(gf.Program.make([], [gf.Step.make(gf.GF_S_CALL, fmt_id=999, every=1,
                                                   flags=gf.GF_STEP_BLOCKING)], 1), inst)
    with pytest.raises(gf.GfError):           # the referenced array slot is empty
        cctx.run(gf.Program.make([], [gf.Step.make(gf.GF_S_CALL, fmt_id=cid, every=1,
                                                   flags=gf.GF_STEP_BLOCKING)], 1),
                 gf.Instance.make({0: d0}, sc))
    cctx.sync()


@pytest.mark.parametrize("mode", MODES)
def test_heap_references_are_found_at_call_time(mode):
    """Pointers held in an array and not known when the call site is
    registered: the context's heap finds the live object behind each one and
    the whole object travels (read-write, write-only, read-only). Pointers
    it does not hold travel as values."""
    import torch
    import paper_2306_11686_amd as gf
    from oracle.heap import BalancedHeap
    print(f"call heap references mode={mode}", flush=True)
    with gf.Context(0, rpc_capture=True, rpc_thread=True) as ctx, gf.Heap(0, 65536, 1, 1, 1) as heap:
        ctx.set_heap(heap)
        model = BalancedHeap(65536, 1, 1, 1)
        ops = torch.tensor([1, 40, 0, 1, 20, 0], dtype=torch.int64, device="cuda")
        res = torch.zeros(4, dtype=torch.int64, device="cuda")
        heap.script(ops, 2, res)
        a, b = (int(v) for v in res.cpu().numpy()[::2])
        assert (a, b) == (model.malloc(0, 0, 40), model.malloc(0, 0, 20))
        base = heap.base()
        ptrs = dev(np.array([base + a + 10, base + b, base + 4000, 0x1234], dtype=np.int64))
        fmt1, fmt2, fmt3 = _cstr(b"<%lld>", 8), _cstr(b"%p|", 8), _cstr(b"\n", 8)
        d1, d2, d3 = dev(fmt1), dev(fmt2), dev(fmt3)
        A = gf.CallArg
        out = gf.host_stream("stdout")
        calls = [
            (gf.GF_CALLEE_SNPRINTF, [A.heapref(0, 0, 64, gf.GF_REF_READWRITE), A.const(8),
                                     A.ref(1, 8, mode=gf.GF_REF_READ), A.iteration()]),
            (gf.GF_CALLEE_SNPRINTF, [A.heapref(0, 1, 64, gf.GF_REF_WRITE), A.const(32),
                                     A.ref(1, 8, mode=gf.GF_REF_READ), A.const(-5)]),
            (gf.GF_CALLEE_FWRITE, [A.heapref(0, 0, 64, gf.GF_REF_READ), A.const(1), A.const(3), A.const(out, "p")]),
            (gf.GF_CALLEE_FWRITE, [A.heapref(0, 1, 64, gf.GF_REF_READ), A.const(1), A.const(4), A.const(out, "p")]),
            (gf.GF_CALLEE_FPRINTF, [A.const(out, "p"), A.ref(2, 8, mode=gf.GF_REF_READ),
                                    A.heapref(0, 2, 64, gf.GF_REF_READ)]),
            (gf.GF_CALLEE_FPRINTF, [A.const(out, "p"), A.ref(2, 8, mode=gf.GF_REF_READ),
                                    A.heapref(0, 3, 64, gf.GF_REF_READ)]),
            (gf.GF_CALLEE_FWRITE, [A.ref(3, 1, mode=gf.GF_REF_READ), A.const(1), A.const(1), A.const(out, "p")]),
        ]
        ids = [ctx.register_call(c, args) for c, args in calls]
        body = [gf.Step.make(gf.GF_S_CALL, fmt_id=i, every=1, flags=gf.GF_STEP_BLOCKING) for i in ids]
        sc = scalars()
        ctx.take_output()
        ctx.run(gf.Program.make([], body, 3), gf.Instance.make({0: ptrs, 1: d1, 2: d2, 3: d3}, sc),
                mode=_mode(gf, mode))
        ctx.sync()
        text = ctx.take_output()
        line = "{}<-5>%#x|%#x|\n" % (base + 4000, 0x1234)
        assert text == "".join(line.format(f"<{k}>") for k in range(1, 4))
        ctx.set_heap(None)


@pytest.mark.parametrize("mode", MODES)
def test_call_after_the_last_region_sees_every_workgroups_writes(oracle_lib, mode, tmp_path):
    """A program whose last region writes an array that a host call then
    ships: the barrier after that region is kept, so the first workgroup
    copies what every workgroup wrote (the phase region's result, 64
    elements per workgroup over 128 workgroups), and fwrite puts exactly
    those bytes in a file."""
    import torch
    import paper_2306_11686_amd as gf
    import gf_inputs as gi
    print(f"call after last region mode={mode}", flush=True)
    n, P, s = 8192, 3, 4097
    a0 = gi.um11(12, 21, np.arange(n, dtype=np.uint64))
    a, b = dev(a0), torch.zeros(n, dtype=torch.float64, device="cuda")
    libc = ctypes.CDLL(None)
    libc.fopen.restype = ctypes.c_void_p
    path = tmp_path / "phase_result.bin"
    f = libc.fopen(str(path).encode(), b"wb")
    assert f
    try:
        with gf.Context(0, rpc_thread=True, rpc_payload=8 * n) as ctx:
            args = [gf.CallArg.ref(1, 8 * n, mode=gf.GF_REF_READ), gf.CallArg.const(8), gf.CallArg.const(n),
                    gf.CallArg.const(f, "p")]
            cid = ctx.register_call(gf.GF_CALLEE_FWRITE, args)
            pro = [gf.Step.make(gf.GF_R_PHASES, arr=(0, 1, -1), np=0, chunk=P, mask=s),
                   gf.Step.make(gf.GF_S_CALL, fmt_id=cid, every=1, flags=gf.GF_STEP_BLOCKING, sc=(0,))]
            sc = scalars()
            ctx.run(gf.Program.make(pro, [], 0), gf.Instance.make({0: a, 1: b}, sc, ip=(n,)),
                    mode=_mode(gf, mode), launch=gf.Launch.make(wg_size=64, num_wg=128))
            ctx.sync()
    finally:
        libc.fclose(ctypes.c_void_p(f))
    _, rb = oracle_lib.phases(a0, P, s)    # three phases: the result is in the second buffer
    assert np.array_equal(host(b), rb)
    assert host(sc)[0] == n                 # fwrite's count of items written
    assert np.array_equal(np.frombuffer(path.read_bytes(), dtype=np.float64), rb)
