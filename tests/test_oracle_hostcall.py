"""Pins of the host-call oracle (oracle/hostcall.py) against hand-worked
results of the C library calls. Each case is chosen so that a plausible
mistake fails one check: a wrong object start or pointer offset, a missing
copy-in of a read-write object, a copy-back of a read-only object, no
zero-fill of a write-only object, a double passed as an int, a scalar
rounded instead of truncated. CPU only."""
import ctypes
import os

import numpy as np
import pytest

from oracle import hostcall as hc


def _cstr(s: bytes, size: int) -> np.ndarray:
    a = np.zeros(size, dtype=np.uint8)
    a[:len(s)] = np.frombuffer(s, dtype=np.uint8)
    return a


def test_snprintf_into_write_only_object_at_an_offset():
    fmt = _cstr(b"v=%lld|%.3f", 32)
    buf = np.full(40, 0xAB, dtype=np.uint8)
    arrays = {0: buf, 1: fmt}
    # object = bytes [8, 24) of slot 0, pointer 2 bytes into it
    ret, out = hc.call("snprintf", [("ref", 0, 8, 16, 2, "w"), ("const", "i", 14), ("ref", 1, 0, 32, 0, "r"),
                                    ("const", "i", 42), ("const", "d", 2.5)], arrays)
    assert ret == 10 and out == b""
    want = np.full(40, 0xAB, dtype=np.uint8)
    want[8:24] = 0                                   # write-only: zero-filled, then copied back whole
    want[10:21] = np.frombuffer(b"v=42|2.500\0", dtype=np.uint8)
    assert np.array_equal(buf, want)
    assert np.array_equal(fmt, _cstr(b"v=%lld|%.3f", 32))  # read-only: never written back


def test_snprintf_truncates_at_its_size_argument():
    arrays = {0: np.zeros(16, dtype=np.uint8), 1: _cstr(b"%lld", 8)}
    ret, _ = hc.call("snprintf", [("ref", 0, 0, 16, 0, "w"), ("const", "i", 4), ("ref", 1, 0, 8, 0, "r"),
                                  ("const", "i", 123456)], arrays)
    assert ret == 6                                   # the length it would have written
    assert bytes(arrays[0][:5]) == b"123\0\0"


def test_read_write_object_keeps_bytes_the_callee_does_not_write():
    arrays = {0: np.full(12, 0xCD, dtype=np.uint8), 1: _cstr(b"ab", 4)}
    ret, _ = hc.call("snprintf", [("ref", 0, 0, 12, 4, "rw"), ("const", "i", 8), ("ref", 1, 0, 4, 0, "r")],
                     arrays)
    assert ret == 2
    want = np.full(12, 0xCD, dtype=np.uint8)
    want[4:7] = np.frombuffer(b"ab\0", dtype=np.uint8)
    assert np.array_equal(arrays[0], want)


def test_sscanf_writes_through_references_into_typed_arrays():
    text = _cstr(b"17 0.125 -3", 16)
    ints = np.zeros(4, dtype=np.int64)
    dbls = np.zeros(3, dtype=np.float64)
    arrays = {0: text, 1: _cstr(b"%lld %lf %lld", 16), 2: ints, 3: dbls}
    # %lld -> ints[1] (object = the whole array, pointer 8 bytes in),
    # %lf -> dbls[2] (object = that element alone), %lld -> ints[3]
    ret, _ = hc.call("sscanf", [("ref", 0, 0, 16, 0, "r"), ("ref", 1, 0, 16, 0, "r"), ("ref", 2, 0, 32, 8, "rw"),
                                ("ref", 3, 16, 8, 0, "w"), ("ref", 2, 24, 8, 0, "w")], arrays)
    assert ret == 3
    assert ints.tolist() == [0, 17, 0, -3]
    assert dbls.tolist() == [0.0, 0.0, 0.125]


def test_fprintf_to_stdout_returns_the_formatted_bytes():
    arrays = {0: _cstr(b"%s|%lld|%.2f|%lld\n", 32), 1: _cstr(b"hi", 8)}
    scal = np.zeros(16)
    scal[3] = -2.75
    ret, out = hc.call("fprintf", [("const", "p", hc.STDOUT), ("ref", 0, 0, 32, 0, "r"), ("ref", 1, 0, 8, 0, "rw"),
                                   ("iter",), ("scalar", "d", 3), ("scalar", "i", 3)], arrays, scal, it=4)
    assert out == b"hi|5|-2.75|-2\n" and ret == len(out)   # iter+1; the int cast truncates toward zero
    assert bytes(arrays[1][:3]) == b"hi\0"


def test_prologue_iteration_argument_is_zero():
    arrays = {0: _cstr(b"%lld", 8)}
    _, out = hc.call("fprintf", [("const", "p", hc.STDERR), ("ref", 0, 0, 8, 0, "r"), ("iter",)], arrays, it=-1)
    assert out == b"0"


def test_fwrite_to_stderr_returns_the_raw_bytes():
    payload = np.arange(10, dtype=np.uint8)
    ret, out = hc.call("fwrite", [("ref", 0, 2, 6, 1, "r"), ("const", "i", 2), ("const", "i", 2),
                                  ("const", "p", hc.STDERR)], {0: payload})
    assert ret == 2 and out == bytes([3, 4, 5, 6])


def test_fread_from_a_file_fills_a_write_only_object(tmp_path):
    path = tmp_path / "data.bin"
    path.write_bytes(bytes(range(100, 140)))
    libc = ctypes.CDLL(None)
    libc.fopen.restype = ctypes.c_void_p
    f = libc.fopen(str(path).encode(), b"rb")
    assert f
    try:
        dst = np.full(64, 7, dtype=np.uint8)
        ret, _ = hc.call("fread", [("ref", 0, 16, 32, 0, "w"), ("const", "i", 4), ("const", "i", 5),
                                   ("const", "p", f)], {0: dst})
    finally:
        libc.fclose(ctypes.c_void_p(f))
    assert ret == 5
    want = np.full(64, 7, dtype=np.uint8)
    want[16:48] = 0
    want[16:36] = np.arange(100, 120, dtype=np.uint8)
    assert np.array_equal(dst, want)


def test_references_outside_their_array_are_rejected():
    with pytest.raises(ValueError):
        hc.call("fwrite", [("ref", 0, 8, 16, 0, "r"), ("const", "i", 1), ("const", "i", 1),
                           ("const", "p", hc.STDOUT)], {0: np.zeros(10, dtype=np.uint8)})
    with pytest.raises(ValueError):
        hc.call("fwrite", [("ref", 0, 0, 4, 5, "r"), ("const", "i", 1), ("const", "i", 1),
                           ("const", "p", hc.STDOUT)], {0: np.zeros(10, dtype=np.uint8)})


def test_heap_reference_ships_the_whole_object_found_by_the_allocator():
    """A pointer into the middle of a heap object: the whole object goes to
    the host, the callee gets the same offset into the copy, and read-write
    bytes it does not touch are kept."""
    from oracle.heap import BalancedHeap
    model = BalancedHeap(4096, 1, 1, 1)
    a = model.malloc(0, 0, 40)                     # 48-byte object at offset 16
    b = model.malloc(0, 0, 20)                     # 32-byte object at offset 80
    mem = np.full(4096, 0xAA, dtype=np.uint8)
    addr = 0x7000_0000
    ptrs = np.array([addr + a + 10, addr + b, addr + 4000, 0x1234], dtype=np.int64)
    fmt = _cstr(b"<%lld>", 8)
    heap = (addr, mem, model)
    ret, _ = hc.call("snprintf", [("heapref", 0, 0, 64, "rw"), ("const", "i", 8), ("ref", 1, 0, 8, 0, "r"),
                                  ("iter",)], {0: ptrs, 1: fmt}, it=6, heap=heap)
    assert ret == 3
    want = np.full(4096, 0xAA, dtype=np.uint8)
    want[a + 10:a + 14] = np.frombuffer(b"<7>\0", dtype=np.uint8)
    assert np.array_equal(mem, want)
    # write-only: the whole 32-byte object comes back, zero-filled past the text
    hc.call("snprintf", [("heapref", 0, 1, 64, "w"), ("const", "i", 32), ("ref", 1, 0, 8, 0, "r"),
                         ("const", "i", -5)], {0: ptrs, 1: fmt}, heap=heap)
    assert bytes(mem[b:b + 32]) == b"<-5>" + bytes(28)
    # an object larger than the limit, a pointer to no live object and a
    # pointer outside the heap all travel as plain values
    for k, limit in ((0, 32), (2, 64), (3, 64)):
        _, out = hc.call("fprintf", [("const", "p", hc.STDOUT), ("ref", 1, 0, 8, 0, "r"),
                                     ("heapref", 0, k, limit, "r")], {0: ptrs, 1: _cstr(b"%p", 8)}, heap=heap)
        assert out == b"%#x" % int(ptrs[k])
