"""Host library calls of the serial program: the oracle side of GF_S_CALL.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test suite uses
it; the product library never does, and nothing here is shared with it.

In the legacy program a call such as ``fprintf`` or ``sscanf`` runs on the
host and receives pointers into the program's own objects. Section 3.2 of the
paper keeps those semantics on the GPU by describing each pointer argument as
a reference (object, size, offset into the object, access mode). The object
is made available to the host, the call gets a pointer at the same offset
into the host's copy, and the object is copied back if the call may write it.
This module makes the call itself, with libc through ctypes, on host copies
of the objects, and applies what the callee wrote. A parity test compares it
with the device path, which ships the objects through the RPC payload.

Argument descriptors:

* ``("const", type, value)``: a value word. ``type`` is ``'i'`` (int64),
  ``'d'`` (double) or ``'p'`` (a host pointer such as a ``FILE *``).
* ``("scalar", type, slot)``: ``scal[slot]``, either as a double ``'d'`` or
  converted to int64 ``'i'`` (the C cast, truncation toward zero).
* ``("iter",)``: the 1-based body iteration, or 0 in the prologue.
* ``("ref", slot, start, size, offset, mode)``: a pointer ``offset`` bytes
  into the object ``arrays[slot]`` bytes ``[start, start + size)``. ``mode``
  is ``"r"``, ``"w"`` or ``"rw"``.
* ``("heapref", slot, element, max_bytes, mode)``: a pointer held in element
  ``element`` of the int64 array ``arrays[slot]``, whose object is not known
  in advance. The object is found at call time in the record the heap
  allocator keeps (Section 3.2, with the allocator of Section 3.4). That
  record is the ``heap=(address, memory, model)`` argument: the heap's
  device address, a uint8 array mirroring its bytes, and the
  ``oracle.heap.BalancedHeap`` model of its allocations. The object is
  shipped like a reference, with the pointer at the same offset into it. A
  pointer outside every live object, or an object larger than ``max_bytes``,
  is passed as a value.

Reading of write-only objects: the paper marks an object write-only when its
value at the call is unspecified, so it is not copied to the host. Here the
host copy starts at zero, and after the call the whole object is written
back. Bytes the callee leaves untouched therefore come back as zero, the
same contract the library documents.

Output that ``fprintf`` or ``fwrite`` sends to the host's stdout or stderr is
returned as bytes rather than written: for ``fprintf`` these are the bytes
``snprintf`` produces for the same format and arguments, as the C standard
defines them.
"""
from __future__ import annotations

import ctypes

import numpy as np

_libc = ctypes.CDLL(None)
STDOUT = ctypes.c_void_p.in_dll(_libc, "stdout").value
STDERR = ctypes.c_void_p.in_dll(_libc, "stderr").value

CALLEES = ("fprintf", "snprintf", "sscanf", "fwrite", "fread")


def _bytes_of(arr: np.ndarray) -> np.ndarray:
    """A writable uint8 view of a contiguous numpy array."""
    if not arr.flags["C_CONTIGUOUS"]:
        raise ValueError("objects live in contiguous arrays")
    return arr.reshape(-1).view(np.uint8)


def _word(kind_type, value):
    if kind_type == "i":
        return ctypes.c_longlong(int(value))
    if kind_type == "d":
        return ctypes.c_double(float(value))
    if kind_type == "p":
        return ctypes.c_void_p(value)
    raise ValueError(f"argument type {kind_type!r}")


def call(callee: str, args, arrays: dict, scal=None, it: int = -1, heap=None):
    """Make one call. ``arrays`` maps slot -> numpy array, and the objects of
    write and read-write references in it are updated in place. ``it`` is the
    0-based body iteration (-1 in the prologue). Returns ``(ret, out)``,
    where ``ret`` is the callee's return value and ``out`` is the bytes
    written to stdout or stderr (``b""`` when there are none)."""
    if callee not in CALLEES:
        raise ValueError(callee)
    cargs = []
    objects = []  # (view of the program's bytes, host copy, mode)
    for a in args:
        kind = a[0]
        if kind == "const":
            cargs.append(_word(a[1], a[2]))
        elif kind == "scalar":
            v = float(scal[a[2]])
            cargs.append(_word("i", int(v)) if a[1] == "i" else _word("d", v))
        elif kind == "iter":
            cargs.append(ctypes.c_longlong(it + 1))
        elif kind == "ref":
            _, slot, start, size, offset, mode = a
            if mode not in ("r", "w", "rw") or not 0 <= offset <= size or size < 1 or start < 0:
                raise ValueError(f"reference {a}")
            view = _bytes_of(arrays[slot])[start:start + size]
            if len(view) != size:
                raise ValueError("object outside its array")
            host = ctypes.create_string_buffer(size)
            if "r" in mode:
                ctypes.memmove(host, view.tobytes(), size)
            objects.append((view, host, mode))
            cargs.append(ctypes.c_void_p(ctypes.addressof(host) + offset))
        elif kind == "heapref":
            _, slot, element, max_bytes, mode = a
            p = int(np.asarray(arrays[slot]).reshape(-1).view(np.uint64)[element])
            found = None
            if heap is not None:
                addr, mem, model = heap
                off = p - addr
                if 0 <= off < mem.size:
                    found = model.find(off)
            if found is None or found[1] > max_bytes:
                cargs.append(ctypes.c_void_p(p))
                continue
            start, size = found
            view = mem[start:start + size]
            host = ctypes.create_string_buffer(size)
            if "r" in mode:
                ctypes.memmove(host, view.tobytes(), size)
            objects.append((view, host, mode))
            cargs.append(ctypes.c_void_p(ctypes.addressof(host) + (p - addr - start)))
        else:
            raise ValueError(f"argument kind {kind!r}")

    out = b""
    if callee == "fprintf":
        f = cargs[0].value
        if f in (STDOUT, STDERR):
            n = _libc.snprintf(None, ctypes.c_size_t(0), *cargs[1:])
            buf = ctypes.create_string_buffer(max(n, 0) + 1)
            ret = _libc.snprintf(buf, ctypes.c_size_t(len(buf)), *cargs[1:])
            out = buf.raw[:max(ret, 0)]
        else:
            ret = _libc.fprintf(*cargs)
    elif callee == "snprintf":
        ret = _libc.snprintf(cargs[0], ctypes.c_size_t(cargs[1].value), *cargs[2:])
    elif callee == "sscanf":
        ret = _libc.sscanf(*cargs)
    elif callee == "fwrite":
        size, n, f = cargs[1].value, cargs[2].value, cargs[3].value
        if f in (STDOUT, STDERR):
            out = ctypes.string_at(cargs[0].value, size * n) if size > 0 else b""
            ret = n
        else:
            _libc.fwrite.restype = ctypes.c_size_t
            ret = _libc.fwrite(cargs[0], ctypes.c_size_t(size), ctypes.c_size_t(n), ctypes.c_void_p(f))
    else:  # fread
        _libc.fread.restype = ctypes.c_size_t
        ret = _libc.fread(cargs[0], ctypes.c_size_t(cargs[1].value), ctypes.c_size_t(cargs[2].value),
                          ctypes.c_void_p(cargs[3].value))

    for view, host, mode in objects:
        if "w" in mode:
            view[:] = np.frombuffer(host.raw, dtype=np.uint8)
    return int(ret), out
