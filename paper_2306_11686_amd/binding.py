"""ctypes marshalling for libgf.so; names and layouts mirror include/gf.h."""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libgf.so")

GF_OK, GF_EINVAL, GF_ENOMEM, GF_EHIP, GF_ETIMEOUT, GF_ERPC, GF_EDEVICE, GF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
_STATUS = {0: "GF_OK", -1: "GF_EINVAL", -2: "GF_ENOMEM", -3: "GF_EHIP", -4: "GF_ETIMEOUT", -5: "GF_ERPC",
           -6: "GF_EDEVICE", -7: "GF_EUNSUPPORTED"}

GF_OP_SUM, GF_OP_MAX, GF_OP_NONE = 0, 1, -1
GF_F64, GF_U32, GF_U64, GF_I64 = 0, 1, 2, 3
GF_EXEC_PER_REGION, GF_EXEC_PERSISTENT, GF_EXEC_PER_REGION_GRAPH, GF_EXEC_KERNEL_SPLIT = 0, 1, 2, 3

GF_R_JACOBI2D, GF_R_JACOBI3D, GF_R_SPMV, GF_R_DOT, GF_R_AXPBY, GF_R_HIST, GF_R_OWNER, GF_R_PHASES = \
    1, 2, 3, 4, 5, 6, 7, 8
GF_S_SET, GF_S_COPY, GF_S_DIV, GF_S_SQRT, GF_S_SWAP, GF_S_RECORD, GF_S_PRINTF, GF_S_CALL = \
    32, 33, 34, 35, 36, 37, 38, 39
GF_STEP_BLOCKING, GF_STEP_TIMED, GF_STEP_NOWAIT = 1, 2, 4
GF_LAUNCH_GIVEN, GF_LAUNCH_PREDICTED, GF_LAUNCH_TUNED, GF_LAUNCH_TUNED_CACHED = 0, 1, 2, 3

GF_CALLEE_FPRINTF, GF_CALLEE_SNPRINTF, GF_CALLEE_SSCANF, GF_CALLEE_FWRITE, GF_CALLEE_FREAD = 1, 2, 3, 4, 5
GF_ARG_CONST, GF_ARG_SCALAR, GF_ARG_ITER, GF_ARG_REF, GF_ARG_HEAPREF = 0, 1, 2, 3, 4
GF_REF_READ, GF_REF_WRITE, GF_REF_READWRITE = 1, 2, 3
GF_CALL_MAX_ARGS, GF_CALL_MAX_REFS, GF_CALL_MAX_SITES = 8, 4, 64

GF_MAX_ARRAYS = 16
GF_MAX_SCALARS = 16
GF_MAX_IPARAMS = 8


class GfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Step(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("arr", ctypes.c_int32 * 5), ("sc", ctypes.c_int32 * 3),
                ("red_op", ctypes.c_int32), ("np", ctypes.c_int32), ("every", ctypes.c_int32),
                ("fmt_id", ctypes.c_int32), ("nargs", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("mask", ctypes.c_uint32), ("chunk", ctypes.c_int64), ("c", ctypes.c_double)]

    @classmethod
    def make(cls, kind, arr=(), sc=(), red_op=GF_OP_NONE, np=0, every=0, fmt_id=0, nargs=0, flags=0,
             mask=0, chunk=0, c=0.0):
        s = cls()
        s.kind = kind
        for i in range(5):
            s.arr[i] = arr[i] if i < len(arr) else -1
        for i in range(3):
            s.sc[i] = sc[i] if i < len(sc) else -1
        s.red_op, s.np, s.every, s.fmt_id, s.nargs = red_op, np, every, fmt_id, nargs
        s.flags, s.mask, s.chunk, s.c = flags, mask, chunk, float(c)
        return s


class Program(ctypes.Structure):
    _fields_ = [("n_prologue", ctypes.c_int32), ("prologue", ctypes.POINTER(Step)),
                ("n_body", ctypes.c_int32), ("body", ctypes.POINTER(Step)), ("iters", ctypes.c_int32)]

    @classmethod
    def make(cls, prologue, body, iters):
        p = cls()
        p._pro = (Step * max(1, len(prologue)))(*prologue)
        p._body = (Step * max(1, len(body)))(*body)
        p.n_prologue = len(prologue)
        p.prologue = ctypes.cast(p._pro, ctypes.POINTER(Step))
        p.n_body = len(body)
        p.body = ctypes.cast(p._body, ctypes.POINTER(Step))
        p.iters = iters
        return p


class Instance(ctypes.Structure):
    _fields_ = [("arr", ctypes.c_void_p * GF_MAX_ARRAYS), ("scal", ctypes.c_void_p),
                ("ip", ctypes.c_int64 * GF_MAX_IPARAMS)]

    @classmethod
    def make(cls, arrays: dict, scal_ptr: int, ip=()):
        """arrays: {slot: device pointer (int) or a tensor}; scal_ptr: device pointer of 16 doubles.
        Tensors passed here are referenced by the instance, so that a
        temporary one is not freed (and its memory handed to another tensor)
        while the instance is still in use."""
        inst = cls()
        for k, v in arrays.items():
            inst.arr[k] = _ptr(v)
        inst.scal = _ptr(scal_ptr)
        for i, v in enumerate(ip):
            inst.ip[i] = int(v)
        inst._keep = [v for v in list(arrays.values()) + [scal_ptr] if not isinstance(v, int)]
        return inst


class Launch(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_int32), ("num_wg", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("tile_z", ctypes.c_int32), ("items", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("prefetch", ctypes.c_int32)]

    @classmethod
    def make(cls, wg_size=0, num_wg=0, tile_y=0, tile_z=0, items=0, xcd_remap=1, prefetch=0):
        return cls(wg_size, num_wg, tile_y, tile_z, items, xcd_remap, prefetch)


class RunStats(ctypes.Structure):
    _fields_ = [("regions", ctypes.c_int32), ("launches", ctypes.c_int32), ("barriers", ctypes.c_int32),
                ("num_wg", ctypes.c_int32), ("wg_size", ctypes.c_int32), ("rpc_posted", ctypes.c_int32),
                ("candidate", ctypes.c_int32), ("launch_source", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class CtxOpts(ctypes.Structure):
    _fields_ = [("rpc_slots", ctypes.c_int32), ("rpc_capture", ctypes.c_int32), ("rpc_thread", ctypes.c_int32),
                ("rpc_timeout_us", ctypes.c_int64), ("barrier_timeout_us", ctypes.c_int64),
                ("rpc_payload", ctypes.c_int64), ("tune_fallback", ctypes.c_int32)]


class CallArg(ctypes.Structure):
    """One argument record of a host call site (gf_call_arg)."""
    _fields_ = [("kind", ctypes.c_int32), ("type", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("value", ctypes.c_int64), ("start", ctypes.c_int64),
                ("size", ctypes.c_int64), ("offset", ctypes.c_int64)]

    @classmethod
    def const(cls, value, type="i"):
        """A value word: an int ('i'), a float ('d') or a host pointer ('p')."""
        a = cls()
        a.kind, a.type = GF_ARG_CONST, ord(type)
        if type == "d":
            a.value = ctypes.c_int64.from_buffer_copy(ctypes.c_double(float(value))).value
        else:
            a.value = ctypes.c_int64(int(value)).value
        return a

    @classmethod
    def scalar(cls, slot, type="d"):
        a = cls()
        a.kind, a.type, a.slot = GF_ARG_SCALAR, ord(type), slot
        return a

    @classmethod
    def iteration(cls):
        a = cls()
        a.kind, a.type = GF_ARG_ITER, ord("i")
        return a

    @classmethod
    def ref(cls, slot, size, start=0, offset=0, mode=GF_REF_READWRITE):
        """A pointer `offset` bytes into the object of `size` bytes at byte
        `start` of array slot `slot`."""
        a = cls()
        a.kind, a.type, a.slot, a.mode = GF_ARG_REF, ord("p"), slot, mode
        a.start, a.size, a.offset = start, size, offset
        return a

    @classmethod
    def heapref(cls, slot, element, max_bytes, mode=GF_REF_READWRITE):
        """A heap pointer held in element `element` of int64 array slot
        `slot`: its object is found in the context's heap at call time."""
        a = cls()
        a.kind, a.type, a.slot, a.mode = GF_ARG_HEAPREF, ord("p"), slot, mode
        a.start, a.size, a.offset = element, max_bytes, 0
        return a


class HeapOpts(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_int64), ("thread_slots", ctypes.c_int32), ("team_slots", ctypes.c_int32),
                ("first_ratio", ctypes.c_int32), ("vendor", ctypes.c_int32), ("lock_timeout_us", ctypes.c_int64)]


GF_HEAP_OP_MALLOC, GF_HEAP_OP_FREE, GF_HEAP_OP_FIND = 1, 2, 3
GF_HEAP_BENCH_ROUNDTRIP, GF_HEAP_BENCH_HOLD, GF_HEAP_BENCH_RELEASE = 0, 1, 2


class CallStats(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64), ("dev_args_us", ctypes.c_double), ("dev_copy_in_us", ctypes.c_double),
                ("dev_wait_us", ctypes.c_double), ("dev_copy_out_us", ctypes.c_double),
                ("host_decode_us", ctypes.c_double), ("host_call_us", ctypes.c_double),
                ("host_reply_us", ctypes.c_double), ("transit_us", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def host_stream(name: str) -> int:
    """The host FILE * of the process's stdout or stderr (a value argument
    for fprintf / fwrite call sites)."""
    if name not in ("stdout", "stderr"):
        raise ValueError(name)
    return ctypes.c_void_p.in_dll(ctypes.CDLL(None), name).value


def _ptr(v) -> int:
    if v is None:
        return 0
    if isinstance(v, int):
        return v
    if hasattr(v, "data_ptr"):
        return v.data_ptr()
    raise TypeError(f"cannot take a device pointer of {type(v)}")


_lib = None

# name -> (restype, argtypes); every function declared in include/gf.h
_SIGS = {
    "gf_ctx_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(CtxOpts), ctypes.POINTER(ctypes.c_void_p)]),
    "gf_ctx_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "gf_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "gf_region_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Program), ctypes.POINTER(Instance),
                                     ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Launch),
                                     ctypes.POINTER(RunStats), ctypes.c_void_p]),
    "gf_reduce": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_void_p]),
    "gf_reduce_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "gf_rpc_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "gf_rpc_register_format": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_char_p]),
    "gf_rpc_take_output": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64]),
    "gf_rpc_register_call": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(CallArg),
                                              ctypes.c_int32]),
    "gf_rpc_call_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(CallStats),
                                         ctypes.c_int32]),
    "gf_heap_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(HeapOpts), ctypes.POINTER(ctypes.c_void_p)]),
    "gf_heap_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "gf_heap_reset": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gf_heap_script": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "gf_heap_bench": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "gf_heap_counts": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32]),
    "gf_heap_tops": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int32]),
    "gf_heap_base": (ctypes.c_void_p, [ctypes.c_void_p]),
    "gf_ctx_set_heap": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gf_sync": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(RunStats)]),
    "gf_persistent_capacity": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Program), ctypes.c_int32]),
    "gf_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_void_p]),
    "gf_tune_candidates": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Program), ctypes.POINTER(Instance),
                                            ctypes.POINTER(Launch)]),
    "gf_tune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Program), ctypes.POINTER(Instance), ctypes.c_int32,
                                 ctypes.c_int32, ctypes.POINTER(Launch), ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "gf_tune_pick": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_float), ctypes.c_int32]),
    "gf_region_run_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Program), ctypes.POINTER(Instance),
                                             ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Launch),
                                             ctypes.POINTER(RunStats), ctypes.c_void_p]),
    "gf_batch_plan": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                       ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "gf_batch_misplaced": (ctypes.c_int64, [ctypes.c_void_p]),
    "gf_tune_batched": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Program), ctypes.POINTER(Instance),
                                         ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Launch),
                                         ctypes.POINTER(ctypes.c_float), ctypes.c_void_p]),
    "gf_mlp_forward": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 2 + [ctypes.c_int32] +
                       [ctypes.c_void_p] * 4),
    "gf_mlp_backward": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 7 + [ctypes.c_int32, ctypes.c_float,
                                                                                    ctypes.c_void_p, ctypes.c_void_p]),
    "gf_mlp_loss": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_float,
                                                                                ctypes.c_void_p, ctypes.c_void_p]),
    "gf_adam_step": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_float,
                                                                                 ctypes.c_float, ctypes.c_float,
                                                                                 ctypes.c_float, ctypes.c_int32,
                                                                                 ctypes.c_void_p]),
    "gf_train_predictor": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 6 + [ctypes.c_int32, ctypes.c_float,
                                                                                      ctypes.c_int32, ctypes.c_float,
                                                                                      ctypes.c_void_p,
                                                                                      ctypes.c_void_p]),
    "gf_predictor_set": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "gf_predict": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint8),
                                    ctypes.POINTER(ctypes.c_float)]),
    "gf_nest_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Program), ctypes.POINTER(Instance),
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "gf_predict_launch": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Program), ctypes.POINTER(Instance),
                                           ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Launch), ctypes.c_void_p]),
}

GF_MLP_IN, GF_MLP_HIDDEN, GF_MLP_OUT = 8, 64, 32
GF_MLP_NPARAMS = 64 * 8 + 64 + 64 * 64 + 64 + 32 * 64 + 32

GF_NUM_CANDIDATES = 32


def lib_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libgf.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"libgf.so is not built ({_LIB_PATH}); run python -m paper_2306_11686_amd.build")
    import torch  # noqa: F401  -- binds the process to torch's HIP runtime first
    lib = ctypes.CDLL(_LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return sorted(_SIGS)


# Contexts and heaps still open when the interpreter exits are closed by an
# exit hook, before module teardown; a finalizer that runs later (during
# interpreter finalization) makes no HIP call and leaks the handle instead.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass


def tune_pick(ms) -> int:
    """Host-only argmin over finite timings (the library's gf_tune_pick)."""
    lib = load_library()
    arr = (ctypes.c_float * len(ms))(*ms)
    return lib.gf_tune_pick(arr, len(ms))


def batch_plan(items, weights=None, budget: int = 4096, align: bool = True):
    """Host-only plan of a batched persistent launch (the library's
    gf_batch_plan): (grid, group sizes, XCD per instance or -1)."""
    lib = load_library()
    n = len(items)
    it = (ctypes.c_int64 * n)(*[int(v) for v in items])
    w = (ctypes.c_double * n)(*[float(v) for v in weights]) if weights is not None else None
    g = (ctypes.c_int32 * n)()
    x = (ctypes.c_int32 * n)()
    grid = lib.gf_batch_plan(n, it, w, budget, 1 if align else 0, g, x)
    if grid < 0:
        raise GfError(grid, "gf_batch_plan: invalid arguments")
    return grid, list(g), list(x)


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Context:
    """One libgf context on a HIP device."""

    def __init__(self, device: int = 0, rpc_slots: int = 0, rpc_capture: bool = False, rpc_thread: bool = False,
                 rpc_timeout_us: int = 0, barrier_timeout_us: int = 0, rpc_payload: int = 0,
                 tune_fallback: bool = True):
        self.lib = load_library()
        opts = CtxOpts(rpc_slots, 1 if rpc_capture else 0, 1 if rpc_thread else 0, rpc_timeout_us,
                       barrier_timeout_us, rpc_payload, 0 if tune_fallback else -1)
        h = ctypes.c_void_p()
        st = self.lib.gf_ctx_create(device, ctypes.byref(opts), ctypes.byref(h))
        if st != GF_OK:
            raise GfError(st, "gf_ctx_create failed")
        self.h = h
        self.device = device
        _LIVE.add(self)

    def close(self):
        """Destroy the context (waits for the device, joins the server
        thread). Idempotent."""
        h, self.h = getattr(self, "h", None), None
        if h:
            self.lib.gf_ctx_destroy(h)

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        if st < 0:
            raise GfError(st, self.lib.gf_last_error(self.h).decode())
        return st

    def last_error(self) -> str:
        return self.lib.gf_last_error(self.h).decode()

    def run(self, program: Program, instances, mode: int = GF_EXEC_PERSISTENT, launch: Launch | None = None,
            stream=None) -> dict:
        if isinstance(instances, Instance):
            instances = [instances]
        arr = (Instance * len(instances))(*instances)
        stats = RunStats()
        st = self.lib.gf_region_run(self.h, ctypes.byref(program), arr, len(instances), mode,
                                    ctypes.byref(launch) if launch is not None else None, ctypes.byref(stats),
                                    _stream_handle(stream))
        self._check(st)
        return stats.as_dict()

    def run_batched(self, program: Program, instances, launches, mode: int = GF_EXEC_PERSISTENT,
                    stream=None) -> dict:
        """One run of many instances with a launch shape per instance
        (rows per tile, relative share of the grid)."""
        if len(launches) != len(instances):
            raise ValueError("one launch per instance")
        arr = (Instance * len(instances))(*instances)
        ls = (Launch * len(launches))(*launches)
        stats = RunStats()
        self._check(self.lib.gf_region_run_batched(self.h, ctypes.byref(program), arr, len(instances), mode, ls,
                                                   ctypes.byref(stats), _stream_handle(stream)))
        return stats.as_dict()

    def batch_misplaced(self) -> int:
        """Workgroups of the last batched persistent launch found on another
        XCD than its table assumed (0: groups kept to one XCD; -1: no check)."""
        return int(self.lib.gf_batch_misplaced(self.h))

    def tune_batched(self, program: Program, instances, reps: int = 3, stream=None):
        """The batched autotuner: returns (launches, one per instance; median ms of the best run)."""
        arr = (Instance * len(instances))(*instances)
        out = (Launch * len(instances))()
        ms = ctypes.c_float(0.0)
        self._check(self.lib.gf_tune_batched(self.h, ctypes.byref(program), arr, len(instances), reps, out,
                                             ctypes.byref(ms), _stream_handle(stream)))
        return [out[i] for i in range(len(instances))], float(ms.value)

    def reduce(self, op: int, dtype: int, d_in, n: int, d_out, stream=None):
        self._check(self.lib.gf_reduce(self.h, op, dtype, _ptr(d_in), n, _ptr(d_out), _stream_handle(stream)))

    def reduce_noalloc(self, op: int, dtype: int, d_in, n: int, d_out, stream=None):
        self._check(self.lib.gf_reduce_noalloc(self.h, op, dtype, _ptr(d_in), n, _ptr(d_out),
                                               _stream_handle(stream)))

    def rpc_poll(self, max_requests: int = 1 << 20, timeout_us: int = 0) -> int:
        return self._check(self.lib.gf_rpc_poll(self.h, max_requests, timeout_us))

    def register_format(self, fmt: str, sig: str) -> int:
        return self._check(self.lib.gf_rpc_register_format(self.h, fmt.encode(), sig.encode()))

    def register_call(self, callee: int, args) -> int:
        arr = (CallArg * max(1, len(args)))(*args)
        return self._check(self.lib.gf_rpc_register_call(self.h, callee, arr, len(args)))

    def set_heap(self, heap):
        """Let host calls look up GF_ARG_HEAPREF pointers in `heap` (None: no heap)."""
        self._check(self.lib.gf_ctx_set_heap(self.h, heap.h if heap is not None else None))

    def call_stats(self, call_id: int, reset: bool = False) -> dict:
        out = CallStats()
        self._check(self.lib.gf_rpc_call_stats(self.h, call_id, ctypes.byref(out), 1 if reset else 0))
        return out.as_dict()

    def take_output(self, cap: int = 1 << 20) -> str:
        buf = ctypes.create_string_buffer(cap)
        self._check(self.lib.gf_rpc_take_output(self.h, buf, cap))
        return buf.value.decode()

    def sync(self, stream=None) -> dict:
        stats = RunStats()
        self._check(self.lib.gf_sync(self.h, _stream_handle(stream), ctypes.byref(stats)))
        return stats.as_dict()

    def capacity(self, program: Program, wg_size: int = 0) -> int:
        return self.lib.gf_persistent_capacity(self.h, ctypes.byref(program), wg_size)

    def tune_candidates(self, program: Program, instance: Instance):
        out = (Launch * GF_NUM_CANDIDATES)()
        self._check(self.lib.gf_tune_candidates(self.h, ctypes.byref(program), ctypes.byref(instance), out))
        return list(out)

    def tune(self, program: Program, instances, mode: int = GF_EXEC_PERSISTENT, candidates=None, reps: int = 3,
             stream=None):
        """Time candidate launches on real runs; returns (ms list, best index)."""
        if isinstance(instances, Instance):
            instances = [instances]
        arr = (Instance * len(instances))(*instances)
        n = len(candidates) if candidates is not None else GF_NUM_CANDIDATES
        cand = (Launch * n)(*candidates) if candidates is not None else None
        ms = (ctypes.c_float * n)()
        best = ctypes.c_int32(-1)
        self._check(self.lib.gf_tune(self.h, ctypes.byref(program), arr, len(instances), mode, cand, n, reps, ms,
                                     ctypes.byref(best), _stream_handle(stream)))
        return [float(v) for v in ms], best.value

    # -- launch-config predictor ------------------------------------------
    def mlp_forward(self, params, feats, batch, y, z1=None, z2=None, stream=None):
        self._check(self.lib.gf_mlp_forward(self.h, _ptr(params), _ptr(feats), batch, _ptr(y), _ptr(z1), _ptr(z2),
                                            _stream_handle(stream)))

    def mlp_backward(self, params, feats, z1, z2, y, target, mask, batch, inv_norm, grads, stream=None):
        self._check(self.lib.gf_mlp_backward(self.h, _ptr(params), _ptr(feats), _ptr(z1), _ptr(z2), _ptr(y),
                                             _ptr(target), _ptr(mask), batch, inv_norm, _ptr(grads),
                                             _stream_handle(stream)))

    def mlp_loss(self, y, target, mask, count, inv_norm, loss, stream=None):
        self._check(self.lib.gf_mlp_loss(self.h, _ptr(y), _ptr(target), _ptr(mask), count, inv_norm, _ptr(loss),
                                         _stream_handle(stream)))

    def adam_step(self, params, grads, m, v, n, lr, beta1, beta2, eps, t, stream=None):
        self._check(self.lib.gf_adam_step(self.h, _ptr(params), _ptr(grads), _ptr(m), _ptr(v), n, lr, beta1, beta2,
                                          eps, t, _stream_handle(stream)))

    def train_predictor(self, params, m, v, feats, target, mask, batch, inv_norm, epochs, lr, loss_hist=None,
                        stream=None):
        self._check(self.lib.gf_train_predictor(self.h, _ptr(params), _ptr(m), _ptr(v), _ptr(feats), _ptr(target),
                                                _ptr(mask), batch, inv_norm, epochs, lr, _ptr(loss_hist),
                                                _stream_handle(stream)))

    def predictor_set(self, params, mean, std):
        P = (ctypes.c_float * GF_MLP_NPARAMS)(*[float(v) for v in params])
        M = (ctypes.c_float * GF_MLP_IN)(*[float(v) for v in mean])
        S = (ctypes.c_float * GF_MLP_IN)(*[float(v) for v in std])
        self._check(self.lib.gf_predictor_set(self.h, P, M, S))

    def predict(self, features, valid=None, want_scores=False):
        f = (ctypes.c_double * GF_MLP_IN)(*[float(v) for v in features])
        vm = (ctypes.c_uint8 * GF_MLP_OUT)(*[1 if x else 0 for x in valid]) if valid is not None else None
        sc = (ctypes.c_float * GF_MLP_OUT)()
        r = self.lib.gf_predict(self.h, f, vm, sc)
        if r < -1:
            self._check(r)
        return (r, [float(v) for v in sc]) if want_scores else r

    def nest_features(self, program: Program, instances, stream=None):
        """The predictor's raw features of `program` bound to `instances`."""
        if isinstance(instances, Instance):
            instances = [instances]
        arr = (Instance * len(instances))(*instances)
        out = (ctypes.c_double * GF_MLP_IN)()
        self._check(self.lib.gf_nest_features(self.h, ctypes.byref(program), arr, len(instances), out,
                                              _stream_handle(stream)))
        return [float(v) for v in out]

    def predict_launch(self, program: Program, instances, mode: int = GF_EXEC_PERSISTENT, stream=None):
        """(candidate index, Launch) chosen by the installed predictor, or (-1, None)."""
        if isinstance(instances, Instance):
            instances = [instances]
        arr = (Instance * len(instances))(*instances)
        out = Launch()
        r = self.lib.gf_predict_launch(self.h, ctypes.byref(program), arr, len(instances), mode, ctypes.byref(out),
                                       _stream_handle(stream))
        if r < -1:
            self._check(r)
        return (r, out) if r >= 0 else (-1, None)

    def copy(self, dst, src, nbytes: int, num_wg: int = 0, stream=None):
        self._check(self.lib.gf_copy(self.h, _ptr(dst), _ptr(src), nbytes, num_wg, _stream_handle(stream)))


class Heap:
    """The balanced device heap (include/gf_heap.h)."""

    def __init__(self, device: int = 0, nbytes: int = 1 << 26, thread_slots: int = 32, team_slots: int = 16,
                 first_ratio: int = 4, vendor: bool = False, lock_timeout_us: int = 0):
        self.lib = load_library()
        self.opts = HeapOpts(nbytes, thread_slots, team_slots, first_ratio, 1 if vendor else 0, lock_timeout_us)
        h = ctypes.c_void_p()
        st = self.lib.gf_heap_create(device, ctypes.byref(self.opts), ctypes.byref(h))
        if st != GF_OK:
            raise GfError(st, "gf_heap_create failed")
        self.h = h
        _LIVE.add(self)

    def close(self):
        """Destroy the heap. Idempotent."""
        h, self.h = getattr(self, "h", None), None
        if h:
            self.lib.gf_heap_destroy(h)

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st, what):
        if st != GF_OK:
            raise GfError(st, what)

    def reset(self, stream=None):
        self._check(self.lib.gf_heap_reset(self.h, _stream_handle(stream)), "gf_heap_reset")

    def script(self, d_ops, n_ops: int, d_res, stream=None):
        self._check(self.lib.gf_heap_script(self.h, _ptr(d_ops), n_ops, _ptr(d_res), _stream_handle(stream)),
                    "gf_heap_script")

    def bench(self, teams: int, threads: int, nbytes: int, mode: int = GF_HEAP_BENCH_ROUNDTRIP, d_ptrs=None,
              stream=None):
        self._check(self.lib.gf_heap_bench(self.h, teams, threads, nbytes, mode, _ptr(d_ptrs),
                                           _stream_handle(stream)), "gf_heap_bench")

    def counts(self, reset: bool = False) -> dict:
        out = (ctypes.c_uint64 * 4)()
        self._check(self.lib.gf_heap_counts(self.h, out, 1 if reset else 0), "gf_heap_counts")
        return {"null": out[0], "corrupt": out[1], "timeouts": out[2], "bad_frees": out[3]}

    def base(self) -> int:
        """Device address of the heap's first byte."""
        return self.lib.gf_heap_base(self.h) or 0

    def tops(self):
        n = self.opts.thread_slots * self.opts.team_slots
        out = (ctypes.c_uint32 * n)()
        self._check(self.lib.gf_heap_tops(self.h, out, n), "gf_heap_tops")
        return list(out)
