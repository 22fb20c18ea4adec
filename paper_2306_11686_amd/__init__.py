"""GPU-First execution of legacy loop programs on MI355X: Python binding.

A thin ctypes layer over libgf.so (include/gf.h). Every step of a run
executes in the library's HIP kernels; this module only marshals arguments.
PyTorch supplies device memory (tensors) and streams. The library must be
built (``python -m paper_2306_11686_amd.build``); importing the binding on a
machine without it raises instead of falling back to anything else.
"""
from __future__ import annotations

from .binding import (  # noqa: F401
    GF_EXEC_PER_REGION, GF_EXEC_PERSISTENT, GF_EXEC_PER_REGION_GRAPH, GF_EXEC_KERNEL_SPLIT,
    GF_OP_SUM, GF_OP_MAX, GF_OP_NONE, GF_F64, GF_U32, GF_U64, GF_I64,
    GF_R_JACOBI2D, GF_R_JACOBI3D, GF_R_SPMV, GF_R_DOT, GF_R_AXPBY, GF_R_HIST, GF_R_OWNER, GF_R_PHASES,
    GF_S_SET, GF_S_COPY, GF_S_DIV, GF_S_SQRT, GF_S_SWAP, GF_S_RECORD, GF_S_PRINTF, GF_S_CALL,
    GF_STEP_BLOCKING, GF_STEP_TIMED, GF_STEP_NOWAIT, GF_LAUNCH_GIVEN, GF_LAUNCH_PREDICTED, GF_LAUNCH_TUNED,
    GF_LAUNCH_TUNED_CACHED, GF_NUM_CANDIDATES, GF_MLP_IN, GF_MLP_HIDDEN, GF_MLP_OUT, GF_MLP_NPARAMS,
    GF_CALLEE_FPRINTF, GF_CALLEE_SNPRINTF, GF_CALLEE_SSCANF, GF_CALLEE_FWRITE, GF_CALLEE_FREAD,
    GF_ARG_CONST, GF_ARG_SCALAR, GF_ARG_ITER, GF_ARG_REF, GF_ARG_HEAPREF, GF_REF_READ, GF_REF_WRITE, GF_REF_READWRITE,
    GF_CALL_MAX_ARGS, GF_CALL_MAX_REFS, GF_CALL_MAX_SITES,
    GF_HEAP_OP_MALLOC, GF_HEAP_OP_FREE, GF_HEAP_OP_FIND, GF_HEAP_BENCH_ROUNDTRIP, GF_HEAP_BENCH_HOLD,
    GF_HEAP_BENCH_RELEASE, Heap,
    GfError, Context, Step, Launch, Program, Instance, CallArg, CallStats, host_stream, lib_path, load_library,
    exported_symbols, tune_pick, batch_plan,
)
from . import programs  # noqa: F401
