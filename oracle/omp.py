"""The legacy 3D Jacobi loop built for the CPU with OpenMP (legacy_omp.c).

TIMING ONLY: the comparison point the paper uses for every parallel region
(the CPU OpenMP build of the same loop), timed on the host's cores by the
benchmark's CPU leg. It is not a parity reference.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblegacy_omp.so")
_SRC = os.path.join(_HERE, "legacy_omp.c")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SRC) > os.path.getmtime(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SRC) > os.path.getmtime(_SO):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        lib.lo_jacobi3d.restype = ctypes.c_double
        lib.lo_jacobi3d.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_int32]
        lib.lo_max_threads.restype = ctypes.c_int32
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().lo_max_threads())


def jacobi3d(u: np.ndarray, w: np.ndarray, sweeps: int, threads: int = 0) -> float:
    """`sweeps` sweeps in place on (u, w) (swapped after each); returns the
    last sweep's max residual."""
    for a in (u, w):
        if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"] or a.ndim != 3:
            raise ValueError("u and w must be contiguous float64 n^3 arrays")
    n = u.shape[0]
    return float(_load().lo_jacobi3d(n, u.ctypes.data, w.ctypes.data, sweeps, threads))
