"""Seeded synthetic inputs for the legacy-loop workloads.

This module only *draws* inputs: grids, right-hand sides, the 27-point CSR
matrix, histogram keys, instance sizes and loop-nest features. It holds none
of the arithmetic of the method being executed (no stencil, no SpMV, no
reduction), so both the GPU path and the CPU oracle may consume what it
produces without sharing any of the computation under test.

Random numbers come from one counter-based generator: the SplitMix64 output
function of Steele, Lea and Flood ("Fast Splittable Pseudorandom Number
Generators", OOPSLA 2014), evaluated at counter positions so that every value
depends only on (seed, stream, linear index):

    base(seed, stream) = mix64(seed * GAMMA + stream)
    H(seed, stream, i) = mix64(base + (i + 1) * GAMMA)      (mod 2**64)

i.e. H(seed, stream, i) is the (i+1)-th output of a SplitMix64 generator whose
state starts at ``base``. ``U01 = (H >> 11) * 2**-53`` is exact in double.

Stream ids: 1 grids (2D/3D Jacobi), 2 CG right-hand side, 3 uniform histogram
keys (and the high key bits of Zipf keys), 4 Zipf rank draws, 5 batched
instance sides, 7 loop-nest features, 1000+i interior of batched instance i.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_FILL_SO = os.path.join(_HERE, "libgfinputs.so")
_fill = None


def build(force: bool = True) -> str:
    """Compile the bulk-fill helper (fill.c) used for large grids and keys."""
    if force or not os.path.exists(_FILL_SO):
        tmp = _FILL_SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "fill.c")])
        os.replace(tmp, _FILL_SO)
    return _FILL_SO


def _fill_lib():
    global _fill
    if _fill is None:
        src = os.path.join(_HERE, "fill.c")
        if not os.path.exists(_FILL_SO) or os.path.getmtime(src) > os.path.getmtime(_FILL_SO):
            try:
                build(force=True)
            except (OSError, subprocess.CalledProcessError):
                return None
        lib = ctypes.CDLL(_FILL_SO)
        U64, I64, P = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
        lib.gfi_u01.argtypes = [U64, U64, U64, I64, P]
        lib.gfi_grid3d.argtypes = [I64, U64, U64, P]
        lib.gfi_keys_u32.argtypes = [U64, U64, U64, I64, P]
        lib.gfi_keys_zipf.argtypes = [U64, U64, U64, I64, P, I64, P]
        _fill = lib
    return _fill

GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_U64 = np.uint64

STREAM_GRID = 1
STREAM_CG_RHS = 2
STREAM_HIST = 3
STREAM_ZIPF = 4
STREAM_SIDES = 5
STREAM_NESTS = 7
STREAM_INSTANCE0 = 1000


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output mixing function on a uint64 array (wraps mod 2**64)."""
    z = np.asarray(z, dtype=_U64)
    z = (z ^ (z >> _U64(30))) * _U64(_M1)
    z = (z ^ (z >> _U64(27))) * _U64(_M2)
    return z ^ (z >> _U64(31))


def stream_base(seed: int, stream: int) -> np.uint64:
    v = (int(seed) * GAMMA + int(stream)) & 0xFFFFFFFFFFFFFFFF
    return mix64(np.array([v], dtype=_U64))[0]


def hash_u64(seed: int, stream: int, idx) -> np.ndarray:
    """H(seed, stream, idx) for an integer array of linear indices."""
    idx = np.asarray(idx, dtype=_U64)
    with np.errstate(over="ignore"):
        return mix64(stream_base(seed, stream) + (idx + _U64(1)) * _U64(GAMMA))


def splitmix64_sequence(state: int, n: int) -> np.ndarray:
    """First n outputs of a plain SplitMix64 generator started at ``state``."""
    idx = np.arange(n, dtype=_U64)
    with np.errstate(over="ignore"):
        return mix64(_U64(state) + (idx + _U64(1)) * _U64(GAMMA))


def u01(seed: int, stream: int, idx) -> np.ndarray:
    """Uniform [0, 1) doubles: the top 53 bits of H scaled by 2**-53 (exact)."""
    return (hash_u64(seed, stream, idx) >> _U64(11)).astype(np.float64) * (2.0 ** -53)


def um11(seed: int, stream: int, idx) -> np.ndarray:
    """Uniform [-1, 1) doubles: 2*U01 - 1 (exact in double)."""
    return 2.0 * u01(seed, stream, idx) - 1.0


# --------------------------------------------------------------------------
# Jacobi grids: an N^d array whose outer layer is the zero Dirichlet boundary
# --------------------------------------------------------------------------

def grid2d(n: int, seed: int = 1, stream: int = STREAM_GRID) -> np.ndarray:
    """n x n row-major float64 grid; interior U01 keyed by the linear index."""
    u = np.zeros((n, n), dtype=np.float64)
    if n > 2:
        idx = np.arange(n * n, dtype=np.uint64).reshape(n, n)
        u[1:-1, 1:-1] = u01(seed, stream, idx[1:-1, 1:-1])
    return u


def grid3d(n: int, seed: int = 1, stream: int = STREAM_GRID, out: np.ndarray | None = None,
           fast: bool = True) -> np.ndarray:
    """n^3 float64 grid u[z][y][x] (x fastest); interior U01; built plane by plane.

    fast=True uses the compiled fill (same definition) when it is available."""
    lib = _fill_lib() if fast else None
    if lib is not None:
        u = np.empty((n, n, n), dtype=np.float64) if out is None else out
        lib.gfi_grid3d(n, seed, stream, u.ctypes.data_as(ctypes.c_void_p))
        return u
    u = np.zeros((n, n, n), dtype=np.float64) if out is None else out
    if out is not None:
        u[0] = 0.0
        u[-1] = 0.0
    if n <= 2:
        u[...] = 0.0
        return u
    plane = n * n
    yx = np.arange(plane, dtype=np.uint64).reshape(n, n)
    chunk = max(1, (1 << 22) // plane)
    for z0 in range(1, n - 1, chunk):
        z1 = min(n - 1, z0 + chunk)
        idx = (np.arange(z0, z1, dtype=np.uint64)[:, None, None] * np.uint64(plane)) + yx[None]
        blk = u01(seed, stream, idx)
        blk[:, 0, :] = 0.0
        blk[:, -1, :] = 0.0
        blk[:, :, 0] = 0.0
        blk[:, :, -1] = 0.0
        u[z0:z1] = blk
    return u


def eigenmode2d(n: int, p: int = 1, q: int = 1) -> np.ndarray:
    """sin(p*pi*i*h) * sin(q*pi*j*h), h = 1/(n-1); zero on the boundary."""
    h = 1.0 / (n - 1)
    i = np.arange(n)
    sx = np.sin(p * np.pi * i * h)
    sy = np.sin(q * np.pi * i * h)
    u = np.outer(sy, sx)
    u[0, :] = u[-1, :] = 0.0
    u[:, 0] = u[:, -1] = 0.0
    return u


def eigenmode3d(n: int, p: int = 1, q: int = 1, r: int = 1) -> np.ndarray:
    h = 1.0 / (n - 1)
    i = np.arange(n)
    sx = np.sin(p * np.pi * i * h)
    sy = np.sin(q * np.pi * i * h)
    sz = np.sin(r * np.pi * i * h)
    u = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    u[0] = u[-1] = 0.0
    u[:, 0] = u[:, -1] = 0.0
    u[:, :, 0] = u[:, :, -1] = 0.0
    return np.ascontiguousarray(u)


# --------------------------------------------------------------------------
# CG inputs: 27-point matrix in CSR and the right-hand side
# --------------------------------------------------------------------------

def poisson27_csr(m: int):
    """CSR of the 27-point operator on an m^3 grid.

    Row id = i + m*j + m*m*k. A row holds every neighbour (di, dj, dk) in
    {-1,0,1}^3 that stays in the grid, columns ascending; 26 on the diagonal,
    -1 off the diagonal. Returns (rowptr int32, col int32, val float64).
    """
    n = m * m * m
    if (3 * m - 2) ** 3 >= 2 ** 31:  # nnz and columns are int32
        raise ValueError("grid too large for int32 CSR")
    rows = np.arange(n, dtype=np.int64)
    i = rows % m
    j = (rows // m) % m
    k = rows // (m * m)
    counts = np.zeros(n, dtype=np.int64)
    offs = []
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                offs.append((dk, dj, di))
    # lexicographic (dk, dj, di) with -1 < 0 < 1 is ascending column order
    valid = []
    for dk, dj, di in offs:
        ok = ((i + di >= 0) & (i + di < m) & (j + dj >= 0) & (j + dj < m)
              & (k + dk >= 0) & (k + dk < m))
        valid.append(ok)
        counts += ok
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    nnz = int(rowptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    pos = rowptr[:-1].copy()
    for (dk, dj, di), ok in zip(offs, valid):
        r = rows[ok]
        p = pos[ok]
        col[p] = (r + di + m * dj + m * m * dk).astype(np.int32)
        val[p] = 26.0 if (dk, dj, di) == (0, 0, 0) else -1.0
        pos[ok] += 1
    return rowptr.astype(np.int32), col, val


def cg_rhs(n: int, seed: int = 1) -> np.ndarray:
    return um11(seed, STREAM_CG_RHS, np.arange(n, dtype=np.uint64))


# --------------------------------------------------------------------------
# Histogram keys
# --------------------------------------------------------------------------

def hist_keys_uniform(n: int, seed: int = 1, chunk: int = 1 << 24, fast: bool = True) -> np.ndarray:
    lib = _fill_lib() if fast else None
    if lib is not None:
        keys = np.empty(n, dtype=np.uint32)
        lib.gfi_keys_u32(seed, STREAM_HIST, 0, n, keys.ctypes.data_as(ctypes.c_void_p))
        return keys
    keys = np.empty(n, dtype=np.uint32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        keys[s:e] = (hash_u64(seed, STREAM_HIST, np.arange(s, e, dtype=np.uint64)) >> _U64(32)).astype(np.uint32)
    return keys


def zipf_cdf(ranks: int = 65536, s: float = 1.1) -> np.ndarray:
    """CDF over ranks 1..ranks with P(r) proportional to r**-s, summed in increasing r."""
    w = np.arange(1, ranks + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    cdf = c / c[-1]
    cdf[-1] = 1.0
    return cdf


def hist_keys_zipf(n: int, seed: int = 1, ranks: int = 65536, s: float = 1.1,
                   chunk: int = 1 << 22, fast: bool = True) -> np.ndarray:
    """key = (rank-1) | (high 16 random bits << 16): bin (key mod 65536) = rank-1."""
    cdf = zipf_cdf(ranks, s)
    lib = _fill_lib() if fast else None
    if lib is not None:
        keys = np.empty(n, dtype=np.uint32)
        lib.gfi_keys_zipf(seed, STREAM_ZIPF, STREAM_HIST, n, cdf.ctypes.data_as(ctypes.c_void_p), ranks,
                          keys.ctypes.data_as(ctypes.c_void_p))
        return keys
    keys = np.empty(n, dtype=np.uint32)
    for st in range(0, n, chunk):
        e = min(n, st + chunk)
        idx = np.arange(st, e, dtype=np.uint64)
        r0 = np.searchsorted(cdf, u01(seed, STREAM_ZIPF, idx), side="left")
        np.minimum(r0, ranks - 1, out=r0)
        hi = (hash_u64(seed, STREAM_HIST, idx) >> _U64(48)).astype(np.uint32)
        keys[st:e] = r0.astype(np.uint32) | (hi << np.uint32(16))
    return keys


# --------------------------------------------------------------------------
# Batched instances
# --------------------------------------------------------------------------

def batched_sides(count: int = 256, seed: int = 1, lo: int = 64, hi: int = 2048) -> np.ndarray:
    """Log-uniform integer sides floor(lo * (hi/lo)**U), clamped to [lo, hi]."""
    u = u01(seed, STREAM_SIDES, np.arange(count, dtype=np.uint64))
    n = np.floor(lo * (float(hi) / lo) ** u).astype(np.int64)
    return np.clip(n, lo, hi)


def batched_grid(i: int, n: int, seed: int = 1) -> np.ndarray:
    return grid2d(n, seed, STREAM_INSTANCE0 + int(i))
