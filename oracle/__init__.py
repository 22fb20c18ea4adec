"""Serial CPU oracle for the GPU-First legacy-loop hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package; the product library never does. It shares
no code with the HIP path. The loops live in plain C (``oracle.c``, built with
``-O2 -ffp-contract=off``); this module loads that library with ctypes and
adds the FP64 reference of the launch-config MLP in numpy.

Each legacy loop is executed exactly as the single initial thread of the
paper's execution model would run it (Section 2.1), the multi-team rewrite of
Section 3.3 only changing which thread runs which iteration. Reductions take
OpenMP clause semantics (the paper does not rewrite them, Section 4.3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no contraction, IEEE double)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SRC) > os.path.getmtime(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SRC) > os.path.getmtime(_SO):
        build(force=True)
    lib = ctypes.CDLL(_SO)
    P = ctypes.c_void_p
    I64, I32, U32, D = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    sig = {
        "or_jacobi2d": (ctypes.c_int, [I64, P, P, I32, P, P, I32, P, I64]),
        "or_jacobi3d": (ctypes.c_int, [I64, P, P, I32, P]),
        "or_spmv_csr": (None, [I64, P, P, P, P, P]),
        "or_dot": (D, [I64, P, P]),
        "or_dot_compensated": (D, [I64, P, P, P]),
        "or_axpby": (None, [I64, P, P, D, P]),
        "or_cg": (I32, [I64, P, P, P, P, P, I32, P, P, P, I32]),
        "or_cg_iteration": (I32, [I64, P, P, P, P, P, P, P, P, P, P, P]),
        "or_hist_u32": (None, [I64, P, P, U32]),
        "or_sum_f64": (D, [I64, P]),
        "or_sum_f64_compensated": (D, [I64, P]),
        "or_max_f64": (D, [I64, P]),
        "or_sum_u32": (ctypes.c_uint64, [I64, P]),
        "or_sum_u64": (ctypes.c_uint64, [I64, P]),
        "or_sum_i64": (ctypes.c_int64, [I64, P]),
        "or_max_u32": (ctypes.c_uint32, [I64, P]),
        "or_max_u64": (ctypes.c_uint64, [I64, P]),
        "or_max_i64": (ctypes.c_int64, [I64, P]),
        "or_static_owner": (None, [I64, I64, I64, P]),
        "or_phases": (None, [I64, P, P, I64, I64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _need(a, dtype):
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags.c_contiguous):
        raise TypeError(f"expected a C-contiguous {np.dtype(dtype)} array")
    return a


# ----------------------------------------------------------------------------
# Stencil programs
# ----------------------------------------------------------------------------

def jacobi2d(u0: np.ndarray, sweeps: int, print_every: int = 0):
    """Run the 2D Jacobi program. Returns (grid, res, res_compensated, text)."""
    u = np.array(u0, dtype=np.float64, order="C", copy=True)
    n = u.shape[0]
    w = u.copy()  # same zero boundary; interior is overwritten every sweep
    res = np.zeros(sweeps)
    resc = np.zeros(sweeps)
    cap = 64 * (sweeps // print_every + 1) if print_every > 0 else 1
    buf = ctypes.create_string_buffer(cap)
    which = _load().or_jacobi2d(n, _p(u), _p(w), sweeps, _p(res), _p(resc), print_every,
                                ctypes.cast(buf, ctypes.c_void_p), cap)
    return (u if which == 0 else w), res, resc, buf.value.decode()


def jacobi3d(u0: np.ndarray, sweeps: int):
    """Run the 3D Jacobi program. Returns (grid, res)."""
    u = np.array(u0, dtype=np.float64, order="C", copy=True)
    n = u.shape[0]
    w = u.copy()
    res = np.zeros(sweeps)
    which = _load().or_jacobi3d(n, _p(u), _p(w), sweeps, _p(res))
    return (u if which == 0 else w), res


def jacobi3d_inplace(u: np.ndarray, w: np.ndarray, sweeps: int):
    """As jacobi3d on caller buffers (no copies; for large grids). Returns (which, res)."""
    _need(u, np.float64)
    _need(w, np.float64)
    res = np.zeros(sweeps)
    which = _load().or_jacobi3d(u.shape[0], _p(u), _p(w), sweeps, _p(res))
    return which, res


# ----------------------------------------------------------------------------
# CG building blocks
# ----------------------------------------------------------------------------

def spmv(rowptr, col, val, x):
    _need(rowptr, np.int32); _need(col, np.int32); _need(val, np.float64); _need(x, np.float64)
    y = np.empty(rowptr.shape[0] - 1)
    _load().or_spmv_csr(y.shape[0], _p(rowptr), _p(col), _p(val), _p(x), _p(y))
    return y


def dot(a, b):
    _need(a, np.float64); _need(b, np.float64)
    return _load().or_dot(a.shape[0], _p(a), _p(b))


def dot_compensated(a, b):
    """Returns (compensated dot, sum of |a_i b_i|)."""
    _need(a, np.float64); _need(b, np.float64)
    s = ctypes.c_double(0.0)
    v = _load().or_dot_compensated(a.shape[0], _p(a), _p(b), ctypes.byref(s))
    return v, s.value


def axpby(x, s, y):
    _need(x, np.float64); _need(y, np.float64)
    out = np.empty_like(x)
    _load().or_axpby(x.shape[0], _p(out), _p(x), float(s), _p(y))
    return out


def cg(rowptr, col, val, b, iters: int, compensated: bool = False):
    """Returns (x, rho_hist, alpha_hist, beta_hist, iterations_done)."""
    _need(b, np.float64)
    n = b.shape[0]
    x = np.zeros(n)
    rh = np.zeros(iters); ah = np.zeros(iters); bh = np.zeros(iters)
    k = _load().or_cg(n, _p(rowptr), _p(col), _p(val), _p(b), _p(x), iters, _p(rh), _p(ah), _p(bh),
                      1 if compensated else 0)
    if k < 0:
        raise MemoryError("oracle CG could not allocate")
    return x, rh[:k], ah[:k], bh[:k], k


def cg_iteration(rowptr, col, val, x, r, p, rho):
    """One CG iteration from copies of (x, r, p, rho). Returns dict of the new state."""
    x = x.copy(); r = r.copy(); p = p.copy()
    q = np.empty_like(x)
    rho_c = ctypes.c_double(rho)
    pq = ctypes.c_double(0); al = ctypes.c_double(0); be = ctypes.c_double(0)
    brk = _load().or_cg_iteration(x.shape[0], _p(rowptr), _p(col), _p(val), _p(x), _p(r), _p(p), _p(q),
                                  ctypes.byref(rho_c), ctypes.byref(pq), ctypes.byref(al), ctypes.byref(be))
    return dict(x=x, r=r, p=p, q=q, rho=rho_c.value, pq=pq.value, alpha=al.value, beta=be.value,
                breakdown=bool(brk))


# ----------------------------------------------------------------------------
# Histogram, reductions, schedules
# ----------------------------------------------------------------------------

def hist_u32(keys, nbins: int = 65536, bins=None):
    _need(keys, np.uint32)
    if nbins & (nbins - 1):
        raise ValueError("nbins must be a power of two (bin = key & (nbins-1))")
    h = np.zeros(nbins, dtype=np.uint32) if bins is None else bins
    _load().or_hist_u32(keys.shape[0], _p(keys), _p(h), nbins - 1)
    return h


def reduce(op: str, x: np.ndarray, compensated: bool = False):
    lib = _load()
    x = np.ascontiguousarray(x)
    n = x.shape[0]
    dt = x.dtype
    if op == "sum":
        if dt == np.float64:
            return (lib.or_sum_f64_compensated if compensated else lib.or_sum_f64)(n, _p(x))
        return {np.dtype(np.uint32): lib.or_sum_u32, np.dtype(np.uint64): lib.or_sum_u64,
                np.dtype(np.int64): lib.or_sum_i64}[dt](n, _p(x))
    if op == "max":
        return {np.dtype(np.float64): lib.or_max_f64, np.dtype(np.uint32): lib.or_max_u32,
                np.dtype(np.uint64): lib.or_max_u64, np.dtype(np.int64): lib.or_max_i64}[dt](n, _p(x))
    raise ValueError(op)


def static_owner(n: int, nthreads: int, chunk: int = 0):
    owner = np.empty(n, dtype=np.int32)
    _load().or_static_owner(n, nthreads, chunk, _p(owner))
    return owner


def phases(a0: np.ndarray, phases: int, shift: int):
    """Producer/consumer phases (Section 3.3, manual worksharing with
    barriers): returns (a, b) after the phases; the result is in b after an
    odd number of phases, in a after an even one."""
    a = np.array(a0, dtype=np.float64, copy=True)
    b = np.zeros_like(a)
    _load().or_phases(a.size, _p(a), _p(b), phases, shift)
    return a, b


# ----------------------------------------------------------------------------
# Launch-config MLP (FP64 reference of the FP32 network)
# ----------------------------------------------------------------------------

def mlp_forward(params: dict, feats: np.ndarray):
    """8 -> H -> ReLU -> H -> ReLU -> K on float64 copies of the parameters.

    params: W1 (H,8), b1 (H,), W2 (H,H), b2 (H,), W3 (K,H), b3 (K,).
    Returns (y, cache) with the pre-activations needed by the backward pass.
    """
    f = np.asarray(feats, dtype=np.float64)
    W1, b1 = np.float64(params["W1"]), np.float64(params["b1"])
    W2, b2 = np.float64(params["W2"]), np.float64(params["b2"])
    W3, b3 = np.float64(params["W3"]), np.float64(params["b3"])
    z1 = f @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    y = a2 @ W3.T + b3
    return y, dict(f=f, z1=z1, a1=a1, z2=z2, a2=a2)


def mlp_loss(y: np.ndarray, target: np.ndarray, mask: np.ndarray) -> float:
    """Mean over measured entries (mask == 1) of the squared error."""
    m = np.asarray(mask, dtype=np.float64)
    d = (y - np.asarray(target, dtype=np.float64)) * m
    return float(np.sum(d * d) / np.sum(m))


def mlp_backward(params: dict, cache: dict, y, target, mask) -> dict:
    """Gradients of mlp_loss by the chain rule; relu'(0) = 0."""
    m = np.asarray(mask, dtype=np.float64)
    dy = 2.0 * (y - np.asarray(target, dtype=np.float64)) * m / np.sum(m)
    W2, W3 = np.float64(params["W2"]), np.float64(params["W3"])
    g = {}
    g["W3"] = dy.T @ cache["a2"]
    g["b3"] = dy.sum(axis=0)
    da2 = dy @ W3
    dz2 = da2 * (cache["z2"] > 0.0)
    g["W2"] = dz2.T @ cache["a1"]
    g["b2"] = dz2.sum(axis=0)
    da1 = dz2 @ W2
    dz1 = da1 * (cache["z1"] > 0.0)
    g["W1"] = dz1.T @ cache["f"]
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(param, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) in float64; returns (param, m, v)."""
    p = np.float64(param); g = np.float64(grad)
    m = beta1 * np.float64(m) + (1.0 - beta1) * g
    v = beta2 * np.float64(v) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
