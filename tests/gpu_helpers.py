"""Helpers shared by the GPU parity tests: device tensors and program runs
through the C ABI (paper_2306_11686_amd binding)."""
from __future__ import annotations

import math

import numpy as np


def torch_mod():
    import torch
    return torch


def dev(a: np.ndarray):
    """Copy a numpy array to a new device tensor (synchronous)."""
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t) -> np.ndarray:
    torch = torch_mod()
    torch.cuda.synchronize()
    return t.cpu().numpy()


def scalars(init=None):
    torch = torch_mod()
    s = torch.zeros(16, dtype=torch.float64, device="cuda")
    if init:
        for k, v in init.items():
            s[k] = v
    return s


def run_jacobi3d(ctx, u0: np.ndarray, sweeps: int, mode: int, launch=None, reduce=True):
    """Run the 3D program; returns (final grid, residual history, stats)."""
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    torch = torch_mod()
    n = u0.shape[0]
    u = dev(u0)
    w = u.clone()
    res = torch.zeros(max(1, sweeps), dtype=torch.float64, device="cuda")
    sc = scalars()
    prog = programs.jacobi3d(sweeps, reduce=reduce)
    inst = gf.Instance.make({programs.J3_U: u, programs.J3_W: w, programs.J3_RES: res}, sc, ip=(n,))
    stats = ctx.run(prog, inst, mode=mode, launch=launch)
    ctx.sync()
    final = u if sweeps % 2 == 0 else w
    return host(final), host(res)[:sweeps], stats


def run_jacobi2d(ctx, u0: np.ndarray, sweeps: int, mode: int, launch=None, fmt_id=-1, print_every=10,
                 blocking=False):
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import programs
    torch = torch_mod()
    n = u0.shape[0]
    u = dev(u0)
    w = u.clone()
    res = torch.zeros(max(1, sweeps), dtype=torch.float64, device="cuda")
    sc = scalars()
    prog = programs.jacobi2d(sweeps, fmt_id=fmt_id, print_every=print_every, blocking=blocking)
    inst = gf.Instance.make({programs.J2_U: u, programs.J2_W: w, programs.J2_RES: res}, sc, ip=(n,))
    stats = ctx.run(prog, inst, mode=mode, launch=launch)
    ctx.sync()
    final = u if sweeps % 2 == 0 else w
    return host(final), host(res)[:sweeps], stats


def rel_sum_ok(gpu: float, ref: float, abs_sum: float, tol: float = 1e-12) -> bool:
    """|gpu - ref| <= tol * sum |terms| (the order-of-summation tolerance)."""
    if abs_sum == 0.0:
        return gpu == ref
    return abs(gpu - ref) <= tol * abs_sum


def isclose_rel(a, b, tol=1e-12):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.all(np.abs(a - b) <= tol * np.maximum(np.abs(b), math.ulp(1.0) * 0))
