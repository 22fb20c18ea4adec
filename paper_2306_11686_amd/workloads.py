"""Device inputs of the standard workloads (seeded, synthetic).

Each builder returns (program, instance or instances, tensors to keep
alive, reset callable or None). Sizes follow the workload names:
jacobi3d_512 (512^3, 200 sweeps), jacobi2d_256 (256^2, 100 sweeps, printf
every 10), cg_128 (27-point CSR on 128^3, 500 iterations), hist_2^28 (2^28
u32 keys, 65,536 bins), batched_256 (256 uneven 2D instances, 50 sweeps).
"""
from __future__ import annotations

import gf_inputs as gi

from . import programs
from .binding import Instance


def _torch():
    import torch
    return torch


def jacobi3d(n: int = 512, sweeps: int = 200, seed: int = 1):
    torch = _torch()
    u = torch.from_numpy(gi.grid3d(n, seed=seed)).cuda()
    w = u.clone()
    res = torch.zeros(max(1, sweeps), dtype=torch.float64, device="cuda")
    sc = torch.zeros(16, dtype=torch.float64, device="cuda")
    inst = Instance.make({programs.J3_U: u, programs.J3_W: w, programs.J3_RES: res}, sc, ip=(n,))
    return programs.jacobi3d(sweeps), inst, [u, w, res, sc], None


def jacobi2d(ctx=None, n: int = 256, sweeps: int = 100, seed: int = 1, printf: bool = True):
    torch = _torch()
    fmt = ctx.register_format(programs.JACOBI2D_FORMAT, "id") if (ctx is not None and printf) else -1
    u = torch.from_numpy(gi.grid2d(n, seed=seed)).cuda()
    w = u.clone()
    res = torch.zeros(sweeps, dtype=torch.float64, device="cuda")
    sc = torch.zeros(16, dtype=torch.float64, device="cuda")
    inst = Instance.make({programs.J2_U: u, programs.J2_W: w, programs.J2_RES: res}, sc, ip=(n,))
    return programs.jacobi2d(sweeps, fmt_id=fmt, print_every=10), inst, [u, w, res, sc], None


def cg(m: int = 128, iters: int = 500, seed: int = 1):
    torch = _torch()
    N = m ** 3
    rowptr, col, val = gi.poisson27_csr(m)
    b = torch.from_numpy(gi.cg_rhs(N, seed=seed)).cuda()
    t = {programs.CG_ROWPTR: torch.from_numpy(rowptr).cuda(), programs.CG_COL: torch.from_numpy(col).cuda(),
         programs.CG_VAL: torch.from_numpy(val).cuda(),
         programs.CG_X: torch.zeros(N, dtype=torch.float64, device="cuda"),
         programs.CG_R: b.clone(), programs.CG_P: b.clone(),
         programs.CG_Q: torch.zeros(N, dtype=torch.float64, device="cuda"),
         programs.CG_RHO: torch.zeros(iters, dtype=torch.float64, device="cuda")}
    sc = torch.zeros(16, dtype=torch.float64, device="cuda")
    inst = Instance.make(t, sc, ip=(N,))

    def reset():
        t[programs.CG_X].zero_()
        t[programs.CG_R].copy_(b)
        t[programs.CG_P].copy_(b)

    return programs.cg(iters), inst, list(t.values()) + [b, sc], reset


def histogram(n: int = 1 << 28, nbins: int = 65536, dist: str = "uniform", seed: int = 1):
    torch = _torch()
    keys = gi.hist_keys_uniform(n, seed=seed) if dist == "uniform" else gi.hist_keys_zipf(n, seed=seed)
    tk = torch.from_numpy(keys).cuda()
    del keys
    bins = torch.zeros(nbins, dtype=torch.int32, device="cuda")
    sc = torch.zeros(16, dtype=torch.float64, device="cuda")
    inst = Instance.make({0: tk, 1: bins}, sc, ip=(n,))
    return programs.histogram(nbins), inst, [tk, bins, sc], bins.zero_


def batched(count: int = 256, sweeps: int = 50, seed: int = 1):
    torch = _torch()
    sides = gi.batched_sides(count, seed=seed)
    insts, keep = [], []
    for i, n in enumerate(sides):
        n = int(n)
        u = torch.from_numpy(gi.batched_grid(i, n, seed)).cuda()
        w = u.clone()
        r = torch.zeros(sweeps, dtype=torch.float64, device="cuda")
        sc = torch.zeros(16, dtype=torch.float64, device="cuda")
        keep += [u, w, r, sc]
        insts.append(Instance.make({programs.J2_U: u, programs.J2_W: w, programs.J2_RES: r}, sc, ip=(n,)))
    return programs.jacobi2d(sweeps), insts, keep, None

