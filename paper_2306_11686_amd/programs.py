"""Step lists of the legacy loop programs (host-side descriptions only).

Each builder returns a Program whose slots follow the documented layout; the
caller binds device tensors to the slots with Instance.make. The programs
are the serial code of the initial thread with its `parallel for` regions
(paper, Section 2.1 and Section 3.3); reductions are OpenMP clauses on a
scalar variable that the preceding serial SET initialises.
"""
from __future__ import annotations

import math

from .binding import (GF_OP_MAX, GF_OP_NONE, GF_OP_SUM, GF_R_AXPBY, GF_R_DOT, GF_R_HIST, GF_R_JACOBI2D,
                      GF_R_JACOBI3D, GF_R_OWNER, GF_R_PHASES, GF_R_SPMV, GF_S_COPY, GF_S_DIV, GF_S_PRINTF,
                      GF_S_RECORD, GF_S_SET, GF_S_SQRT, GF_S_SWAP, GF_STEP_NOWAIT, Program, Step)

JACOBI2D_FORMAT = "sweep %d residual %.10e\n"

# slot layouts
J3_U, J3_W, J3_RES = 0, 1, 2          # arrays; scalar 0 = residual; ip[0] = n
J2_U, J2_W, J2_RES = 0, 1, 2          # arrays; scalars 0 = acc, 1 = residual; ip[0] = n
CG_ROWPTR, CG_COL, CG_VAL, CG_X, CG_R, CG_P, CG_Q, CG_RHO = range(8)
CG_S_RHO, CG_S_PQ, CG_S_ALPHA, CG_S_RHONEW, CG_S_BETA = range(5)


def jacobi3d(sweeps: int, reduce: bool = True) -> Program:
    """3D 7-point Jacobi: per sweep res = -inf; parallel for reduction(max:res);
    record res; swap(u, w)."""
    body = []
    if reduce:
        body.append(Step.make(GF_S_SET, sc=(0,), c=-math.inf))
    body.append(Step.make(GF_R_JACOBI3D, arr=(J3_U, J3_W), sc=(0,), red_op=GF_OP_MAX if reduce else GF_OP_NONE,
                          np=0))
    if reduce:
        body.append(Step.make(GF_S_RECORD, arr=(J3_RES,), sc=(0,)))
    body.append(Step.make(GF_S_SWAP, arr=(J3_U, J3_W)))
    return Program.make([], body, sweeps)


def jacobi2d(sweeps: int, fmt_id: int = -1, print_every: int = 10, blocking: bool = False) -> Program:
    """2D 5-point Jacobi: acc = 0; parallel for reduction(+:acc); res = sqrt(acc);
    record res; every `print_every` sweeps printf(fmt, sweep, res) via RPC; swap."""
    body = [
        Step.make(GF_S_SET, sc=(0,), c=0.0),
        Step.make(GF_R_JACOBI2D, arr=(J2_U, J2_W), sc=(0,), red_op=GF_OP_SUM, np=0),
        Step.make(GF_S_SQRT, sc=(1, 0)),
        Step.make(GF_S_RECORD, arr=(J2_RES,), sc=(1,)),
    ]
    if fmt_id >= 0 and print_every > 0:
        body.append(Step.make(GF_S_PRINTF, sc=(1,), every=print_every, fmt_id=fmt_id, nargs=2,
                              flags=1 if blocking else 0))
    body.append(Step.make(GF_S_SWAP, arr=(J2_U, J2_W)))
    return Program.make([], body, sweeps)


def cg(iters: int, nowait: bool = True) -> Program:
    """Conjugate gradients, every loop a separate region. The caller sets
    x = 0, r = b, p = b. rho_hist[k] = rho after iteration k.

    With `nowait`, the two axpby loops of the update drop their barriers, as
    an OpenMP author would mark them: x += alpha p touches nothing the next
    loop uses, and r -= alpha q shares its static schedule with the dot that
    reads r (each thread reads back only the elements it wrote)."""
    pro = [
        Step.make(GF_S_SET, sc=(CG_S_RHO,), c=0.0),
        Step.make(GF_R_DOT, arr=(CG_R, CG_R), sc=(CG_S_RHO,), red_op=GF_OP_SUM, np=0),
    ]
    return Program.make(pro, list(_cg_body(nowait)), iters)


def _cg_body(nowait: bool = True):
    nw = GF_STEP_NOWAIT if nowait else 0
    return [
        Step.make(GF_R_SPMV, arr=(CG_ROWPTR, CG_COL, CG_VAL, CG_P, CG_Q), np=0),
        Step.make(GF_S_SET, sc=(CG_S_PQ,), c=0.0),
        Step.make(GF_R_DOT, arr=(CG_P, CG_Q), sc=(CG_S_PQ,), red_op=GF_OP_SUM, np=0),
        Step.make(GF_S_DIV, sc=(CG_S_ALPHA, CG_S_RHO, CG_S_PQ)),
        Step.make(GF_R_AXPBY, arr=(CG_X, CG_X, CG_P), sc=(-1, CG_S_ALPHA), c=1.0, np=0, flags=nw),
        Step.make(GF_R_AXPBY, arr=(CG_R, CG_R, CG_Q), sc=(-1, CG_S_ALPHA), c=-1.0, np=0, flags=nw),
        Step.make(GF_S_SET, sc=(CG_S_RHONEW,), c=0.0),
        Step.make(GF_R_DOT, arr=(CG_R, CG_R), sc=(CG_S_RHONEW,), red_op=GF_OP_SUM, np=0),
        Step.make(GF_S_DIV, sc=(CG_S_BETA, CG_S_RHONEW, CG_S_RHO)),
        Step.make(GF_S_COPY, sc=(CG_S_RHO, CG_S_RHONEW)),
        Step.make(GF_R_AXPBY, arr=(CG_P, CG_R, CG_P), sc=(-1, CG_S_BETA), c=1.0, np=0),
        Step.make(GF_S_RECORD, arr=(CG_RHO,), sc=(CG_S_RHO,)),
    ]


def cg_iterations_only(iters: int, nowait: bool = True) -> Program:
    """The CG body without its prologue: continues from the state (x, r, p) and
    the scalar rho already held by the instance."""
    return Program.make([], list(_cg_body(nowait)), iters)


def histogram(nbins: int = 65536) -> Program:
    """One region: bins[key & (nbins-1)] += 1 (arrays 0 = keys, 1 = bins; ip[0] = n)."""
    if nbins & (nbins - 1):
        raise ValueError("nbins must be a power of two")
    return Program.make([Step.make(GF_R_HIST, arr=(0, 1), np=0, mask=nbins - 1)], [], 0)


def owner_map(chunk: int = 0) -> Program:
    """One schedule(static[,chunk]) region writing the executing global thread id."""
    return Program.make([Step.make(GF_R_OWNER, arr=(0,), np=0, chunk=chunk)], [], 0)


def phases(n_phases: int, shift: int, owner: bool = True) -> Program:
    """One `parallel` region with manual worksharing: each thread's block of
    [0, n) goes through n_phases producer/consumer phases separated by
    barriers across all workgroups (arrays 0 and 1 = the two buffers, 2 = the
    owner map when requested; ip[0] = n). The result is in array
    n_phases % 2."""
    return Program.make([Step.make(GF_R_PHASES, arr=(0, 1, 2 if owner else -1), np=0, chunk=n_phases,
                                   mask=shift)], [], 0)
