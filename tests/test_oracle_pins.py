"""Pins of the CPU oracle against facts other than itself.

Closed forms (Jacobi eigenmodes, A*1 row classes), textbook special cases
(CG on tiny SPD systems, dense solves), hand-worked fixtures under
tests/golden/, brute force on tiny inputs, and invariants that a dropped
term, a wrong sign or index, or a transposed operand would break.
"""
import math
import os

import numpy as np
import pytest

import gf_inputs as gi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EPS = np.finfo(np.float64).eps


# ----------------------------------------------------------------------------
# Input generator (shared by both sides; pinned to the published SplitMix64)
# ----------------------------------------------------------------------------

def test_splitmix64_published_vectors():
    # SplitMix64 started at state 0: first three outputs as published with the
    # generator (Steele, Lea, Flood 2014; reference implementation outputs).
    seq = gi.splitmix64_sequence(0, 3)
    assert [int(x) for x in seq] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_u01_range_and_mean():
    x = gi.u01(1, 1, np.arange(1 << 18, dtype=np.uint64))
    assert x.min() >= 0.0 and x.max() < 1.0
    assert abs(x.mean() - 0.5) < 4.0 / math.sqrt(12 * x.size) * 3
    y = gi.um11(1, 2, np.arange(1 << 16, dtype=np.uint64))
    assert y.min() >= -1.0 and y.max() < 1.0


def test_grids_depend_only_on_position():
    g = gi.grid3d(9, seed=3)
    idx = 4 * 81 + 5 * 9 + 6
    assert g[4, 5, 6] == gi.u01(3, 1, np.array([idx], dtype=np.uint64))[0]
    assert np.all(g[0] == 0) and np.all(g[:, :, -1] == 0)
    g2 = gi.grid2d(7, seed=2)
    assert g2[3, 2] == gi.u01(2, 1, np.array([3 * 7 + 2], dtype=np.uint64))[0]


def test_compiled_fills_match_numpy_definition():
    gi.build(force=False)
    for n in (3, 8, 17):
        assert np.array_equal(gi.grid3d(n, seed=5), gi.grid3d(n, seed=5, fast=False))
    assert np.array_equal(gi.hist_keys_uniform(5000, seed=3), gi.hist_keys_uniform(5000, seed=3, fast=False))
    assert np.array_equal(gi.hist_keys_zipf(5000, seed=3), gi.hist_keys_zipf(5000, seed=3, fast=False))


def test_zipf_hottest_bin_mass():
    keys = gi.hist_keys_zipf(1 << 20, seed=1)
    H = np.sum(np.arange(1, 65537, dtype=np.float64) ** -1.1)
    frac = np.mean((keys & 0xFFFF) == 0)
    assert abs(frac - 1.0 / H) < 0.003  # 1/H = 0.1372..., sd ~ 3.4e-4


# ----------------------------------------------------------------------------
# 2D Jacobi
# ----------------------------------------------------------------------------

def _read_golden_jacobi():
    lines = [l.strip() for l in open(os.path.join(GOLDEN, "jacobi2d_4x4.txt")) if l.strip() and not l.startswith("#")]
    blocks, res = {}, {}
    i = 0
    while i < len(lines):
        tag = lines[i]
        if tag == "input" or tag.startswith("sweep"):
            blocks[tag] = np.array([[float(v) for v in lines[i + k].split()] for k in range(1, 5)])
            i += 5
        elif tag.startswith("residual"):
            res[len(res) + 1] = float(tag.split()[1])
            i += 1
        else:
            raise AssertionError(tag)
    return blocks, res


def test_jacobi2d_hand_worked_4x4(oracle_lib):
    blocks, res = _read_golden_jacobi()
    g1, r1, _, _ = oracle_lib.jacobi2d(blocks["input"], 1)
    assert np.array_equal(g1, blocks["sweep 1"])
    assert r1[0] == res[1]
    g2, r2, _, _ = oracle_lib.jacobi2d(blocks["input"], 2)
    assert np.array_equal(g2, blocks["sweep 2"])
    assert r2[1] == res[2]


@pytest.mark.parametrize("n,p,q,k", [(33, 1, 1, 40), (33, 3, 2, 25), (21, 17, 19, 12), (40, 1, 5, 30)])
def test_jacobi2d_eigenmode_closed_form(oracle_lib, n, p, q, k):
    # u0 = sin(p pi x) sin(q pi y) is an eigenvector of the 5-point Jacobi
    # operator: u_k = lam^k u0 with lam = (cos(p pi h) + cos(q pi h)) / 2, and
    # the update difference d_k = (lam - 1) lam^(k-1) u0.
    u0 = gi.eigenmode2d(n, p, q)
    h = 1.0 / (n - 1)
    lam = 0.5 * (math.cos(p * math.pi * h) + math.cos(q * math.pi * h))
    g, res, resc, _ = oracle_lib.jacobi2d(u0, k)
    assert np.max(np.abs(g - lam ** k * u0)) <= 8 * k * EPS * np.max(np.abs(u0))
    l2 = np.sqrt(np.sum(u0 * u0))
    expect = np.array([abs(1 - lam) * abs(lam) ** (s - 1) * l2 for s in range(1, k + 1)])
    assert np.allclose(res, expect, rtol=1e-9, atol=16 * k * EPS * l2)
    assert np.allclose(resc, res, rtol=1e-12)


def test_jacobi2d_zero_fixed_point_and_symmetry(oracle_lib):
    z = np.zeros((17, 17))
    g, res, _, _ = oracle_lib.jacobi2d(z, 3)
    assert np.all(g == 0) and np.all(res == 0)
    u0 = gi.grid2d(23, seed=5)
    g, res, _, _ = oracle_lib.jacobi2d(u0, 7)
    # the pairwise order ((W+E)+(S+N)) is invariant under transpose and
    # reflections, bit for bit
    gt, rest, _, _ = oracle_lib.jacobi2d(np.ascontiguousarray(u0.T), 7)
    assert np.array_equal(gt, g.T)
    gr, _, _, _ = oracle_lib.jacobi2d(np.ascontiguousarray(u0[:, ::-1]), 7)
    assert np.array_equal(gr, g[:, ::-1])
    assert np.allclose(rest, res, rtol=1e-13)


def test_jacobi2d_brute_force_small(oracle_lib):
    u0 = gi.grid2d(9, seed=2)
    u = u0.copy()
    for _ in range(3):
        v = u.copy()
        acc = []
        for j in range(1, 8):
            for i in range(1, 8):
                v[j, i] = ((u[j, i - 1] + u[j, i + 1]) + (u[j - 1, i] + u[j + 1, i])) * 0.25
                acc.append((v[j, i] - u[j, i]) ** 2)
        u = v
    g, res, _, _ = oracle_lib.jacobi2d(u0, 3)
    assert np.array_equal(g, u)
    assert abs(res[-1] - math.sqrt(math.fsum(acc))) <= 1e-14 * res[-1]


def test_jacobi2d_printf_text(oracle_lib):
    u0 = gi.grid2d(19, seed=1)
    _, res, _, text = oracle_lib.jacobi2d(u0, 30, print_every=10)
    lines = text.splitlines()
    assert [l.split()[1] for l in lines] == ["10", "20", "30"]
    for l, s in zip(lines, (10, 20, 30)):
        assert l == "sweep %d residual %.10e" % (s, res[s - 1])


# ----------------------------------------------------------------------------
# 3D Jacobi
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n,p,q,r,k", [(17, 1, 1, 1, 20), (20, 2, 3, 1, 15), (15, 13, 12, 11, 9)])
def test_jacobi3d_eigenmode_closed_form(oracle_lib, n, p, q, r, k):
    u0 = gi.eigenmode3d(n, p, q, r)
    h = 1.0 / (n - 1)
    lam = (math.cos(p * math.pi * h) + math.cos(q * math.pi * h) + math.cos(r * math.pi * h)) / 3.0
    g, res = oracle_lib.jacobi3d(u0, k)
    mx = np.max(np.abs(u0))
    assert np.max(np.abs(g - lam ** k * u0)) <= 10 * k * EPS * mx
    expect = np.array([abs(1 - lam) * abs(lam) ** (s - 1) * mx for s in range(1, k + 1)])
    assert np.allclose(res, expect, rtol=1e-9, atol=20 * k * EPS * mx)


def test_jacobi3d_brute_force_and_invariants(oracle_lib):
    u0 = gi.grid3d(7, seed=4)
    u = u0.copy()
    c6 = 1.0 / 6.0
    for _ in range(2):
        v = u.copy()
        m = -math.inf
        for z in range(1, 6):
            for y in range(1, 6):
                for x in range(1, 6):
                    v[z, y, x] = (((u[z, y, x - 1] + u[z, y, x + 1]) + (u[z, y - 1, x] + u[z, y + 1, x]))
                                  + (u[z - 1, y, x] + u[z + 1, y, x])) * c6
                    m = max(m, abs(v[z, y, x] - u[z, y, x]))
        u = v
    g, res = oracle_lib.jacobi3d(u0, 2)
    assert np.array_equal(g, u)
    assert res[-1] == m
    # x <-> y transpose keeps ((x)+(y))+(z) bit-exact
    gt, rt = oracle_lib.jacobi3d(np.ascontiguousarray(u0.transpose(0, 2, 1)), 2)
    assert np.array_equal(gt, g.transpose(0, 2, 1))
    assert np.array_equal(rt, res)
    z, rz = oracle_lib.jacobi3d(np.zeros((6, 6, 6)), 2)
    assert np.all(z == 0) and np.all(rz == 0)


# ----------------------------------------------------------------------------
# SpMV / 27-point matrix
# ----------------------------------------------------------------------------

def test_poisson27_structure_and_ones(oracle_lib):
    m = 5
    rowptr, col, val = gi.poisson27_csr(m)
    assert col.size == (3 * m - 2) ** 3
    y = oracle_lib.spmv(rowptr, col, val, np.ones(m ** 3))
    # A*1 = 26 - (#neighbours): interior 0, face 9, edge 15, corner 19
    idx = np.arange(m ** 3)
    i, j, k = idx % m, (idx // m) % m, idx // (m * m)
    nb = sum(((c == 0) | (c == m - 1)).astype(int) for c in (i, j, k))
    expect = np.choose(nb, [0.0, 9.0, 15.0, 19.0])
    assert np.array_equal(y, expect)


def test_poisson27_symmetric_and_affine(oracle_lib):
    m = 6
    rowptr, col, val = gi.poisson27_csr(m)
    n = m ** 3
    dense = np.zeros((n, n))
    for r in range(n):
        for kk in range(rowptr[r], rowptr[r + 1]):
            dense[r, col[kk]] = val[kk]
        assert np.all(np.diff(col[rowptr[r]:rowptr[r + 1]]) > 0)
    assert np.array_equal(dense, dense.T)
    idx = np.arange(n)
    i, j, k = idx % m, (idx // m) % m, idx // (m * m)
    x = 3.0 * i - 2.0 * j + 5.0 * k + 1.0  # affine: exact in double
    y = oracle_lib.spmv(rowptr, col, val, x)
    interior = (i > 0) & (i < m - 1) & (j > 0) & (j < m - 1) & (k > 0) & (k < m - 1)
    # sum over the 27-point neighbourhood of an affine function = 27 f(centre)
    assert np.all(y[interior] == 0.0)
    xr = gi.cg_rhs(n, seed=3)
    assert np.allclose(oracle_lib.spmv(rowptr, col, val, xr), dense @ xr, rtol=0, atol=1e-13)


# ----------------------------------------------------------------------------
# CG
# ----------------------------------------------------------------------------

def test_cg_textbook_2x2(oracle_lib):
    vals = {}
    for l in open(os.path.join(GOLDEN, "cg_2x2.txt")):
        if l.strip() and not l.startswith("#"):
            t = l.split()
            vals[t[0]] = [float(v) for v in t[1:]]
    rowptr = np.array([0, 2, 4], dtype=np.int32)
    col = np.array([0, 1, 0, 1], dtype=np.int32)
    val = np.array(vals["A"])
    b = np.array(vals["b"])
    x1, rh1, _, _, k1 = oracle_lib.cg(rowptr, col, val, b, 1)
    assert k1 == 1 and np.array_equal(x1, np.array(vals["x1"])) and rh1[0] == vals["rho1"][0]
    x2, _, _, _, _ = oracle_lib.cg(rowptr, col, val, b, 2)
    assert np.allclose(x2, vals["x2"], rtol=0, atol=4 * EPS)


@pytest.mark.parametrize("kdist", [1, 3, 5])
def test_cg_diagonal_k_distinct_eigenvalues(oracle_lib, kdist):
    n = 40
    d = np.array([1.0 + 2.0 * (i % kdist) for i in range(n)])
    rowptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    b = gi.cg_rhs(n, seed=2)
    x, rh, _, _, k = oracle_lib.cg(rowptr, col, d, b, kdist)
    assert np.allclose(x, b / d, rtol=0, atol=1e-13)


@pytest.mark.parametrize("m", [3, 4])
def test_cg_27pt_small_vs_dense_solve(oracle_lib, m):
    rowptr, col, val = gi.poisson27_csr(m)
    n = m ** 3
    dense = np.zeros((n, n))
    for r in range(n):
        dense[r, col[rowptr[r]:rowptr[r + 1]]] = val[rowptr[r]:rowptr[r + 1]]
    b = gi.cg_rhs(n, seed=1)
    xs = np.linalg.solve(dense, b)
    x, rh, _, _, k = oracle_lib.cg(rowptr, col, val, b, 2 * n)
    cond = np.linalg.cond(dense)
    assert np.max(np.abs(x - xs)) <= cond * 1e-14 * np.max(np.abs(xs))
    # A-norm of the error never increases along CG iterations (checked for
    # the first n iterations, where rounding has not yet reached the floor)
    errs = []
    for it in range(1, 12):
        xi, _, _, _, _ = oracle_lib.cg(rowptr, col, val, b, it)
        e = xi - xs
        errs.append(e @ dense @ e)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) + 1e-28 for i in range(len(errs) - 1))


def test_cg_iteration_matches_full_run(oracle_lib):
    rowptr, col, val = gi.poisson27_csr(6)
    b = gi.cg_rhs(216, seed=4)
    x_full, rh, ah, bh, _ = oracle_lib.cg(rowptr, col, val, b, 5)
    x = np.zeros(216); r = b.copy(); p = r.copy(); rho = oracle_lib.dot(r, r)
    for it in range(5):
        s = oracle_lib.cg_iteration(rowptr, col, val, x, r, p, rho)
        x, r, p, rho = s["x"], s["r"], s["p"], s["rho"]
        assert rho == rh[it] and s["alpha"] == ah[it] and s["beta"] == bh[it]
    assert np.array_equal(x, x_full)


def test_axpby_and_dot(oracle_lib):
    x = gi.cg_rhs(1000, seed=1); y = gi.cg_rhs(1000, seed=2)
    assert np.array_equal(oracle_lib.axpby(x, -0.375, y), x + (-0.375) * y)
    d, s = oracle_lib.dot_compensated(x, y)
    assert d == math.fsum((x * y).tolist())
    assert abs(oracle_lib.dot(x, y) - d) <= 1000 * EPS * s


# ----------------------------------------------------------------------------
# Reductions, histogram, schedule
# ----------------------------------------------------------------------------

def test_reductions_exact_cases(oracle_lib):
    n = 100003
    x = (np.arange(n) % 1024).astype(np.float64)  # integer-valued: exact in any order
    assert oracle_lib.reduce("sum", x) == float(sum(int(v) for v in (np.arange(n) % 1024)))
    r = gi.um11(1, 9, np.arange(n, dtype=np.uint64))
    assert oracle_lib.reduce("sum", r, compensated=True) == math.fsum(r.tolist())
    perm = np.random.default_rng(0).permutation(n).astype(np.float64)
    assert oracle_lib.reduce("max", perm) == n - 1
    u = (np.arange(n, dtype=np.uint64) * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)
    assert oracle_lib.reduce("sum", u.astype(np.uint32)) == int(sum(int(v) for v in u))
    assert oracle_lib.reduce("max", u.astype(np.uint32)) == int(u.max())
    i64 = np.arange(-n, n, 7, dtype=np.int64)
    assert oracle_lib.reduce("sum", i64) == int(sum(int(v) for v in i64))
    assert oracle_lib.reduce("max", i64) == int(i64.max())


def test_histogram_invariants(oracle_lib):
    n = 1 << 20
    keys = np.arange(n, dtype=np.uint32)
    h = oracle_lib.hist_u32(keys)
    assert np.all(h == n // 65536)
    eq = np.full(12345, 0xDEADBEEF, dtype=np.uint32)
    h = oracle_lib.hist_u32(eq)
    assert h[0xBEEF] == 12345 and h.sum() == 12345
    ku = gi.hist_keys_uniform(1 << 18, seed=2)
    h = oracle_lib.hist_u32(ku)
    assert np.array_equal(h, np.bincount(ku & 0xFFFF, minlength=65536).astype(np.uint32))
    assert int(h.sum()) == ku.size


@pytest.mark.parametrize("n,t,c", [(1000, 7, 0), (1000, 1000, 0), (5, 64, 0), (1003, 64, 3), (0, 8, 0), (4096, 256, 16)])
def test_static_schedule_invariants(oracle_lib, n, t, c):
    owner = oracle_lib.static_owner(n, t, c)
    if n == 0:
        return
    assert owner.min() >= 0 and owner.max() < t
    if c == 0:
        assert np.all(np.diff(owner) >= 0)  # contiguous blocks in thread order
        sizes = np.bincount(owner, minlength=t)
        assert sizes.max() - sizes.min() <= 1
        assert np.all(np.diff(sizes) <= 0)  # the first n % t threads get one more
    else:
        assert np.array_equal(owner, (np.arange(n) // c) % t)


# ----------------------------------------------------------------------------
# Launch-config MLP reference
# ----------------------------------------------------------------------------

def _mlp_params(rng, H=16, K=5):
    return {"W1": rng.standard_normal((H, 8)) * 0.5, "b1": rng.standard_normal(H) * 0.1,
            "W2": rng.standard_normal((H, H)) * 0.3, "b2": rng.standard_normal(H) * 0.1,
            "W3": rng.standard_normal((K, H)) * 0.3, "b3": rng.standard_normal(K) * 0.1}


def test_mlp_gradients_central_differences(oracle_lib):
    rng = np.random.default_rng(3)
    P = _mlp_params(rng)
    f = rng.standard_normal((6, 8))
    t = rng.standard_normal((6, 5))
    m = (rng.random((6, 5)) > 0.3).astype(np.float64)
    y, cache = oracle_lib.mlp_forward(P, f)
    assert np.min(np.abs(cache["z1"])) > 1e-3 and np.min(np.abs(cache["z2"])) > 1e-3
    g = oracle_lib.mlp_backward(P, cache, y, t, m)
    h = 1e-6
    for name in P:
        flat = P[name].reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[idx]
            flat[idx] = old + h
            lp = oracle_lib.mlp_loss(oracle_lib.mlp_forward(P, f)[0], t, m)
            flat[idx] = old - h
            lm = oracle_lib.mlp_loss(oracle_lib.mlp_forward(P, f)[0], t, m)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, idx, fd, an)


def test_mlp_closed_form_constant_output(oracle_lib):
    # W3 = 0 makes y = b3 for every sample: dL/db3 = 2 sum_b m (b3 - t) / sum m,
    # and nothing flows into the hidden layers.
    rng = np.random.default_rng(4)
    P = _mlp_params(rng)
    P["W3"][:] = 0.0
    f = rng.standard_normal((9, 8)); t = rng.standard_normal((9, 5))
    m = (rng.random((9, 5)) > 0.5).astype(np.float64)
    y, cache = oracle_lib.mlp_forward(P, f)
    assert np.array_equal(y, np.broadcast_to(P["b3"], y.shape))
    g = oracle_lib.mlp_backward(P, cache, y, t, m)
    assert np.allclose(g["b3"], 2 * np.sum(m * (P["b3"] - t), axis=0) / m.sum(), rtol=1e-14)
    for k in ("W1", "b1", "W2", "b2"):
        assert np.all(g[k] == 0.0)


def test_adam_first_step_closed_form(oracle_lib):
    # at t = 1 the bias corrections give mhat = g, vhat = g^2
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    p1, m1, v1 = oracle_lib.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_constant_gradient_moves_the_same_every_step(oracle_lib):
    # With g fixed, m_t = (1 - beta1^t) g and v_t = (1 - beta2^t) g^2, so the
    # bias-corrected moments are g and g^2 at every t and each step moves the
    # parameter by exactly -lr * g / (|g| + eps). Dropping the decayed previous
    # moment (beta1 * m or beta2 * v) or taking the correction at the wrong t
    # changes the step from t = 2 on.
    g = np.array([0.75, -3.0, 2e-4, 5.0])
    p = np.array([0.3, -1.0, 2.0, 0.0])
    m = np.zeros(4); v = np.zeros(4)
    step = 0.02 * g / (np.abs(g) + 1e-8)
    for t in range(1, 41):
        q, m, v = oracle_lib.adam_step(p, g, m, v, t, lr=0.02)
        assert np.allclose(p - q, step, rtol=1e-9, atol=0), t
        assert np.allclose(m, (1.0 - 0.9 ** t) * g, rtol=1e-12, atol=0)
        assert np.allclose(v, (1.0 - 0.999 ** t) * g * g, rtol=1e-12, atol=0)
        p = q


def test_adam_two_steps_worked_by_hand(oracle_lib):
    # Hand-worked, beta1 = 0.9, beta2 = 0.999, lr = 0.1, p0 = 0, g1 = 2, g2 = 1:
    #   t=1: m1 = 0.2, v1 = 0.004, mhat = 2, vhat = 4, p1 = -0.1 * 2 / (2 + eps)
    #   t=2: m2 = 0.9*0.2 + 0.1*1 = 0.28, v2 = 0.999*0.004 + 0.001*1 = 0.004996,
    #        mhat = 0.28 / 0.19 = 28/19, vhat = 0.004996 / 0.001999 = 4996/1999,
    #        p2 = p1 - 0.1 * (28/19) / (sqrt(4996/1999) + eps)
    #           = -0.0999999995 - 0.0932180... = -0.1932180...
    # The second coordinate takes the negated gradients and must mirror the first.
    eps = 1e-8
    p1, m1, v1 = oracle_lib.adam_step(np.zeros(2), np.array([2.0, -2.0]), np.zeros(2), np.zeros(2), 1, lr=0.1)
    assert abs(m1[0] - 0.2) < 1e-15 and abs(v1[0] - 0.004) < 1e-17
    p2, m2, v2 = oracle_lib.adam_step(p1, np.array([1.0, -1.0]), m1, v1, 2, lr=0.1)
    assert abs(m2[0] - 0.28) < 1e-15 and abs(v2[0] - 0.004996) < 1e-17
    want = -0.1 * 2.0 / (2.0 + eps) - 0.1 * (28.0 / 19.0) / (np.sqrt(4996.0 / 1999.0) + eps)
    assert abs(p2[0] - want) < 1e-14 and p2[1] == -p2[0] and m2[1] == -m2[0] and v2[1] == v2[0]
    assert abs(p2[0] - (-0.1932180)) < 1e-7


# ---------------------------------------------------------------------------
# Producer/consumer phases (manual worksharing with barriers, Section 3.3)
# ---------------------------------------------------------------------------

def _phase_result(a, b, phases):
    return b if phases % 2 else a


@pytest.mark.parametrize("n,phases,shift", [(10, 3, 4), (7, 5, 0), (13, 1, 12), (64, 6, 17)])
def test_phases_of_all_ones_double_every_phase(oracle_lib, n, phases, shift):
    a, b = oracle_lib.phases(np.ones(n), phases, shift)
    assert np.array_equal(_phase_result(a, b, phases), np.full(n, 2.0 ** phases))


@pytest.mark.parametrize("n,phases,shift,k", [(11, 4, 3, 5), (16, 5, 6, 0), (9, 3, 8, 8), (30, 6, 7, 29)])
def test_phases_of_a_unit_impulse_count_binomial_paths(oracle_lib, n, phases, shift, k):
    """Phase p adds the value s places ahead, so after P phases element i
    holds sum over m of C(P, m) * a0[(i + m*s) mod n]: with a unit impulse at
    k, the binomial weights of the m with i + m*s = k (mod n)."""
    import math
    a0 = np.zeros(n)
    a0[k] = 1.0
    a, b = oracle_lib.phases(a0, phases, shift)
    want = np.array([sum(math.comb(phases, m) for m in range(phases + 1) if (i + m * shift) % n == k)
                     for i in range(n)], dtype=np.float64)
    assert np.array_equal(_phase_result(a, b, phases), want)


def test_one_phase_adds_the_rotated_array(oracle_lib):
    rng = np.random.default_rng(3)
    a0 = rng.standard_normal(101)
    a, b = oracle_lib.phases(a0, 1, 37)
    assert np.array_equal(a, a0)                      # the source is only read
    assert np.array_equal(b, a0 + np.roll(a0, -37))  # b[i] = a[i] + a[(i + 37) % n]


def test_openmp_build_of_the_legacy_loop_matches_the_oracle(oracle_lib):
    """The CPU OpenMP build (a timing baseline) computes the same grid and
    residual as the serial oracle, bit for bit, on several threads."""
    import gf_inputs as gi
    from oracle import omp
    u0 = gi.grid3d(37, seed=5)
    g, r = oracle_lib.jacobi3d(u0, 3)
    u, w = u0.copy(), u0.copy()
    m = omp.jacobi3d(u, w, 3, threads=3)
    assert np.array_equal(w, g) and m == r[-1]
