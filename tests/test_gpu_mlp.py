"""GPU parity of the launch-config MLP kernels against the FP64 oracle.

Forward outputs and every gradient tensor must match the oracle (run in
float64 on the same float32 weights and inputs) to a relative Frobenius
error of 1e-5; fixtures reject draws with any |pre-activation| < 1e-3 so the
FP32 and FP64 ReLU masks agree. Adam matches the oracle's update; training
on the device lowers the loss; the host predictor equals the argmin of the
device forward pass.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

H, K, IN = 64, 32, 8
NP = H * IN + H + H * H + H + K * H + K


def _split(flat):
    o = 0
    out = {}
    for name, shape in (("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (K, H)), ("b3", (K,))):
        size = int(np.prod(shape))
        out[name] = flat[o:o + size].reshape(shape)
        o += size
    return out


def _fixture(batch, seed, max_tries=200):
    """float32 parameters and features whose pre-activations stay >= 1e-3 away
    from zero in float64."""
    rng = np.random.default_rng(seed)
    for _ in range(max_tries):
        flat = (rng.standard_normal(NP) * 0.2).astype(np.float32)
        f = rng.standard_normal((batch, IN)).astype(np.float32)
        P = _split(flat)
        y, cache = oracle.mlp_forward(P, f)
        if np.min(np.abs(cache["z1"])) > 1e-3 and np.min(np.abs(cache["z2"])) > 1e-3:
            return flat, f, P
    pytest.skip("no fixture without near-zero pre-activations")


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("batch", [1, 15, 37])
def test_forward_and_backward_match_fp64_oracle(gfx, batch):
    import torch
    flat, f, P = _fixture(batch, seed=batch)
    rng = np.random.default_rng(100 + batch)
    tgt = rng.standard_normal((batch, K)).astype(np.float32)
    mask = (rng.random((batch, K)) > 0.25).astype(np.float32)
    mask[0, 0] = 1.0
    dp = torch.from_numpy(flat).cuda()
    df = torch.from_numpy(f).cuda()
    y = torch.zeros(batch, K, device="cuda")
    z1 = torch.zeros(batch, H, device="cuda")
    z2 = torch.zeros(batch, H, device="cuda")
    gfx.mlp_forward(dp, df, batch, y, z1, z2)
    y_ref, cache = oracle.mlp_forward(P, f)
    torch.cuda.synchronize()
    assert _rel(y.cpu().numpy(), y_ref) <= 1e-5
    assert _rel(z1.cpu().numpy(), cache["z1"]) <= 1e-5
    assert _rel(z2.cpu().numpy(), cache["z2"]) <= 1e-5
    inv = 1.0 / float(mask.sum())
    g = torch.zeros(NP, device="cuda")
    gfx.mlp_backward(dp, df, z1, z2, y, torch.from_numpy(tgt).cuda(), torch.from_numpy(mask).cuda(), batch, inv, g)
    g_ref = oracle.mlp_backward(P, cache, y_ref, tgt, mask)
    gg = _split(g.cpu().numpy())
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert _rel(gg[name], g_ref[name]) <= 1e-5, name
    loss = torch.zeros(1, device="cuda")
    gfx.mlp_loss(y, torch.from_numpy(tgt).cuda(), torch.from_numpy(mask).cuda(), batch * K, inv, loss)
    assert abs(float(loss.cpu()[0]) - oracle.mlp_loss(y_ref, tgt, mask)) <= 1e-5 * oracle.mlp_loss(y_ref, tgt, mask)


def _plain_draw(batch, seed):
    """float32 parameters and features with no filter: determinism does not
    depend on the ReLU masks agreeing with a float64 evaluation."""
    rng = np.random.default_rng(seed)
    flat = (rng.standard_normal(NP) * 0.2).astype(np.float32)
    f = rng.standard_normal((batch, IN)).astype(np.float32)
    return flat, f


def test_backward_is_deterministic(gfx):
    import torch
    batch = 300
    flat, f = _plain_draw(batch, seed=3)
    tgt = np.random.default_rng(5).standard_normal((batch, K)).astype(np.float32)
    mask = np.ones((batch, K), np.float32)
    dp, df = torch.from_numpy(flat).cuda(), torch.from_numpy(f).cuda()
    y = torch.zeros(batch, K, device="cuda"); z1 = torch.zeros(batch, H, device="cuda"); z2 = torch.zeros_like(z1)
    gfx.mlp_forward(dp, df, batch, y, z1, z2)
    outs = []
    for _ in range(3):
        g = torch.zeros(NP, device="cuda")
        gfx.mlp_backward(dp, df, z1, z2, y, torch.from_numpy(tgt).cuda(), torch.from_numpy(mask).cuda(), batch,
                         1.0 / mask.sum(), g)
        outs.append(g.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])


def test_adam_matches_oracle(gfx):
    import torch
    rng = np.random.default_rng(9)
    p = rng.standard_normal(1000).astype(np.float32)
    m = np.zeros(1000, np.float32); v = np.zeros(1000, np.float32)
    dp, dm, dv = torch.from_numpy(p.copy()).cuda(), torch.from_numpy(m).cuda(), torch.from_numpy(v).cuda()
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in range(1, 6):
        g = rng.standard_normal(1000).astype(np.float32)
        gfx.adam_step(dp, torch.from_numpy(g).cuda(), dm, dv, 1000, 1e-2, 0.9, 0.999, 1e-8, t)
        pr, mr, vr = oracle.adam_step(pr, g, mr, vr, t, lr=1e-2)
    torch.cuda.synchronize()
    assert np.max(np.abs(dp.cpu().numpy() - pr)) <= 1e-5


def test_training_lowers_loss_and_host_predict_matches_device(gfx):
    import torch
    rng = np.random.default_rng(11)
    batch = 512
    f = rng.standard_normal((batch, IN)).astype(np.float32)
    # a smooth target the network can fit: per-candidate linear+abs features
    Wt = rng.standard_normal((K, IN)).astype(np.float32) * 0.5
    tgt = (np.abs(f @ Wt.T) + 0.1).astype(np.float32)
    mask = np.ones_like(tgt)
    flat = (rng.standard_normal(NP) * 0.1).astype(np.float32)
    dp = torch.from_numpy(flat).cuda()
    dm = torch.zeros(NP, device="cuda"); dv = torch.zeros(NP, device="cuda")
    hist = torch.zeros(300, device="cuda")
    gfx.train_predictor(dp, dm, dv, torch.from_numpy(f).cuda(), torch.from_numpy(tgt).cuda(),
                        torch.from_numpy(mask).cuda(), batch, 1.0 / mask.sum(), 300, 3e-3, hist)
    torch.cuda.synchronize()
    h = hist.cpu().numpy()
    assert np.all(np.isfinite(h)) and h[-1] < 0.5 * h[0]
    # host predictor (identity standardisation of log2(1+x) features)
    params = dp.cpu().numpy()
    raw = np.abs(rng.standard_normal((20, IN))) * 3
    z = np.log2(1.0 + raw)
    gfx.predictor_set(params, np.zeros(IN), np.ones(IN))
    y = torch.zeros(20, K, device="cuda")
    gfx.mlp_forward(dp, torch.from_numpy(z.astype(np.float32)).cuda(), 20, y)
    yd = y.cpu().numpy()
    for i in range(20):
        idx, scores = gfx.predict(raw[i], want_scores=True)
        assert np.allclose(scores, yd[i], rtol=1e-5, atol=1e-5)
        assert idx == int(np.argmin(scores))
    # out of distribution -> -1 (defer to the tuner)
    assert gfx.predict(np.full(IN, 1e9)) == -1
