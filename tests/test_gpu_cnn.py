"""GPU: the warm-start network (forward, gradients, Adam, the network start of the solve) against the oracle.

Bars.  The library and the oracle both round layer inputs and weights to bfloat16; the library accumulates in
FP32, the oracle exactly, and the bicubic input differs by FP32 rounding.  A rounding decision can therefore
flip by one bfloat16 step (2^-8 relative) where the two sums straddle a rounding boundary, which happens for a
small fraction of the activations.  The network output must match to relative L2 <= 2e-3, the estimate z0 to
1e-4, the loss to 1e-4 relative and each layer's weight and bias gradient to relative L2 <= 1e-2 (gradients
additionally pass through bfloat16 once per layer).  Adam's first step is exact up to FP32 rounding.
"""
import numpy as np
import pytest

from oracle import cnn
from paper_2103_09943_amd import binding as B
from paper_2103_09943_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def ctx(torch_dev):
    c = B.Context(0)
    yield c
    c.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def params_for(seed, last_std=0.05):
    return scenes.cnn_init_params(np.random.default_rng(np.random.SeedSequence([41, seed])), last_std=last_std)


def small_scene(seed, N=2, side=64, c=4, ragged=False):
    sc, _ = scenes.config_scene(2, seed, side=side)
    X, Y = sc.X[:N], sc.Y
    if ragged:  # W not a multiple of the 64-pixel tiles: crop to 96 columns
        X, Y = X[:, :, : 96 // c], Y[:, :96]
    return np.ascontiguousarray(X), np.ascontiguousarray(Y), sc


@pytest.mark.parametrize("ragged", [False, True])
def test_forward_matches_oracle(ctx, torch_dev, ragged):
    flat = params_for(1)
    ctx.cnn_set_weights(flat)
    X, Y, _ = small_scene(1, side=128, ragged=ragged)
    z0, out = ctx.cnn_warm_start(dev(torch_dev, X), dev(torch_dev, Y), 4, z0=True, net_out=True)
    params = cnn.unflatten(flat)
    for b in range(X.shape[0]):
        inp, x_up, s = cnn.net_input(X[b], Y, 4)
        want, _ = cnn.forward(params, inp, quantize=True)
        assert rel(host(out[b]), want[0]) < 2e-3
        assert rel(host(z0[b]), x_up + s * want[0]) < 1e-4


def test_weights_roundtrip_and_rejects_nonfinite(ctx, torch_dev):
    flat = params_for(2)
    ctx.cnn_set_weights(flat)
    np.testing.assert_array_equal(ctx.cnn_get_weights(), flat)
    bad = flat.copy()
    bad[100] = np.nan
    with pytest.raises(B.LlpError) as ei:
        ctx.cnn_set_weights(bad)
    assert ei.value.status == B.E_NONFINITE


def test_gradients_match_oracle(ctx, torch_dev):
    flat = params_for(3, last_std=0.1)
    ctx.cnn_set_weights(flat)
    X, Y, sc = small_scene(3, N=2, side=64)
    Z = sc.Z[:2]
    loss, g = ctx.cnn_loss_grad(dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, Z), 4)
    params = cnn.unflatten(flat)
    # the oracle's loss is the mean over the pixels of all bands of the scene
    tot_loss, tot = 0.0, None
    for b in range(2):
        inp, _, _ = cnn.net_input(X[b], Y, 4)
        t = cnn.training_target(X[b], Z[b], 4)
        lb, gb = cnn.loss_and_grads(params, inp, t, quantize=True)
        tot_loss += lb / 2
        gb = [(dW / 2, db / 2) for dW, db in gb]
        tot = gb if tot is None else [(a[0] + b_[0], a[1] + b_[1]) for a, b_ in zip(tot, gb)]
    assert abs(loss - tot_loss) <= 1e-4 * tot_loss
    got = cnn.unflatten(g)
    for k, ((gW, gb_), (wW, wb)) in enumerate(zip(got, tot)):
        assert rel(gW, wW) < 1e-2, (k, rel(gW, wW))
        assert rel(gb_, wb) < 1e-2, (k, rel(gb_, wb))


def test_adam_first_step(ctx, torch_dev):
    flat = params_for(4, last_std=0.1)
    ctx.cnn_set_weights(flat)
    X, Y, sc = small_scene(4, N=2, side=64)
    args = (dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, sc.Z[:2]), 4)
    _, g = ctx.cnn_loss_grad(*args)
    lr = 1e-3
    loss = ctx.cnn_train_step(*args, lr=lr)
    assert np.isfinite(loss)
    new = ctx.cnn_get_weights().astype(np.float64)
    want = flat.astype(np.float64) - lr * g / (np.abs(g.astype(np.float64)) + 1e-8)
    np.testing.assert_allclose(new, want, rtol=0, atol=2e-6)


def test_training_reduces_loss(ctx, torch_dev):
    flat = params_for(5, last_std=1e-3)
    ctx.cnn_set_weights(flat)
    X, Y, sc = small_scene(5, N=4, side=128)
    args = (dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, sc.Z[:4]), 4)
    first = ctx.cnn_train_step(*args, lr=2e-3)
    for _ in range(60):
        last = ctx.cnn_train_step(*args, lr=2e-3)
    assert last < 0.7 * first, (first, last)


def test_network_start_of_the_solve(ctx, torch_dev):
    """init_mode 2: the bands start from the network's estimate; the solve still reaches the tolerance."""
    flat = params_for(6, last_std=1e-3)
    ctx.cnn_set_weights(flat)
    sc, st = scenes.config_scene(2, 6, side=128)
    Xd, Yd, ud = dev(torch_dev, sc.X), dev(torch_dev, sc.Y), dev(torch_dev, sc.u)
    kw = dict(r=st.r, lam=st.lam, eps=st.eps, max_iters=5000, tol=1e-6)
    Zc, cold, _ = ctx.pansharpen(Xd, Yd, ud, **kw)
    Zw, warm, status = ctx.pansharpen(Xd, Yd, ud, init="cnn", **kw)
    assert status == B.OK
    assert all(r["init"] == B.INIT_NET for r in warm), warm
    assert all(r["init"] == B.INIT_ZERO for r in cold)
    assert all(r["true_rel_residual"] <= 1e-6 for r in warm)
    # the (nearly untrained) network's estimate is about the bicubic upsampling: a start closer than zero
    assert np.mean([w["iters"] for w in warm]) < np.mean([c["iters"] for c in cold])
    np.testing.assert_allclose([w["objective"] for w in warm], [c["objective"] for c in cold], rtol=1e-6)


def test_rejected_network_start_equals_cold_start(ctx, torch_dev):
    """A network whose estimate is worse than Z = 0 is rejected band by band: the solve is then the cold one,
    bit for bit."""
    flat = params_for(7, last_std=50.0)
    ctx.cnn_set_weights(flat)
    sc, st = scenes.config_scene(2, 7, side=96)
    Xd, Yd, ud = dev(torch_dev, sc.X), dev(torch_dev, sc.Y), dev(torch_dev, sc.u)
    kw = dict(r=st.r, lam=st.lam, eps=st.eps, max_iters=300, tol=1e-6)
    Zc, cold, _ = ctx.pansharpen(Xd, Yd, ud, **kw)
    Zw, warm, _ = ctx.pansharpen(Xd, Yd, ud, init="cnn", **kw)
    assert all(r["init"] == B.INIT_NET_REJECTED for r in warm), warm
    assert torch_dev.equal(Zc, Zw)
    for w, c in zip(warm, cold):
        w = dict(w)
        w["init"] = c["init"]
        assert w == c
    # without an iteration the report still gives the residual of the cold start, not the rejected one's
    kw["max_iters"] = 0
    _, cold0, _ = ctx.pansharpen(Xd, Yd, ud, **kw)
    _, warm0, _ = ctx.pansharpen(Xd, Yd, ud, init="cnn", **kw)
    assert all(r["true_rel_residual"] == pytest.approx(1.0, rel=1e-6) for r in cold0), cold0
    assert [r["true_rel_residual"] for r in warm0] == [r["true_rel_residual"] for r in cold0]


def test_batch_network_start_matches_single(ctx, torch_dev):
    flat = params_for(8, last_std=1e-3)
    ctx.cnn_set_weights(flat)
    host_sc = [scenes.config_scene(2, s, side=side)[0] for s, side in enumerate([96, 128, 64])]
    ds = [tuple(dev(torch_dev, a) for a in (sc.X, sc.Y, sc.u)) for sc in host_sc]
    kw = dict(r=1, lam=1e-2, eps=1e-3, max_iters=400, tol=1e-6)
    outs, reps, _ = ctx.pansharpen_batch(ds, inits="cnn", **kw)
    for (X, Y, u), Z, rs in zip(ds, outs, reps):
        Zs, rs_s, _ = ctx.pansharpen(X, Y, u, init="cnn", **kw)
        assert torch_dev.equal(Z, Zs) and rs == rs_s
        assert all(r["init"] in (B.INIT_NET, B.INIT_NET_REJECTED) for r in rs)


def test_adam_three_steps_match_oracle(ctx, torch_dev):
    """Three consecutive training steps against the oracle's Adam fed with the library's own gradient at each
    step (the moments and bias corrections past the first step)."""
    flat = params_for(9, last_std=0.1)
    ctx.cnn_set_weights(flat)
    X, Y, sc = small_scene(9, N=2, side=64)
    args = (dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, sc.Z[:2]), 4)
    lr = 1e-3
    params = cnn.unflatten(flat)
    state = (0, [], [])
    for step in range(3):
        _, g = ctx.cnn_loss_grad(*args)  # the gradient the next training step uses (deterministic)
        ctx.cnn_train_step(*args, lr=lr)
        params, state = cnn.adam_step(params, cnn.unflatten(g), state, lr)
        got = ctx.cnn_get_weights().astype(np.float64)
        want = cnn.flatten(params)
        # FP32 master weights and moments against FP64: each step moves a weight by at most about lr
        np.testing.assert_allclose(got, want, rtol=0, atol=3e-6 * (step + 1), err_msg=f"step {step + 1}")
        params = cnn.unflatten(got)  # continue from the library's FP32 weights


def test_gradients_match_oracle_at_training_size(ctx, torch_dev):
    """A 4-band 256 x 256 training scene: 1024 tiles of 4 x 64 pixels for the weight-gradient kernel's 512
    persistent workgroups, so every workgroup accumulates two tiles."""
    flat = params_for(10, last_std=0.1)
    ctx.cnn_set_weights(flat)
    sc, _ = scenes.config_scene(3, 10)
    X, Y, Z = sc.X, sc.Y, sc.Z
    assert X.shape == (4, 64, 64) and Y.shape == (256, 256)
    loss, g = ctx.cnn_loss_grad(dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, Z), 4)
    params = cnn.unflatten(flat)
    tot_loss, tot = 0.0, None
    for b in range(4):
        inp, _, _ = cnn.net_input(X[b], Y, 4)
        t = cnn.training_target(X[b], Z[b], 4)
        lb, gb = cnn.loss_and_grads(params, inp, t, quantize=True)
        tot_loss += lb / 4
        gb = [(dW / 4, db / 4) for dW, db in gb]
        tot = gb if tot is None else [(a[0] + b_[0], a[1] + b_[1]) for a, b_ in zip(tot, gb)]
    assert abs(loss - tot_loss) <= 1e-4 * tot_loss
    for k, ((gW, gb_), (wW, wb)) in enumerate(zip(cnn.unflatten(g), tot)):
        assert rel(gW, wW) < 1e-2, (k, rel(gW, wW))
        assert rel(gb_, wb) < 1e-2, (k, rel(gb_, wb))


def test_forward_matches_oracle_at_512(ctx, torch_dev):
    """The network's estimate on a held-out 512 x 512 band (the size of the warm-start evaluation scenes)."""
    flat = params_for(11)
    ctx.cnn_set_weights(flat)
    sc, _ = scenes.config_scene(3, 2000)
    X, Y = np.ascontiguousarray(sc.X[:1]), sc.Y
    z0, out = ctx.cnn_warm_start(dev(torch_dev, X), dev(torch_dev, Y), 4, z0=True, net_out=True)
    inp, x_up, s = cnn.net_input(X[0], Y, 4)
    want, _ = cnn.forward(cnn.unflatten(flat), inp, quantize=True)
    assert rel(host(out[0]), want[0]) < 2e-3
    assert rel(host(z0[0]), x_up + s * want[0]) < 1e-4
