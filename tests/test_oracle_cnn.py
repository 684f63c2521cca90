"""Pins of the warm-start network oracle (oracle.cnn) against brute force, exact identities, finite
differences and torch's own bfloat16 conversion.  The network is not in the paper: these pins fix its
arithmetic, not its usefulness."""
import numpy as np
import pytest

from oracle import cnn
from paper_2103_09943_amd import scenes


def rng(*key):
    return np.random.default_rng(np.random.SeedSequence([31, *key]))


# -------------------------------------------------------------------------------------------- bfloat16 ---

def test_bf16_rounding_known_values():
    e = 2.0 ** -8
    vals = np.array([1.0, 1 + e, 1 + 3 * e, -(1 + 3 * e), 1 + 1.5 * e, 3.0, 0.0, 2.0 ** -130])
    want = np.array([1.0, 1.0, 1 + 4 * e, -(1 + 4 * e), 1 + 2 * e, 3.0, 0.0, 2.0 ** -130])
    np.testing.assert_array_equal(cnn.bf16(vals), want)


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    x = rng(1).standard_normal(10000) * 10.0 ** rng(2).uniform(-6, 6, 10000)
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(x), want)


# ------------------------------------------------------------------------------------------ upsampling ---

@pytest.mark.parametrize("c", [2, 3, 4])
def test_bicubic_interpolates_lr_samples(c):
    X = rng(3, c).standard_normal((2, 6, 5))
    up = cnn.bicubic(X, c)
    np.testing.assert_allclose(up[:, ::c, ::c], X, atol=1e-14)


def test_bicubic_constant_and_quadratic():
    c = 4
    np.testing.assert_allclose(cnn.bicubic(np.full((8, 8), 2.5), c), 2.5, atol=1e-14)
    # Keys' kernel (a = -1/2) reproduces quadratics away from the periodic seam
    m = np.arange(16, dtype=float)
    q = 0.3 * m ** 2 - 1.1 * m + 0.7
    X = np.tile(q[:, None], (1, 16))
    up = cnn.bicubic(X, c)
    x = np.arange(16 * c) / c
    want = 0.3 * x ** 2 - 1.1 * x + 0.7
    inner = slice(2 * c, 13 * c)
    np.testing.assert_allclose(up[inner, 5], want[inner], atol=1e-12)


def test_keys_weights_partition_of_unity():
    for t in np.linspace(0, 1, 11):
        w = cnn.keys_weight(np.array([t + 1, t, 1 - t, 2 - t]))
        assert abs(w.sum() - 1.0) < 1e-14


# ---------------------------------------------------------------------------------------- convolution ---

def conv_brute(x, W, b):
    C, H, Wd = x.shape
    O = W.shape[0]
    out = np.zeros((O, H, Wd))
    for o in range(O):
        for i in range(H):
            for j in range(Wd):
                s = b[o]
                for c in range(C):
                    for dy in range(3):
                        for dx in range(3):
                            s += W[o, c, dy, dx] * x[c, (i + dy - 1) % H, (j + dx - 1) % Wd]
                out[o, i, j] = s
    return out


def test_conv_matches_brute_force():
    r = rng(4)
    x = r.standard_normal((3, 5, 7))
    W = r.standard_normal((2, 3, 3, 3))
    b = r.standard_normal(2)
    np.testing.assert_allclose(cnn.conv3x3(x, W, b), conv_brute(x, W, b), atol=1e-12)


def test_conv_adjoint_and_weight_grad_identities():
    r = rng(5)
    x = r.standard_normal((3, 6, 5))
    W = r.standard_normal((4, 3, 3, 3))
    g = r.standard_normal((4, 6, 5))
    lhs = np.sum(cnn.conv3x3(x, W, np.zeros(4)) * g)
    np.testing.assert_allclose(lhs, np.sum(x * cnn.conv3x3_adjoint(g, W)), rtol=1e-12)
    dW, db = cnn.conv3x3_weight_grad(g, x)
    np.testing.assert_allclose(lhs, np.sum(dW * W), rtol=1e-12)  # <g, conv(x, W)> is linear in W
    np.testing.assert_allclose(db, g.sum(axis=(1, 2)), rtol=1e-12)


def test_gradients_match_finite_differences():
    layers = (2, 3, 3, 1)
    r = rng(6)
    params = [(r.standard_normal(ws) * 0.5, r.standard_normal(bs) * 0.1) for ws, bs in cnn.init_shapes(layers)]
    inp = r.standard_normal((2, 6, 7))
    target = r.standard_normal((1, 6, 7))
    _, grads = cnn.loss_and_grads(params, inp, target, quantize=False)
    h = 1e-6
    for k, (W, b) in enumerate(params):
        for arr, garr in ((W, grads[k][0]), (b, grads[k][1])):
            flat = arr.reshape(-1)
            for idx in r.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp, _ = cnn.loss_and_grads(params, inp, target, quantize=False)
                flat[idx] = old - h
                lm, _ = cnn.loss_and_grads(params, inp, target, quantize=False)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - garr.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd)


def test_quantised_forward_rounds_inputs_and_weights():
    """With bfloat16-exact inputs and weights the reduced-precision forward equals the exact one."""
    layers = (2, 3, 1)
    r = rng(7)
    params = [(cnn.bf16(r.standard_normal(ws)), r.standard_normal(bs)) for ws, bs in cnn.init_shapes(layers)]
    inp = cnn.bf16(r.standard_normal((2, 5, 5)))
    out_q, cache = cnn.forward(params, inp, quantize=True)
    out_e, _ = cnn.forward(params, inp, quantize=False)
    # the first layer sees identical operands; the second its rounded input
    np.testing.assert_array_equal(cache[0][2], cnn.conv3x3(inp, params[0][0], params[0][1]))
    h = np.maximum(cache[0][2], 0)
    np.testing.assert_allclose(out_q, cnn.conv3x3(cnn.bf16(h), params[1][0], params[1][1]), atol=1e-12)
    assert np.max(np.abs(out_q - out_e)) <= 2.0 ** -7 * np.max(np.abs(out_e)) * 10


def test_adam_first_step_closed_form():
    r = rng(8)
    params = [(r.standard_normal((2, 2, 3, 3)), r.standard_normal(2))]
    grads = [(r.standard_normal((2, 2, 3, 3)), r.standard_normal(2))]
    lr, eps = 1e-2, 1e-8
    new, state = cnn.adam_step(params, grads, (0, [], []), lr, eps=eps)
    for (p, q), (g, _) in zip([(params[0][0], new[0][0]), (params[0][1], new[0][1])], [(grads[0][0], 0),
                                                                                      (grads[0][1], 0)]):
        np.testing.assert_allclose(q, p - lr * g / (np.abs(g) + eps), rtol=1e-12)
    assert state[0] == 1


def test_flat_layout_roundtrip_and_size():
    flat = scenes.cnn_init_params(rng(9))
    assert flat.size == 28641  # 2*32*9+32 + 3*(32*32*9+32) + 32*9+1
    params = cnn.unflatten(flat)
    np.testing.assert_array_equal(cnn.flatten(params), flat.astype(np.float64))


def test_warm_start_with_zero_last_layer_is_bicubic():
    flat = scenes.cnn_init_params(rng(10), last_std=0.0)
    params = cnn.unflatten(flat)
    X = rng(11).standard_normal((2, 6, 6))
    Y = rng(12).uniform(0, 1, (24, 24))
    z0 = cnn.warm_start(params, X, Y, 4)
    np.testing.assert_allclose(z0, cnn.bicubic(X, 4), atol=1e-14)


def test_training_target_inverts_warm_start():
    r = rng(13)
    X = r.standard_normal((6, 6))
    Z = r.standard_normal((24, 24))
    t = cnn.training_target(X, Z, 4)
    _, s = cnn.band_stats(X)
    np.testing.assert_allclose(cnn.bicubic(X, 4) + s * t[0], Z, atol=1e-12)
