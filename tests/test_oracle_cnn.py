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


def test_adam_constant_gradient_closed_form_over_steps():
    """With the same gradient g at every step, Adam's bias corrections make m_hat = g and v_hat = g^2 exactly
    (Kingma and Ba, Sec. 3), so every step moves a parameter by lr * g / (|g| + eps).  A wrong bias correction or
    moment update at t >= 2 breaks this."""
    r = rng(20)
    p0 = [(r.standard_normal((2, 1, 3, 3)), r.standard_normal(2))]
    g = [(r.standard_normal((2, 1, 3, 3)), r.standard_normal(2))]
    lr, eps = 3e-3, 1e-8
    params, state = p0, (0, [], [])
    for t in range(1, 6):
        params, state = cnn.adam_step(params, g, state, lr, eps=eps)
        assert state[0] == t
        for k in range(2):
            want = p0[0][k] - t * lr * g[0][k] / (np.abs(g[0][k]) + eps)
            np.testing.assert_allclose(params[0][k], want, rtol=0, atol=1e-13)


def test_adam_three_steps_hand_unrolled():
    """Three Adam steps on scalars, written out from the update rule: gradients 0.5, 0 (a zero-gradient step),
    -2.  Each moment and bias correction is evaluated by hand below."""
    lr, b1, b2, eps = 0.1, 0.9, 0.999, 1e-8
    params = [(np.array([1.0]), np.array([-3.0]))]
    gs = [0.5, 0.0, -2.0]
    state = (0, [], [])
    for gv in gs:
        params, state = cnn.adam_step(params, [(np.array([gv]), np.array([2 * gv]))], state, lr)
    # weight: g = 0.5, 0, -2
    m1, v1 = 0.1 * 0.5, 0.001 * 0.25
    x1 = 1.0 - lr * (m1 / 0.1) / (np.sqrt(v1 / 0.001) + eps)           # = 1 - 0.1 * 0.5/0.5
    m2, v2 = 0.9 * m1, 0.999 * v1
    x2 = x1 - lr * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.998001)) + eps)
    m3, v3 = 0.9 * m2 + 0.1 * (-2.0), 0.999 * v2 + 0.001 * 4.0
    x3 = x2 - lr * (m3 / (1 - 0.729)) / (np.sqrt(v3 / (1 - 0.997002999)) + eps)
    assert abs(x1 - 0.9) < 1e-8
    np.testing.assert_allclose(params[0][0], [x3], rtol=0, atol=1e-12)
    # bias: g = 1, 0, -4 (twice the weight's): Adam is invariant to a constant gradient scale up to eps
    c1 = -3.0 - lr * 1.0
    np.testing.assert_allclose(params[0][1], [c1 + (x3 - 0.9)], rtol=0, atol=1e-6)
    t, m, v = state
    assert t == 3
    np.testing.assert_allclose(m[0], [m3], rtol=1e-13)
    np.testing.assert_allclose(v[0], [v3], rtol=1e-13)


def test_band_stats_population_std_by_loop():
    """band_stats: mean and population standard deviation (divide by the count), 1 for a flat band."""
    r = rng(21)
    a = r.standard_normal((5, 7))
    vals = [float(v) for v in a.ravel()]
    mean = sum(vals) / len(vals)
    std = (sum((v - mean) ** 2 for v in vals) / len(vals)) ** 0.5
    m, s = cnn.band_stats(a)
    assert abs(m - mean) < 1e-14 and abs(s - std) < 1e-14
    # values 1..n: population variance (n^2 - 1)/12
    n = 12
    m, s = cnn.band_stats(np.arange(1, n + 1, dtype=float).reshape(3, 4))
    assert abs(m - 6.5) < 1e-14 and abs(s - np.sqrt((n * n - 1) / 12.0)) < 1e-14
    # a flat band has s = 1 (no division by zero)
    m, s = cnn.band_stats(np.full((4, 4), 0.25))
    assert m == 0.25 and s == 1.0
