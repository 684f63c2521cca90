"""Plain FP64 implementation of the learned warm start of the LLP solve.  TEST INFRASTRUCTURE ONLY.

The paper leaves the initial guess of the conjugate-gradient solve of eq. (Z_ini_matting) open (Sec. III-B).
The library can start it from a small convolutional network's estimate of each HRMS band; this module is the
reference for that network, its training gradients and its optimiser.  None of it is in the paper, so nothing
here is pinned to printed values: the pins are brute force, adjoint identities, finite differences and exact
properties of the interpolation (CPU test suite).

Estimate of band i (X_i the LRMS band, Y the PAN image, c the resolution gap):
    x_up = bicubic(X_i)                      Keys cubic convolution (a = -1/2), periodic, HR pixel c*m on LR m
    m, s = mean and population std of X_i;   m_Y, s_Y the same for Y (s = 1 where the std is 0)
    z0 = x_up + s * net([(x_up - m)/s, (Y - m_Y)/s_Y])
The network has five 3x3 convolution layers (2 -> 32 -> 32 -> 32 -> 32 -> 1 channels) with periodic padding,
ReLU after the first four.  Convolution is cross-correlation:
    out[o][i][j] = b[o] + sum_{c, dy, dx} W[o][c][dy][dx] * x[c][(i+dy-1) mod H][(j+dx-1) mod W].
Its reduced-precision form rounds every layer's input activations and weights to bfloat16 (round to nearest,
ties to even) and accumulates exactly (here: FP64); biases stay unrounded.  Training minimises the mean
squared error between the network output and t = (Z - x_up)/s, Z the plain solver's HRMS band, with Adam.
In the backward pass of the reduced-precision form, the gradient with respect to each layer's output is
rounded to bfloat16 before it enters the weight-gradient and input-gradient products (straight-through: the
roundings themselves count as the identity).
"""
from __future__ import annotations

import numpy as np

LAYERS = (2, 32, 32, 32, 32, 1)
KEYS_A = -0.5


def _f64(a):
    return np.asarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------------------------- bfloat16 ---

def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64 (via the float32 value)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    rounded = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------------------------- upsampling ---

def keys_weight(s):
    """Keys' cubic convolution kernel with a = -1/2 at offset s (in LR pixels)."""
    s = np.abs(_f64(s))
    a = KEYS_A
    w = np.zeros_like(s)
    inner = s <= 1.0
    outer = (s > 1.0) & (s < 2.0)
    w[inner] = (a + 2) * s[inner] ** 3 - (a + 3) * s[inner] ** 2 + 1.0
    w[outer] = a * s[outer] ** 3 - 5 * a * s[outer] ** 2 + 8 * a * s[outer] - 4 * a
    return w


def upsample_matrix(n, c):
    """The (c n) x n matrix of 1-D periodic cubic interpolation: HR sample i sits at LR coordinate i / c."""
    U = np.zeros((c * n, n))
    for i in range(c * n):
        m0 = i // c
        t = i / c - m0
        for k in (-1, 0, 1, 2):
            U[i, (m0 + k) % n] += keys_weight(k - t)
    return U


def bicubic(X, c):
    """Separable periodic bicubic upsampling of every band of X ([N][h][w] or [h][w]) by c."""
    X = _f64(X)
    h, w = X.shape[-2:]
    Uy, Ux = upsample_matrix(h, c), upsample_matrix(w, c)
    return Uy @ X @ Ux.T


# ------------------------------------------------------------------------------------------------ network ---

def conv3x3(x, W, b):
    """Periodic 3x3 cross-correlation: x [C][H][W], W [O][C][3][3], b [O] -> [O][H][W]."""
    x = _f64(x)
    out = np.zeros((W.shape[0],) + x.shape[1:])
    for dy in range(3):
        for dx in range(3):
            shifted = np.roll(x, shift=(1 - dy, 1 - dx), axis=(1, 2))  # shifted[c][i][j] = x[c][i+dy-1][j+dx-1]
            out += np.einsum("oc,chw->ohw", _f64(W[:, :, dy, dx]), shifted)
    return out + _f64(b)[:, None, None]


def conv3x3_adjoint(g, W):
    """Adjoint of conv3x3 in its input (bias excluded): g [O][H][W] -> [C][H][W]."""
    g = _f64(g)
    out = np.zeros((W.shape[1],) + g.shape[1:])
    for dy in range(3):
        for dx in range(3):
            t = np.einsum("oc,ohw->chw", _f64(W[:, :, dy, dx]), g)
            out += np.roll(t, shift=(dy - 1, dx - 1), axis=(1, 2))  # out[c][i][j] += t[c][i-dy+1][j-dx+1]
    return out


def conv3x3_weight_grad(g, x):
    """Gradient of <g, conv3x3(x, W, b)> with respect to W [O][C][3][3] and b [O]."""
    g, x = _f64(g), _f64(x)
    dW = np.zeros((g.shape[0], x.shape[0], 3, 3))
    for dy in range(3):
        for dx in range(3):
            shifted = np.roll(x, shift=(1 - dy, 1 - dx), axis=(1, 2))
            dW[:, :, dy, dx] = np.einsum("ohw,chw->oc", g, shifted)
    return dW, g.sum(axis=(1, 2))


def init_shapes(layers=LAYERS):
    return [((layers[k + 1], layers[k], 3, 3), (layers[k + 1],)) for k in range(len(layers) - 1)]


def flatten(params):
    """Parameters in the library's flat layout: for every layer its W [O][C][3][3], then its b [O]."""
    return np.concatenate([np.concatenate([_f64(W).ravel(), _f64(b).ravel()]) for W, b in params])


def unflatten(flat, layers=LAYERS):
    out, k = [], 0
    for ws, bs in init_shapes(layers):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((_f64(flat[k:k + nw]).reshape(ws), _f64(flat[k + nw:k + nw + nb]).reshape(bs)))
        k += nw + nb
    return out


def forward(params, inp, quantize=True):
    """Network output [1][H][W] for input planes inp [2][H][W]; also the per-layer (input, pre-activation)."""
    a = _f64(inp)
    cache = []
    for k, (W, b) in enumerate(params):
        a_in = bf16(a) if quantize else a
        Wq = bf16(W) if quantize else _f64(W)
        z = conv3x3(a_in, Wq, b)
        cache.append((a_in, Wq, z))
        a = np.maximum(z, 0.0) if k < len(params) - 1 else z
    return a, cache


def loss_and_grads(params, inp, target, quantize=True):
    """Mean squared error between forward(inp) and target [1][H][W], and its gradients (list of (dW, db))."""
    out, cache = forward(params, inp, quantize)
    P = out.size
    diff = out - _f64(target)
    loss = float(np.sum(diff * diff) / P)
    g = 2.0 * diff / P  # gradient with respect to the last layer's output
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        a_in, Wq, z = cache[k]
        if k < len(params) - 1:
            g = g * (z > 0)  # ReLU
        gq = bf16(g) if quantize else g
        grads[k] = conv3x3_weight_grad(gq, a_in)
        if k > 0:
            g = conv3x3_adjoint(gq, Wq)
    return loss, grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) of every parameter array; state = (t, [m], [v])."""
    t, m, v = state
    t += 1
    new_params, new_m, new_v = [], [], []
    flat_p = [a for pair in params for a in pair]
    flat_g = [a for pair in grads for a in pair]
    if not m:
        m = [np.zeros_like(_f64(p)) for p in flat_p]
        v = [np.zeros_like(_f64(p)) for p in flat_p]
    for p, g, mi, vi in zip(flat_p, flat_g, m, v):
        mi = beta1 * mi + (1 - beta1) * g
        vi = beta2 * vi + (1 - beta2) * g * g
        mhat = mi / (1 - beta1 ** t)
        vhat = vi / (1 - beta2 ** t)
        new_params.append(_f64(p) - lr * mhat / (np.sqrt(vhat) + eps))
        new_m.append(mi)
        new_v.append(vi)
    pairs = [(new_params[2 * k], new_params[2 * k + 1]) for k in range(len(params))]
    return pairs, (t, new_m, new_v)


# ------------------------------------------------------------------------------------------ warm start ---

def band_stats(a):
    a = _f64(a)
    m = float(a.mean())
    s = float(a.std())
    return m, (s if s > 0 else 1.0)


def net_input(Xi, Y, c):
    """Input planes [2][H][W] of band Xi, with its upsampled band and its (mean, std)."""
    x_up = bicubic(Xi, c)
    m, s = band_stats(Xi)
    mY, sY = band_stats(Y)
    return np.stack([(x_up - m) / s, (_f64(Y) - mY) / sY]), x_up, s


def warm_start(params, X, Y, c, quantize=True):
    """Initial HRMS estimate [N][H][W] for every band of X."""
    out = []
    for Xi in _f64(X):
        inp, x_up, s = net_input(Xi, Y, c)
        o, _ = forward(params, inp, quantize)
        out.append(x_up + s * o[0])
    return np.stack(out)


def training_target(Xi, Zi, c):
    """Target [1][H][W] of the network for band Xi whose plain-solver HRMS band is Zi."""
    x_up = bicubic(Xi, c)
    _, s = band_stats(Xi)
    return ((_f64(Zi) - x_up) / s)[None]
