"""The cross-channel priors the paper compares in Sec. IV (Table "cross_channel_prior"): every one of them is the
window penalty of eq. (reg2) with the Laplacian replaced by one or two other filters.  FP64.  TEST
INFRASTRUCTURE ONLY.

For a set of filters F_1..F_m (circular convolutions), minimising the window penalty over the per-window
coefficients gives, by the same theorem as for eq. (initialize_z_fast), the quadratic
(lambda/2) sum_d (F_d Z)^T M_{F_d Y} (F_d Z), so the per-band problem is
(B^T D^T D B + lambda sum_d F_d^T M_{F_d Y} F_d) Z = B^T D^T X.  The filters, as the paper defines them:

* LLP: the 5-point Laplacian S of eq. (reg2);
* LGC: the horizontal and vertical gradients of eq. (reg2_lgc) (two filters);
* LPP: the identity (the pixels themselves);
* LPF: the blur kernel u;
* HPF: delta - u.

A filter is an odd square tap array with the kernel convention of the data term (centre tap at offset 0,
true convolution).  The LGC gradient [-1 1] is read as the forward difference z[j+1] - z[j]; the orientation
does not change F^T M_{F Y} F (see oracle/lgc.py, which states the same operator with explicit differences).
"""
from __future__ import annotations

import numpy as np

from .llp import Problem, _f64, apply_data, blur, blur_adjoint, decimate, kernel_otf, matting_apply, matting_stats

KINDS = ("llp", "lgc", "lpp", "lpf", "hpf")


def prior_filters(kind, u):
    """The tap arrays of a prior (Sec. IV, cross-channel prior comparison; eq. reg2, eq. reg2_lgc)."""
    u = _f64(u)
    if kind == "llp":
        return [np.array([[0.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 0.0]])]
    if kind == "lgc":
        gh = np.zeros((3, 3))
        gh[1, 0], gh[1, 1] = 1.0, -1.0  # tap at offset (0, -1): z[i][j+1] - z[i][j]
        gv = np.zeros((3, 3))
        gv[0, 1], gv[1, 1] = 1.0, -1.0  # tap at offset (-1, 0): z[i+1][j] - z[i][j]
        return [gh, gv]
    if kind == "lpp":
        return [np.ones((1, 1))]
    if kind == "lpf":
        return [u.copy()]
    if kind == "hpf":
        f = -u.copy()
        R = (u.shape[0] - 1) // 2
        f[R, R] += 1.0
        return [f]
    raise ValueError(f"unknown prior {kind!r}")


class PriorProblem(Problem):
    """A scene's operator data under one of the priors: the data term of eq. (Z_ini_matting) and, per filter,
    the filter's spectrum, the guide F_d Y and its window statistics."""

    def __init__(self, kind, **kw):
        self.kind = kind
        super().__init__(**kw)

    def __post_init__(self):
        super().__post_init__()
        self.filters = prior_filters(self.kind, self.u)
        self.fotf = [kernel_otf(f, self.H, self.W) for f in self.filters]
        self.guides = [blur(self.Y, o) for o in self.fotf]
        self.gstats = [matting_stats(G, self.r, self.eps) for G in self.guides]


def apply_prior(Z, prob: PriorProblem):
    """lambda sum_d F_d^T M_{F_d Y} F_d Z for every band of Z."""
    Z = _f64(Z)
    out = np.zeros_like(Z)
    for o, G, st in zip(prob.fotf, prob.guides, prob.gstats):
        L = blur(Z, o)
        ML = np.stack([matting_apply(G, L[i], prob.r, prob.eps, st) for i in range(Z.shape[0])])
        out += blur_adjoint(ML, o)
    return prob.lam * out


def apply_A_prior(Z, prob: PriorProblem):
    return apply_data(Z, prob) + apply_prior(Z, prob)


def objective_prior(Z, X, prob: PriorProblem):
    """Per band: 1/2 ||D B Z - X||^2 + lambda/2 sum_d (F_d Z)^T M_d (F_d Z)."""
    Z = _f64(Z)
    res = decimate(blur(Z, prob.otf), prob.c) - _f64(X)
    val = 0.5 * np.sum(res * res, axis=(-2, -1))
    for o, G, st in zip(prob.fotf, prob.guides, prob.gstats):
        L = blur(Z, o)
        for i in range(Z.shape[0]):
            val[i] += 0.5 * prob.lam * np.sum(L[i] * matting_apply(G, L[i], prob.r, prob.eps, st))
    return val


def cg_prior(prob: PriorProblem, b, z0=None, max_iters=50, tol=0.0):
    """Textbook conjugate gradients on the prior's system, every band independently, from z0 (default 0);
    stops a band when ||r|| <= tol ||b|| (recursive residual) or after max_iters.  Returns (z, iterations)."""
    b = _f64(b)
    N = b.shape[0]
    z = np.zeros_like(b) if z0 is None else _f64(z0).copy()
    r = b - apply_A_prior(z, prob) if z0 is not None else b.copy()
    p = r.copy()
    rho = np.sum(r * r, axis=(-2, -1))
    bnorm = np.sqrt(np.sum(b * b, axis=(-2, -1)))
    active = np.ones(N, dtype=bool)
    if tol > 0:
        active &= np.sqrt(rho) > tol * bnorm
    iters = np.zeros(N, dtype=np.int64)
    for _ in range(max_iters):
        if not active.any():
            break
        idx = np.nonzero(active)[0]
        q = apply_A_prior(p[idx], prob)
        alpha = rho[idx] / np.sum(p[idx] * q, axis=(-2, -1))
        z[idx] += alpha[:, None, None] * p[idx]
        r[idx] -= alpha[:, None, None] * q
        iters[idx] += 1
        rho_new = np.sum(r[idx] * r[idx], axis=(-2, -1))
        p[idx] = r[idx] + (rho_new / rho[idx])[:, None, None] * p[idx]
        rho[idx] = rho_new
        if tol > 0:
            active[idx[np.sqrt(rho_new) <= tol * bnorm[idx]]] = False
    return z, iters
