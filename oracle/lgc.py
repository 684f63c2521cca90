"""The local gradient constraint (LGC) of eq. (reg2_lgc), the cross-channel prior the paper compares LLP with
(Sec. II-D, Sec. IV): the same window penalty as eq. (reg2), once on the horizontal and once on the vertical
gradient of the band and of PAN instead of on their Laplacians.  FP64.  TEST INFRASTRUCTURE ONLY.

Minimising eq. (reg2_lgc) over the window coefficients (a^h, c^h) and (a^v, c^v) gives, by the same theorem as
for eq. (initialize_z_fast), (lambda/2) sum_d (G^d Z)^T M_{G^d Y} (G^d Z), d in {h, v}, M the matting matrix of
eq. (matting_matrix) with the gradient of PAN as the guide.  The per-band problem with this prior is therefore
(B^T D^T D B + lambda sum_d G^dT M_{G^d Y} G^d) Z = B^T D^T X, solved here by conjugate gradients.

Reading: G^h = Z (*) [-1 1] and G^v = Z (*) [-1 1]^T are periodic differences; which of the two taps sits at
offset 0 and the sign do not change G^T M_{G Y} G (a periodic shift S gives M_{S G Y} = S M_{G Y} S^T, and a sign
cancels in the product), so the forward difference z[j+1] - z[j] is used.
"""
from __future__ import annotations

import numpy as np

from .llp import Problem, _f64, apply_data, matting_apply, matting_stats


def grad_h(Z):
    """Horizontal difference Z[..., j+1] - Z[..., j] (periodic)."""
    Z = _f64(Z)
    return np.roll(Z, -1, axis=-1) - Z


def grad_h_adj(Y):
    Y = _f64(Y)
    return np.roll(Y, 1, axis=-1) - Y


def grad_v(Z):
    """Vertical difference Z[..., i+1, :] - Z[..., i, :] (periodic)."""
    Z = _f64(Z)
    return np.roll(Z, -1, axis=-2) - Z


def grad_v_adj(Y):
    Y = _f64(Y)
    return np.roll(Y, 1, axis=-2) - Y


DIRECTIONS = ((grad_h, grad_h_adj), (grad_v, grad_v_adj))


class LgcProblem(Problem):
    """A scene's operator data for the LGC prior: the data term of eq. (Z_ini_matting) and, per direction, the
    window statistics of PAN's gradient (the guide of that direction's matting matrix)."""

    def __post_init__(self):
        super().__post_init__()
        self.guides = [g(self.Y) for g, _ in DIRECTIONS]
        self.gstats = [matting_stats(G, self.r, self.eps) for G in self.guides]


def apply_lgc(Z, prob: LgcProblem):
    """lambda sum_d G^dT M_{G^d Y} G^d Z for every band of Z."""
    Z = _f64(Z)
    out = np.zeros_like(Z)
    for (g, gT), G, st in zip(DIRECTIONS, prob.guides, prob.gstats):
        for i in range(Z.shape[0]):
            out[i] += gT(matting_apply(G, g(Z[i]), prob.r, prob.eps, st))
    return prob.lam * out


def apply_A_lgc(Z, prob: LgcProblem):
    """The matrix of the per-band problem with the LGC prior applied to Z."""
    return apply_data(Z, prob) + apply_lgc(Z, prob)


def objective_lgc(Z, X, prob: LgcProblem):
    """Per band: 1/2 ||D B Z - X||^2 + lambda/2 sum_d (G^d Z)^T M_d (G^d Z)."""
    Z = _f64(Z)
    X = _f64(X)
    from .llp import blur, decimate
    res = decimate(blur(Z, prob.otf), prob.c) - X
    data = 0.5 * np.sum(res * res, axis=(-2, -1))
    reg = np.zeros(Z.shape[0])
    for (g, _), G, st in zip(DIRECTIONS, prob.guides, prob.gstats):
        for i in range(Z.shape[0]):
            l = g(Z[i])
            reg[i] += np.sum(l * matting_apply(G, l, prob.r, prob.eps, st))
    return data + 0.5 * prob.lam * reg


def cg_lgc(prob: LgcProblem, b, max_iters=50, tol=0.0):
    """Textbook conjugate gradients from Z = 0 on the LGC system, every band independently; stops a band when
    ||r|| <= tol ||b|| (recursive residual) or after max_iters.  Returns (z, iterations)."""
    b = _f64(b)
    N = b.shape[0]
    z = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = np.sum(r * r, axis=(-2, -1))
    bnorm = np.sqrt(np.sum(b * b, axis=(-2, -1)))
    active = np.ones(N, dtype=bool)
    iters = np.zeros(N, dtype=np.int64)
    for _ in range(max_iters):
        if not active.any():
            break
        idx = np.nonzero(active)[0]
        q = apply_A_lgc(p[idx], prob)
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
