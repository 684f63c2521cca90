"""The last two steps of Algorithm "Fast Pansharpening" (Sec. III-B), after Z^0: the A, C step of
eq. (ac_h_compute) and the Z step of eq. (Z_solution).  FP64.  TEST INFRASTRUCTURE ONLY.

For every band i, with l = L Z^0_i and G = L Y (the Laplacians of the band's Z^0 and of PAN):

* A, C (eq. ac_h_compute): in every window w_j, a_j = (mean_j(G l) - mu_j pbar_j) / (sigma_j^2 + eps/|w|) and
  c_j = pbar_j - a_j mu_j, with mu_j, sigma_j^2 the mean and population variance of G and pbar_j the mean of l
  over w_j.  These are the (a, c) that minimise the window penalty of eq. (pansharp) for fixed Z.
* guided filter output: Lhat_k = (1/|w|) sum over the windows w_j that contain k of (a_j G_k + c_j).
* Z step (eq. Z_solution): Z = argmin 1/2 ||D B Z - X_i||^2 + (lambda_z / 2) ||L Z - Lhat||^2, solved through its
  normal equations (B^T D^T D B + lambda_z L^T L) Z = B^T D^T X_i + lambda_z L^T Lhat.  Every matrix in them is
  diagonal in the Fourier domain up to D's aliasing, so the system splits into one c^2 x c^2 block per
  low-resolution frequency (the groups of the module llp's preconditioner, with lambda mbar replaced by
  lambda_z); each block is solved directly.

Readings (the paper leaves these open; the design notes list them):
* eps/|w| in the slope's denominator (eq. ac_h_compute prints sigma^2 + eps): with it, (a_j, c_j) are exactly the
  window minimisers that make eq. (pansharp) equal eq. (initialize_z_fast) (Levin's theorem), so the A, C step
  and the matting matrix describe one objective;
* lambda_z = lambda |w| (eq. Z_solution prints lambda): eq. (pansharp) counts every pixel in |w| windows, and
  with (A, C) fixed it equals 1/2 ||D B Z - X||^2 + (lambda |w| / 2) ||L Z - Lhat||^2 plus terms free of Z.  With
  this weight the two steps are one round of exact alternating minimisation of eq. (pansharp): the objective does
  not increase, and the minimiser of eq. (initialize_z_fast) is a fixed point.
"""
from __future__ import annotations

import numpy as np

from .llp import Problem, _f64, laplacian, precond_apply, rhs, window_sum


def ac_coefficients(Z0, prob: Problem):
    """(A, C) of eq. (ac_h_compute) for every band of Z0: one (a_j, c_j) per window (per pixel j)."""
    Z0 = _f64(Z0)
    nw = (2 * prob.r + 1) ** 2
    G = prob.LY
    mu = window_sum(G, prob.r) / nw
    var = window_sum(G * G, prob.r) / nw - mu * mu
    den = var + prob.eps / nw
    A = np.empty_like(Z0)
    C = np.empty_like(Z0)
    for i in range(Z0.shape[0]):
        l = laplacian(Z0[i])
        pbar = window_sum(l, prob.r) / nw
        cov = window_sum(G * l, prob.r) / nw - mu * pbar
        a = np.zeros_like(cov)
        np.divide(cov, den, out=a, where=den != 0)  # a flat window with eps = 0 has no slope (pseudo-inverse)
        A[i] = a
        C[i] = pbar - a * mu
    return A, C


def guided_output(A, C, prob: Problem):
    """Lhat: at every pixel the mean, over the |w| windows that contain it, of a_j G + c_j."""
    nw = (2 * prob.r + 1) ** 2
    G = prob.LY
    return np.stack([(G * window_sum(a, prob.r) + window_sum(c, prob.r)) / nw for a, c in zip(_f64(A), _f64(C))])


def z_weight(prob: Problem):
    """lambda_z of the Z step: lambda |w| (see the module docstring)."""
    return prob.lam * (2 * prob.r + 1) ** 2


def z_step(X, Lhat, prob: Problem, lam_z=None):
    """eq. (Z_solution) for every band: the normal equations solved block by block in the Fourier domain."""
    lam_z = z_weight(prob) if lam_z is None else lam_z
    Lhat = _f64(Lhat)
    b = rhs(X, prob) + lam_z * np.stack([laplacian(x) for x in Lhat])
    # precond_apply solves (B^T D^T D B + lambda mbar L^T L) z = b per aliasing group: mbar = lam_z / lambda
    return precond_apply(b, prob, lam_z / prob.lam)


def polish(Z0, X, prob: Problem, lam_z=None):
    """One round of Algorithm "Fast Pansharpening" after Z^0: A, C, then the Z step.  Returns Z."""
    A, C = ac_coefficients(Z0, prob)
    return z_step(X, guided_output(A, C, prob), prob, lam_z)
