"""Blur-kernel estimation, Algorithm "Blur Kernel Estimation" (Sec. III-A, App. A): the spectral weights omega of
eq. (objective3), then generalized ADMM on eq. (u_solve) with the TGV^2 prior of eq. (reg1) and the simplex of
eq. (simplex).  FP64, host side.  TEST INFRASTRUCTURE ONLY (the GPU path takes the kernel u as an input).

Notation: u is the n x n kernel (n odd, centre tap u[R][R], R = (n-1)/2), handled as an n x n array; the
gradients and E(p) act on the n x n grid.  X' is the stack of LRMS bands that overlap PAN ([N'][h][w]), Y the PAN
image, c the resolution gap.

Readings (the paper leaves these open or prints them garbled; the design notes list them):
* gradients on the kernel grid are periodic forward differences, (D_h u)[i][j] = u[i][(j+1) mod n] - u[i][j] and
  (D_v u)[i][j] = u[(i+1) mod n][j] - u[i][j]: App. A diagonalises the blocks d_1..d_6 with the DFT, which holds
  for circulant differences only;
* the (u, p) step includes the coupling (mu_3 / 2) ||z - u - Lambda_3||^2 of eq. (Lagrangian) (u enters it), so
  d_1 gains mu_3 I and B_1 gains mu_3 (z - Lambda_3).  Without it the printed system is singular at frequency 0
  (d_1, d_4, d_5 all vanish there: the determinant is 0) and u would never see the data term;
* the x, y, z steps use u^t, p^t, Lambda^t; the (u, p) step uses the new x, y, z (Gauss-Seidel order, as
  Algorithm 1 lists the steps); App. A's row 1 prints d_1^T where d_4^T belongs (the block matrix is used);
* E(p)'s two middle columns are equal; the y and Lambda_2 columns 2 and 3 therefore stay equal, and the (u, p)
  step uses their mean (the exact minimiser in general);
* u_1 is the (2l+1) x (2l+1) box on the LR grid and u_2 the (cl+1) x (cl+1) box on the HR grid (the sizes their
  vector lengths state), both unit gain and centred; G is the (N'-1) x N' first-difference matrix;
* the start is u^0 = z^0 = the uniform kernel 1/n^2, p^0 = grad u^0, x^0 = y^0 = 0, Lambda^0 = 0; the returned
  kernel is z (the copy projected onto the simplex; u and z agree at convergence);
* the simplex projection [wang2013] is the sort-and-threshold algorithm.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .llp import _f64


# ----------------------------------------------------------------------------------------- small operators ---

def grad(u):
    """grad u = [D_h u, D_v u] (periodic forward differences on the n x n grid): shape [2][n][n]."""
    return np.stack([np.roll(u, -1, axis=1) - u, np.roll(u, -1, axis=0) - u])


def grad_adj(g):
    """The adjoint of grad: D_h^T g_0 + D_v^T g_1."""
    return (np.roll(g[0], 1, axis=1) - g[0]) + (np.roll(g[1], 1, axis=0) - g[1])


def sym_grad(p):
    """E(p) = [D_h p_1, (D_v p_1 + D_h p_2)/2, (D_v p_1 + D_h p_2)/2, D_v p_2] of eq. (reg1): shape [4][n][n]."""
    gh1 = np.roll(p[0], -1, axis=1) - p[0]
    gv1 = np.roll(p[0], -1, axis=0) - p[0]
    gh2 = np.roll(p[1], -1, axis=1) - p[1]
    gv2 = np.roll(p[1], -1, axis=0) - p[1]
    m = 0.5 * (gv1 + gh2)
    return np.stack([gh1, m, m, gv2])


def shrink2(e, t):
    """shrink_2 of eq. (x_update): max(||e||_2 - t, 0) e / ||e||_2 at every grid point (norm across axis 0)."""
    nrm = np.sqrt(np.sum(e * e, axis=0))
    scale = np.zeros_like(nrm)
    np.divide(np.maximum(nrm - t, 0.0), nrm, out=scale, where=nrm > 0)
    return e * scale


def project_simplex(v):
    """Euclidean projection of v (any shape) onto {s >= 0, sum s = 1} (eq. simplex): sort, find the threshold."""
    x = _f64(v).ravel()
    srt = np.sort(x)[::-1]
    css = np.cumsum(srt) - 1.0
    k = np.arange(1, x.size + 1)
    rho = np.nonzero(srt - css / k > 0)[0][-1]
    theta = css[rho] / (rho + 1.0)
    return np.maximum(x - theta, 0.0).reshape(np.shape(v))


def box_kernel(side):
    return np.full((side, side), 1.0 / (side * side))


def circ_conv(img, k):
    """Circular convolution of an image with a small odd kernel centred at offset 0 (as B(u) in Sec. II-A)."""
    n = k.shape[0]
    R = (n - 1) // 2
    out = np.zeros_like(img, dtype=np.float64)
    for a in range(-R, R + 1):
        for b in range(-R, R + 1):
            out += k[a + R, b + R] * np.roll(img, (a, b), axis=(0, 1))
    return out


def conv_matrix_E(Y, n, c):
    """E = D C(Y) (eq. z_solution): row (m, k) holds the PAN pixels that tap (a, b) of u multiplies to give
    (B(u) Y)[c m][c k], i.e. column (a + R) n + (b + R) is Y[(c m - a) mod H][(c k - b) mod W]."""
    R = (n - 1) // 2
    Y = _f64(Y)
    cols = [np.roll(Y, (a, b), axis=(0, 1))[::c, ::c].ravel() for a in range(-R, R + 1) for b in range(-R, R + 1)]
    return np.stack(cols, axis=1)


# ------------------------------------------------------------------------------------------- omega, eq. 3 ---

def estimate_omega(Xp, Y, c, l, lam_w):
    """omega of eq. (objective3): argmin 1/2 ||B(u_1) X' omega - D B(u_2) Y||^2 + lam_w/2 ||G omega||^2, in closed
    form through its normal equations."""
    Xp = _f64(Xp)
    Np = Xp.shape[0]
    M = np.stack([circ_conv(x, box_kernel(2 * l + 1)).ravel() for x in Xp], axis=1)
    v = circ_conv(_f64(Y), box_kernel(c * l + 1))[::c, ::c].ravel()
    G = np.zeros((Np - 1, Np))
    G[np.arange(Np - 1), np.arange(Np - 1)] = -1.0
    G[np.arange(Np - 1), np.arange(1, Np)] = 1.0
    return np.linalg.solve(M.T @ M + lam_w * G.T @ G, M.T @ v)


# ------------------------------------------------------------------------------------- (u, p) step, App. A ---

def _symbols(n):
    k = np.arange(n)
    sh = np.exp(2j * np.pi * k / n)[None, :] - 1.0  # DFT symbol of D_h (shift along columns)
    sv = np.exp(2j * np.pi * k / n)[:, None] - 1.0  # of D_v
    return np.broadcast_to(sh, (n, n)), np.broadcast_to(sv, (n, n))


def up_blocks(n, a1m1, a2m2, mu3):
    """The Fourier symbols of the blocks of eq. (block_toeplitz) (with the mu_3 coupling, see the readings):
    d1 .. d6 as n x n arrays, d_j^T having the conjugate symbol."""
    sh, sv = _symbols(n)
    ah, av = np.abs(sh) ** 2, np.abs(sv) ** 2
    d1 = a1m1 * (ah + av) + mu3
    d2 = a1m1 + a2m2 * ah + 0.5 * a2m2 * av
    d3 = a1m1 + 0.5 * a2m2 * ah + a2m2 * av
    d4 = -a1m1 * sh
    d5 = -a1m1 * sv
    d6 = 0.5 * a2m2 * np.conj(sh) * sv
    return d1, d2, d3, d4, d5, d6


def det3(a):
    """|.| of App. A for a 3 x 3 array of equally shaped arrays (element-wise)."""
    return (a[0][0] * a[1][1] * a[2][2] + a[0][1] * a[1][2] * a[2][0] + a[0][2] * a[1][0] * a[2][1]
            - a[0][2] * a[1][1] * a[2][0] - a[0][1] * a[1][0] * a[2][2] - a[0][0] * a[2][1] * a[1][2])


def up_solve(B1, B2, B3, a1m1, a2m2, mu3):
    """eq. (u_p_solution): the block system solved per frequency by Cramer's rule.  Returns (u, p1, p2)."""
    n = B1.shape[0]
    d1, d2, d3, d4, d5, d6 = up_blocks(n, a1m1, a2m2, mu3)
    F1, F2, F3 = np.fft.fft2(B1), np.fft.fft2(B2), np.fft.fft2(B3)
    Mx = [[d1, np.conj(d4), np.conj(d5)], [d4, d2, np.conj(d6)], [d5, d6, d3]]
    den = det3(Mx)
    rhs = [F1, F2, F3]
    out = []
    for col in range(3):
        Mc = [[rhs[i] if j == col else Mx[i][j] for j in range(3)] for i in range(3)]
        out.append(np.fft.ifft2(det3(Mc) / den).real)
    return out


def up_rhs(x, y, z, L1, L2, L3, a1m1, a2m2, mu3):
    """B_1, B_2, B_3 of App. A (B_1 with the mu_3 coupling; y_3, Lambda_{2,3}: means of the middle columns)."""
    y3 = 0.5 * (y[1] + y[2])
    l23 = 0.5 * (L2[1] + L2[2])

    def dhT(a):
        return np.roll(a, 1, axis=1) - a

    def dvT(a):
        return np.roll(a, 1, axis=0) - a

    B1 = a1m1 * (dhT(x[0] - L1[0]) + dvT(x[1] - L1[1])) + mu3 * (z - L3)
    B2 = a1m1 * (L1[0] - x[0]) + a2m2 * (dhT(y[0] - L2[0]) + dvT(y3 - l23))
    B3 = a1m1 * (L1[1] - x[1]) + a2m2 * (dvT(y[3] - L2[3]) + dhT(y3 - l23))
    return B1, B2, B3


# ---------------------------------------------------------------------------------------------- z step ---

def z_prepare(E, mu3):
    """The Cholesky factor of E^T E + mu_3 I (constant over the iterations)."""
    return np.linalg.cholesky(E.T @ E + mu3 * np.eye(E.shape[1]))


def z_update(chol, Etf, u, L3, mu3):
    """eq. (z_solution) then the simplex projection: returns (z, the unprojected solution), both n x n."""
    n = u.shape[0]
    zs = np.linalg.solve(chol.T, np.linalg.solve(chol, Etf + mu3 * (u + L3).ravel())).reshape(n, n)
    return project_simplex(zs), zs


# ------------------------------------------------------------------------------------------- Algorithm 1 ---

@dataclasses.dataclass
class TgvParams:
    n: int = 9           # kernel side
    l: int = 1           # box pre-blur size parameter of eq. (objective3)
    lam_w: float = 10.0  # the paper's values (Sec. IV-C)
    alpha1: float = 1.0
    alpha2: float = 0.006
    mu1: float = 100.0
    mu2: float = 100.0
    mu3: float = 100.0
    rho: float = 0.5
    t_max: int = 10000
    th: float = 1e-5


def estimate_kernel(Xp, Y, c, prm: TgvParams, omega=None):
    """Algorithm "Blur Kernel Estimation".  Returns (u, info): u the n x n kernel in the simplex."""
    Xp, Y = _f64(Xp), _f64(Y)
    n = prm.n
    if omega is None:
        omega = estimate_omega(Xp, Y, c, prm.l, prm.lam_w)
    f = np.tensordot(omega, Xp, axes=1).ravel()
    E = conv_matrix_E(Y, n, c)
    chol = z_prepare(E, prm.mu3)
    Etf = E.T @ f
    a1m1, a2m2 = prm.alpha1 * prm.mu1, prm.alpha2 * prm.mu2
    u = np.full((n, n), 1.0 / (n * n))
    z = u.copy()
    p = grad(u)
    x = np.zeros((2, n, n))
    y = np.zeros((4, n, n))
    L1, L2, L3 = np.zeros((2, n, n)), np.zeros((4, n, n)), np.zeros((n, n))
    t = 0
    for t in range(prm.t_max):
        x = shrink2(grad(u) - p + L1, 1.0 / prm.mu1)                                   # eq. (x_update)
        y = shrink2(sym_grad(p) + L2, 1.0 / prm.mu2)                                   # eq. (y_update)
        z, _ = z_update(chol, Etf, u, L3, prm.mu3)                                    # eq. (z_solution)
        B1, B2, B3 = up_rhs(x, y, z, L1, L2, L3, a1m1, a2m2, prm.mu3)
        u_new, p1, p2 = up_solve(B1, B2, B3, a1m1, a2m2, prm.mu3)                    # eq. (u_p_solution)
        p = np.stack([p1, p2])
        L1 = L1 + prm.rho * (grad(u_new) - p - x)
        L2 = L2 + prm.rho * (sym_grad(p) - y)
        L3 = L3 + prm.rho * (u_new - z)
        change = np.linalg.norm(u - u_new) / max(np.linalg.norm(u_new), 1e-300)
        u = u_new
        if change < prm.th:
            break
    return z, {"iters": t + 1, "omega": omega, "u": u}


def relative_kernel_error(U, Uhat):
    """eps_r of eq. (relative_error_kernel), in percent."""
    return 100.0 * np.linalg.norm(_f64(U) - _f64(Uhat)) / np.linalg.norm(_f64(U))
