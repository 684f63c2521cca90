"""Brute-force twins used to pin the oracle on tiny inputs.

Everything here is written from the definitions with explicit loops and dense matrices, independently of
oracle/: circular convolution as a double sum with modular indices, decimation as a selection matrix, the
Laplacian from its 3x3 stencil, the matting matrix assembled entry by entry from eq. (matting_matrix), and the
window penalty of eq. (pansharp_penalty) minimised by a per-window least-squares solve.
"""
from __future__ import annotations

import numpy as np

S_STENCIL = np.array([[0.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 0.0]])


def conv_direct(z, u):
    """(B z)[i, j] = sum_{a,b} u[a+R][b+R] z[(i-a) mod H][(j-b) mod W], by loops."""
    H, W = z.shape
    n = u.shape[0]
    R = (n - 1) // 2
    out = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            s = 0.0
            for a in range(-R, R + 1):
                for b in range(-R, R + 1):
                    s += u[a + R, b + R] * z[(i - a) % H, (j - b) % W]
            out[i, j] = s
    return out


def conv_matrix(u, H, W):
    """HW x HW matrix of circular convolution by u (row-major pixel index i*W + j)."""
    n = u.shape[0]
    R = (n - 1) // 2
    B = np.zeros((H * W, H * W))
    for i in range(H):
        for j in range(W):
            for a in range(-R, R + 1):
                for b in range(-R, R + 1):
                    B[i * W + j, ((i - a) % H) * W + (j - b) % W] += u[a + R, b + R]
    return B


def decimation_matrix(H, W, c):
    """hw x HW selection matrix keeping pixels (c*m, c*k)."""
    h, w = H // c, W // c
    D = np.zeros((h * w, H * W))
    for m in range(h):
        for k in range(w):
            D[m * w + k, (c * m) * W + c * k] = 1.0
    return D


def laplacian_matrix(H, W):
    """HW x HW matrix of periodic convolution by the 3x3 stencil S."""
    L = np.zeros((H * W, H * W))
    for i in range(H):
        for j in range(W):
            for a in range(-1, 2):
                for b in range(-1, 2):
                    L[i * W + j, ((i - a) % H) * W + (j - b) % W] += S_STENCIL[a + 1, b + 1]
    return L


def window_pixels(k_i, k_j, r, H, W):
    return [((k_i + dy) % H) * W + (k_j + dx) % W for dy in range(-r, r + 1) for dx in range(-r, r + 1)]


def window_sum_naive(A, r):
    H, W = A.shape
    flat = A.reshape(-1)
    out = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            out[i, j] = sum(flat[p] for p in window_pixels(i, j, r, H, W))
    return out


def matting_matrix_dense(I, r, eps):
    """Eq. (matting_matrix) assembled literally: sum over windows k containing both m and n of
    delta_mn - (1/|w|) (1 + (I_m - mu_k)(I_n - mu_k) / (eps/|w| + sigma_k^2))."""
    H, W = I.shape
    flat = I.reshape(-1)
    nw = (2 * r + 1) ** 2
    M = np.zeros((H * W, H * W))
    for ki in range(H):
        for kj in range(W):
            pix = window_pixels(ki, kj, r, H, W)
            vals = flat[pix]
            mu = vals.mean()
            var = ((vals - mu) ** 2).mean()
            den = eps / nw + var
            for a, m in enumerate(pix):
                for b, n in enumerate(pix):
                    slope = (vals[a] - mu) * (vals[b] - mu) / den if den != 0 else 0.0
                    M[m, n] += (1.0 if m == n else 0.0) - (1.0 + slope) / nw
    return M


def levin_penalty(alpha, I, r, eps):
    """min over (a_k, c_k) of sum_k [ sum_{i in w_k} (alpha_i - a_k I_i - c_k)^2 + eps a_k^2 ], each window solved
    as a least-squares problem with the regulariser as one extra row (sqrt(eps), 0)."""
    H, W = I.shape
    af, If = alpha.reshape(-1), I.reshape(-1)
    total = 0.0
    for ki in range(H):
        for kj in range(W):
            pix = window_pixels(ki, kj, r, H, W)
            Amat = np.column_stack([If[pix], np.ones(len(pix))])
            rhs = af[pix].copy()
            Amat = np.vstack([Amat, [np.sqrt(eps), 0.0]])
            rhs = np.append(rhs, 0.0)
            coef, *_ = np.linalg.lstsq(Amat, rhs, rcond=None)
            res = Amat @ coef - rhs
            total += float(res @ res)
    return total


def dense_system(u, c, Y, r, lam, eps):
    """Dense A = B^T D^T D B + lambda L^T M_LY L and the dense D B, from explicit matrices."""
    H, W = Y.shape
    B = conv_matrix(u, H, W)
    D = decimation_matrix(H, W, c)
    L = laplacian_matrix(H, W)
    LY = (L @ Y.reshape(-1)).reshape(H, W)
    M = matting_matrix_dense(LY, r, eps)
    DB = D @ B
    return DB.T @ DB + lam * L.T @ M @ L, DB
