"""Pins of oracle.polish (the A, C step of eq. (ac_h_compute) and the Z step of eq. (Z_solution), Sec. III-B)
against brute force and identities that do not reuse its code:

* (a_j, c_j) against a per-window least-squares solve with the regulariser as an extra row;
* the guided-filter output against l - (M l)/|w| with M assembled entry by entry from eq. (matting_matrix);
* the Z step against a dense least-squares solve of the stacked system [D B; sqrt(lambda_z) L] Z = [X; ...];
* one round does not increase eq. (pansharp) (computed with per-window least squares), and the exact minimiser
  of eq. (initialize_z_fast) (dense Cholesky) is its fixed point.
"""
import numpy as np
import pytest

import naive
import oracle
from oracle import polish
from oracle.llp import Problem

CASES = [  # H, W, c, n, r, lam, eps
    (8, 8, 2, 3, 1, 0.1, 1e-3),
    (12, 12, 3, 5, 1, 1e-2, 1e-2),
    (8, 12, 4, 5, 1, 0.05, 1e-3),
    (10, 10, 2, 3, 2, 0.2, 0.1),
    (6, 6, 1, 3, 1, 0.3, 1e-3),
]


def rng_for(*key):
    return np.random.default_rng(np.random.SeedSequence([31, *key]))


def case_data(H, W, c, n, r, lam, eps, N=2):
    rng = rng_for(H, W, c, n, r)
    u = rng.uniform(0, 1, (n, n))
    u /= u.sum()
    Y = rng.uniform(0, 1, (H, W))
    X = rng.standard_normal((N, H // c, W // c))
    Z0 = rng.standard_normal((N, H, W))
    return u, Y, X, Z0, Problem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)


def window_ls(l, G, r, eps):
    """Per window j: argmin over (a, c) of sum_{k in w_j} (l_k - a G_k - c)^2 + eps a^2 (lstsq, extra row)."""
    H, W = G.shape
    lf, Gf = l.reshape(-1), G.reshape(-1)
    a = np.zeros((H, W))
    cc = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            pix = naive.window_pixels(i, j, r, H, W)
            M = np.vstack([np.column_stack([Gf[pix], np.ones(len(pix))]), [np.sqrt(eps), 0.0]])
            coef, *_ = np.linalg.lstsq(M, np.append(lf[pix], 0.0), rcond=None)
            a[i, j], cc[i, j] = coef
    return a, cc


def pansharp_objective(Z, X, u, c, Y, r, lam, eps):
    """eq. (pansharp) with (A, C) minimised out window by window, from explicit matrices."""
    H, W = Y.shape
    B = naive.conv_matrix(u, H, W)
    D = naive.decimation_matrix(H, W, c)
    L = naive.laplacian_matrix(H, W)
    G = (L @ Y.reshape(-1)).reshape(H, W)
    out = []
    for z, x in zip(Z, X):
        res = D @ B @ z.reshape(-1) - x.reshape(-1)
        l = (L @ z.reshape(-1)).reshape(H, W)
        out.append(0.5 * float(res @ res) + 0.5 * lam * naive.levin_penalty(l, G, r, eps))
    return np.array(out)


@pytest.mark.parametrize("case", CASES)
def test_ac_coefficients_are_window_least_squares(case):
    H, W, c, n, r, lam, eps = case
    u, Y, X, Z0, prob = case_data(*case)
    A, C = polish.ac_coefficients(Z0, prob)
    L = naive.laplacian_matrix(H, W)
    G = (L @ Y.reshape(-1)).reshape(H, W)
    for i in range(Z0.shape[0]):
        l = (L @ Z0[i].reshape(-1)).reshape(H, W)
        a, cc = window_ls(l, G, r, eps)
        np.testing.assert_allclose(A[i], a, rtol=1e-9, atol=1e-9 * np.abs(a).max())
        np.testing.assert_allclose(C[i], cc, rtol=1e-9, atol=1e-9 * np.abs(cc).max())


@pytest.mark.parametrize("case", CASES)
def test_guided_output_is_l_minus_M_l_over_w(case):
    H, W, c, n, r, lam, eps = case
    u, Y, X, Z0, prob = case_data(*case)
    Lhat = polish.guided_output(*polish.ac_coefficients(Z0, prob), prob)
    L = naive.laplacian_matrix(H, W)
    G = (L @ Y.reshape(-1)).reshape(H, W)
    M = naive.matting_matrix_dense(G, r, eps)
    nw = (2 * r + 1) ** 2
    for i in range(Z0.shape[0]):
        l = L @ Z0[i].reshape(-1)
        np.testing.assert_allclose(Lhat[i].reshape(-1), l - M @ l / nw, atol=1e-10 * np.abs(l).max())


@pytest.mark.parametrize("case", CASES)
def test_z_step_is_dense_least_squares(case):
    H, W, c, n, r, lam, eps = case
    u, Y, X, Z0, prob = case_data(*case)
    rng = rng_for(99, H, W, c, n, r)
    Lhat = rng.standard_normal(Z0.shape)
    lam_z = polish.z_weight(prob)
    got = polish.z_step(X, Lhat, prob)
    B = naive.conv_matrix(u, H, W)
    D = naive.decimation_matrix(H, W, c)
    L = naive.laplacian_matrix(H, W)
    K = np.vstack([D @ B, np.sqrt(lam_z) * L])
    for i in range(X.shape[0]):
        want, *_ = np.linalg.lstsq(K, np.concatenate([X[i].reshape(-1), np.sqrt(lam_z) * Lhat[i].reshape(-1)]),
                                   rcond=None)
        np.testing.assert_allclose(got[i].reshape(-1), want, atol=1e-9 * np.abs(want).max())


@pytest.mark.parametrize("case", CASES)
def test_polish_does_not_increase_pansharp_objective(case):
    """Exact alternating minimisation of eq. (pansharp): with lambda_z = lambda |w| the round cannot increase it.
    A round with the printed weight lambda is not such a minimisation; the pin would catch that reading."""
    H, W, c, n, r, lam, eps = case
    u, Y, X, Z0, prob = case_data(*case)
    Z1 = polish.polish(Z0, X, prob)
    f0 = pansharp_objective(Z0, X, u, c, Y, r, lam, eps)
    f1 = pansharp_objective(Z1, X, u, c, Y, r, lam, eps)
    assert np.all(f1 <= f0 * (1 + 1e-12)), (f0, f1)
    assert np.all(f1 < f0)  # a random Z0 is far from the minimiser: a strict decrease
    # the same objective through the oracle's Levin form
    np.testing.assert_allclose(oracle.objective_levin(Z1, X, prob), f1, rtol=1e-9)


@pytest.mark.parametrize("case", CASES)
def test_exact_minimiser_is_fixed_point(case):
    H, W, c, n, r, lam, eps = case
    u, Y, X, Z0, prob = case_data(*case)
    A, DB = naive.dense_system(u, c, Y, r, lam, eps)
    Zs = np.linalg.solve(A, (X.reshape(2, -1) @ DB).T).T.reshape(Z0.shape)
    Z1 = polish.polish(Zs, X, prob)
    np.testing.assert_allclose(Z1, Zs, atol=1e-9 * np.abs(Zs).max())
    # and a point that is not the minimiser moves
    assert np.abs(polish.polish(Zs + 0.1 * Z0, X, prob) - (Zs + 0.1 * Z0)).max() > 1e-3
