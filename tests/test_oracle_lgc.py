"""Pins for the oracle's LGC prior (eq. reg2_lgc): the per-direction gradients against difference matrices built
by loops, the operator against the dense matrix lambda sum_d G_d^T M_{G_d Y} G_d assembled from eq.
(matting_matrix) entry by entry, the objective against the per-window least-squares fit of eq. (reg2_lgc) and
the conjugate-gradient solve against a dense solve.  Every twin here is independent of oracle/lgc.py.
"""
import numpy as np
import pytest

import naive
from oracle import lgc


def rng_for(*key):
    return np.random.default_rng(np.random.SeedSequence([29, *key]))


def diff_matrix(H, W, axis, forward=True):
    """HW x HW periodic first difference by loops: forward z[p + e] - z[p], backward z[p] - z[p - e]."""
    G = np.zeros((H * W, H * W))
    for i in range(H):
        for j in range(W):
            p = i * W + j
            if axis == "h":
                nb = i * W + (j + 1) % W if forward else i * W + (j - 1) % W
            else:
                nb = ((i + 1) % H) * W + j if forward else ((i - 1) % H) * W + j
            if forward:
                G[p, nb] += 1.0
                G[p, p] -= 1.0
            else:
                G[p, p] += 1.0
                G[p, nb] -= 1.0
    return G


def dense_lgc(u, c, Y, r, lam, eps, forward=True):
    H, W = Y.shape
    DB = naive.decimation_matrix(H, W, c) @ naive.conv_matrix(u, H, W)
    A = DB.T @ DB
    for axis in ("h", "v"):
        G = diff_matrix(H, W, axis, forward)
        GY = (G @ Y.reshape(-1)).reshape(H, W)
        A = A + lam * G.T @ naive.matting_matrix_dense(GY, r, eps) @ G
    return A, DB


CASES = [  # H, W, c, n, r, lam, eps
    (8, 8, 2, 3, 1, 0.1, 1e-3),
    (6, 9, 3, 3, 1, 0.05, 1e-2),
    (8, 12, 4, 5, 1, 0.2, 1e-3),
    (10, 10, 2, 5, 2, 0.3, 0.1),
]


def tiny(H, W, c, n, r, lam, eps, N=2):
    rng = rng_for(H, W, c, n, r)
    u = rng.uniform(0, 1, (n, n))
    u /= u.sum()
    Y = rng.uniform(0, 1, (H, W))
    X = rng.standard_normal((N, H // c, W // c))
    return u, Y, X, rng


@pytest.mark.parametrize("H,W", [(5, 7), (6, 6)])
def test_gradients_and_adjoints_match_difference_matrices(H, W):
    z = rng_for(1, H, W).standard_normal((H, W))
    for axis, g, gT in (("h", lgc.grad_h, lgc.grad_h_adj), ("v", lgc.grad_v, lgc.grad_v_adj)):
        G = diff_matrix(H, W, axis)
        np.testing.assert_allclose(g(z).reshape(-1), G @ z.reshape(-1), atol=1e-14)
        np.testing.assert_allclose(gT(z).reshape(-1), G.T @ z.reshape(-1), atol=1e-14)
    # a ramp along a direction has difference 1 away from the wrap, 1 - side at the wrap
    ramp = np.tile(np.arange(W, dtype=float), (H, 1))
    gh = lgc.grad_h(ramp)
    np.testing.assert_array_equal(gh[:, :-1], 1.0)
    np.testing.assert_array_equal(gh[:, -1], 1.0 - W)
    np.testing.assert_array_equal(lgc.grad_v(ramp), 0.0)


@pytest.mark.parametrize("case", CASES)
def test_apply_matches_dense_lgc_system(case):
    H, W, c, n, r, lam, eps = case
    u, Y, _, rng = tiny(*case)
    A, _ = dense_lgc(u, c, Y, r, lam, eps)
    prob = lgc.LgcProblem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    Z = rng.standard_normal((3, H, W))
    np.testing.assert_allclose(lgc.apply_A_lgc(Z, prob).reshape(3, -1), Z.reshape(3, -1) @ A.T, atol=1e-10)
    np.testing.assert_allclose(A, A.T, atol=1e-10)


@pytest.mark.parametrize("case", CASES[:2])
def test_operator_independent_of_difference_orientation(case):
    """The reading of the gradient filters: backward differences give the same operator as forward ones."""
    H, W, c, n, r, lam, eps = case
    u, Y, _, _ = tiny(*case)
    Af, _ = dense_lgc(u, c, Y, r, lam, eps, forward=True)
    Ab, _ = dense_lgc(u, c, Y, r, lam, eps, forward=False)
    np.testing.assert_allclose(Af, Ab, atol=1e-10)


@pytest.mark.parametrize("case", CASES[:3])
def test_objective_is_window_least_squares_of_both_gradients(case):
    """Eq. (reg2_lgc) with the window coefficients of each direction fitted in closed form per window."""
    H, W, c, n, r, lam, eps = case
    u, Y, X, rng = tiny(*case)
    prob = lgc.LgcProblem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    Z = rng.standard_normal((2, H, W))
    DB = naive.decimation_matrix(H, W, c) @ naive.conv_matrix(u, H, W)
    got = lgc.objective_lgc(Z, X, prob)
    for i in range(2):
        res = DB @ Z[i].reshape(-1) - X[i].reshape(-1)
        want = 0.5 * float(res @ res)
        for axis in ("h", "v"):
            G = diff_matrix(H, W, axis)
            gz = (G @ Z[i].reshape(-1)).reshape(H, W)
            gy = (G @ Y.reshape(-1)).reshape(H, W)
            want += 0.5 * lam * naive.levin_penalty(gz, gy, r, eps)
        assert got[i] == pytest.approx(want, rel=1e-10)


@pytest.mark.parametrize("case", CASES[:3])
def test_cg_converges_to_dense_solve(case):
    H, W, c, n, r, lam, eps = case
    u, Y, X, _ = tiny(*case)
    A, DB = dense_lgc(u, c, Y, r, lam, eps)
    prob = lgc.LgcProblem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    b = (X.reshape(2, -1) @ DB).reshape(2, H, W)
    want = np.linalg.solve(A, b.reshape(2, -1).T).T
    z, its = lgc.cg_lgc(prob, b, max_iters=20 * H * W, tol=1e-13)
    np.testing.assert_allclose(z.reshape(2, -1), want, rtol=0, atol=1e-8 * np.abs(want).max())
    assert np.all(its < 20 * H * W)


def test_flat_pan_reduces_to_window_mean_smoothing_of_gradients():
    """A constant PAN has zero gradient guides, so every window of both has zero variance: at eps = 0 the slope
    term drops and each direction's M becomes the window-mean operator sum_k (I_k - 1 1^T / |w|) on w_k."""
    H = W = 6
    u = np.zeros((3, 3))
    u[1, 1] = 1.0
    Y = np.full((H, W), 0.7)
    prob = lgc.LgcProblem(u=u, c=1, Y=Y, r=1, lam=1.0, eps=0.0)
    z = rng_for(7).standard_normal((1, H, W))
    nw = 9
    want = np.zeros((H, W))
    for axis in ("h", "v"):
        G = diff_matrix(H, W, axis)
        Wmean = np.zeros((H * W, H * W))
        for ki in range(H):
            for kj in range(W):
                pix = naive.window_pixels(ki, kj, 1, H, W)
                for m in pix:
                    Wmean[m, m] += 1.0
                    for nn in pix:
                        Wmean[m, nn] -= 1.0 / nw
        want += (G.T @ Wmean @ G @ z[0].reshape(-1)).reshape(H, W)
    np.testing.assert_allclose(lgc.apply_lgc(z, prob)[0], want, atol=1e-11)
