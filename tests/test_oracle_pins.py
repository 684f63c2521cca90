"""Pins for the FP64 oracle: brute force on tiny inputs, identities, closed forms and special cases.

None of these checks re-uses the oracle's own formulas: the twins in naive.py are written from the
definitions with loops and dense matrices.
"""
import os

import numpy as np
import pytest

import naive
import oracle
from oracle.llp import Problem
from paper_2103_09943_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng_for(*key):
    return np.random.default_rng(np.random.SeedSequence([7, *key]))


# ----------------------------------------------------------------------------------------------- data term ---

@pytest.mark.parametrize("H,W,n", [(10, 10, 1), (10, 10, 3), (8, 12, 5), (9, 6, 3)])
def test_blur_is_direct_circular_convolution(H, W, n):
    rng = rng_for(1, H, W, n)
    z = rng.standard_normal((H, W))
    u = rng.uniform(0, 1, (n, n))  # asymmetric on purpose: catches convolution/correlation swaps
    got = oracle.blur(z, oracle.kernel_otf(u, H, W))
    np.testing.assert_allclose(got, naive.conv_direct(z, u), atol=1e-12)


@pytest.mark.parametrize("H,W,n", [(8, 8, 3), (6, 9, 5)])
def test_blur_adjoint_is_transpose(H, W, n):
    rng = rng_for(2, H, W, n)
    z = rng.standard_normal((H, W))
    u = rng.uniform(0, 1, (n, n))
    got = oracle.blur_adjoint(z, oracle.kernel_otf(u, H, W))
    want = (naive.conv_matrix(u, H, W).T @ z.reshape(-1)).reshape(H, W)
    np.testing.assert_allclose(got, want, atol=1e-12)


@pytest.mark.parametrize("H,W,c", [(8, 8, 2), (12, 6, 3), (8, 8, 4), (5, 5, 1)])
def test_decimation_and_adjoint(H, W, c):
    rng = rng_for(3, H, W, c)
    z = rng.standard_normal((H, W))
    x = rng.standard_normal((H // c, W // c))
    D = naive.decimation_matrix(H, W, c)
    np.testing.assert_array_equal(oracle.decimate(z, c).reshape(-1), D @ z.reshape(-1))
    np.testing.assert_array_equal(oracle.decimate_adjoint(x, c, H, W).reshape(-1), D.T @ x.reshape(-1))


# ------------------------------------------------------------------------------------------------ LLP term ---

def test_laplacian_reproduces_printed_stencil():
    S = np.loadtxt(os.path.join(GOLDEN, "laplacian_stencil.txt"))
    delta = np.zeros((7, 7))
    delta[3, 3] = 1.0
    got = oracle.laplacian(delta)
    np.testing.assert_array_equal(got[2:5, 2:5], S)
    assert np.count_nonzero(got) == 5


@pytest.mark.parametrize("H,W", [(6, 6), (5, 8)])
def test_laplacian_matrix(H, W):
    z = rng_for(4, H, W).standard_normal((H, W))
    want = (naive.laplacian_matrix(H, W) @ z.reshape(-1)).reshape(H, W)
    np.testing.assert_allclose(oracle.laplacian(z), want, atol=1e-13)


@pytest.mark.parametrize("H,W,r", [(7, 7, 1), (6, 9, 2), (5, 5, 2)])
def test_window_sum_naive(H, W, r):
    a = rng_for(5, H, W, r).standard_normal((H, W))
    np.testing.assert_allclose(oracle.window_sum(a, r), naive.window_sum_naive(a, r), atol=1e-12)
    np.testing.assert_allclose(oracle.window_sum(np.ones((H, W)), r), (2 * r + 1) ** 2)


@pytest.mark.parametrize("H,W,r,eps", [(8, 8, 1, 1e-3), (6, 10, 1, 0.1), (10, 10, 2, 1e-2), (7, 7, 1, 0.0)])
def test_matting_apply_matches_assembled_matrix(H, W, r, eps):
    rng = rng_for(6, H, W, r)
    I = rng.standard_normal((H, W))
    l = rng.standard_normal((H, W))
    M = naive.matting_matrix_dense(I, r, eps)
    np.testing.assert_allclose(oracle.matting_apply(I, l, r, eps).reshape(-1), M @ l.reshape(-1), atol=1e-10)


@pytest.mark.parametrize("H,W,r,eps", [(6, 6, 1, 1e-3), (7, 5, 1, 0.5), (8, 8, 2, 1e-2)])
def test_levin_identity(H, W, r, eps):
    """Theorem 1 of the cited matting work (eq. pansharp_penalty): min_{a,c} J = alpha^T M alpha."""
    rng = rng_for(7, H, W, r)
    I = rng.standard_normal((H, W))
    alpha = rng.standard_normal((H, W))
    M = naive.matting_matrix_dense(I, r, eps)
    a = alpha.reshape(-1)
    quad = a @ M @ a
    assert quad == pytest.approx(naive.levin_penalty(alpha, I, r, eps), rel=1e-10)
    assert float(np.sum(alpha * oracle.matting_apply(I, alpha, r, eps))) == pytest.approx(quad, rel=1e-10)


def test_matting_invariants():
    rng = rng_for(8)
    H = W = 8
    r = 1
    I = rng.standard_normal((H, W))
    nw = 9
    for eps in (0.0, 1e-3, 1.0):
        M = naive.matting_matrix_dense(I, r, eps)
        np.testing.assert_allclose(M, M.T, atol=1e-12)
        ev = np.linalg.eigvalsh(M)
        assert ev.min() > -1e-9 and ev.max() < nw + 1e-9
        np.testing.assert_allclose(oracle.matting_apply(I, np.ones((H, W)), r, eps), 0.0, atol=1e-11)
    # at eps = 0 the guide itself is reproduced exactly by a = 1, c = 0 in every window
    np.testing.assert_allclose(oracle.matting_apply(I, I, r, 0.0), 0.0, atol=1e-10)
    # with eps > 0 it is not
    assert np.abs(oracle.matting_apply(I, I, r, 0.5)).max() > 1e-3


def test_flat_window_pseudo_inverse():
    """A constant guide has sigma^2 = 0; with eps = 0 the slope term is dropped and M l = |w| l - window means."""
    I = np.full((6, 6), 2.5)
    l = rng_for(9).standard_normal((6, 6))
    M = naive.matting_matrix_dense(I, 1, 0.0)
    np.testing.assert_allclose(oracle.matting_apply(I, l, 1, 0.0).reshape(-1), M @ l.reshape(-1), atol=1e-12)


# ---------------------------------------------------------------------------------------------- the system ---

CASES = [  # H, W, c, n, r, lam, eps
    (8, 8, 2, 3, 1, 0.1, 1e-3),
    (12, 12, 3, 5, 1, 1e-2, 1e-2),
    (8, 12, 4, 5, 1, 0.05, 1e-3),
    (10, 10, 2, 3, 2, 0.2, 0.1),
    (6, 6, 1, 3, 1, 0.3, 1e-3),
]


def tiny_problem(H, W, c, n, r, lam, eps, N=2, key=0):
    rng = rng_for(10, H, W, c, n, r, key)
    u = rng.uniform(0, 1, (n, n))
    u /= u.sum()
    Y = rng.uniform(0, 1, (H, W))
    X = rng.standard_normal((N, H // c, W // c))
    return u, Y, X, rng


@pytest.mark.parametrize("case", CASES)
def test_apply_A_and_rhs_match_dense(case):
    H, W, c, n, r, lam, eps = case
    u, Y, X, rng = tiny_problem(*case)
    A, DB = naive.dense_system(u, c, Y, r, lam, eps)
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    Z = rng.standard_normal((2, H, W))
    got = oracle.apply_A(Z, prob).reshape(2, -1)
    np.testing.assert_allclose(got, Z.reshape(2, -1) @ A.T, atol=1e-10)
    np.testing.assert_allclose(oracle.rhs(X, prob).reshape(2, -1), X.reshape(2, -1) @ DB, atol=1e-12)
    np.testing.assert_allclose(A, A.T, atol=1e-10)
    np.linalg.cholesky(A)  # SPD in the generic case


@pytest.mark.parametrize("case", CASES)
def test_cg_converges_to_dense_solve(case):
    H, W, c, n, r, lam, eps = case
    u, Y, X, _ = tiny_problem(*case)
    A, DB = naive.dense_system(u, c, Y, r, lam, eps)
    want = np.linalg.solve(A, (X.reshape(2, -1) @ DB).T).T
    Z, rep = oracle.solve(X, Y, u, c, r, lam, eps, max_iters=20 * H * W, tol=1e-13)
    np.testing.assert_allclose(Z.reshape(2, -1), want, rtol=0, atol=1e-8 * np.abs(want).max())
    assert np.all(rep["rel_residual"] < 1e-11)


def test_cg_fixed_iterate_is_krylov_minimiser():
    """The k-th CG iterate from 0 minimises the A-norm error over span{b, Ab, ..., A^(k-1) b}."""
    case = (8, 8, 2, 3, 1, 0.1, 1e-3)
    H, W, c, n, r, lam, eps = case
    u, Y, X, _ = tiny_problem(*case, N=1)
    A, DB = naive.dense_system(u, c, Y, r, lam, eps)
    b = X.reshape(1, -1)[0] @ DB
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    for k in (1, 3, 6):
        K = np.empty((b.size, k))
        v = b.copy()
        for j in range(k):
            K[:, j] = v
            v = A @ v
        Q, _ = np.linalg.qr(K)
        want = Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ b)
        got, its = oracle.cg(prob, b.reshape(1, H, W), max_iters=k)
        assert its[0] == k
        np.testing.assert_allclose(got.reshape(-1), want, atol=1e-9 * np.abs(want).max())


def test_lambda_zero_gives_min_norm_solution():
    """With lambda = 0 the system is (DB)^T DB z = (DB)^T X; CG from 0 stays in range((DB)^T) and reaches the
    minimum-norm least-squares solution pinv(DB) X."""
    H = W = 8
    c, n = 2, 3
    u, Y, X, _ = tiny_problem(H, W, c, n, 1, 0.0, 1e-3, N=1)
    _, DB = naive.dense_system(u, c, Y, 1, 0.0, 1e-3)
    want = np.linalg.pinv(DB) @ X.reshape(-1)
    Z, _ = oracle.solve(X, Y, u, c, 1, 0.0, 1e-3, max_iters=2000, tol=1e-14)
    np.testing.assert_allclose(Z.reshape(-1), want, atol=1e-8)


def test_identity_kernel_no_decimation_is_smoothing_solve():
    """u = delta, c = 1: A = I + lambda L M L, a pure smoothing system."""
    H = W = 6
    rng = rng_for(11)
    Y = rng.uniform(0, 1, (H, W))
    X = rng.standard_normal((1, H, W))
    u = np.zeros((3, 3))
    u[1, 1] = 1.0
    L = naive.laplacian_matrix(H, W)
    M = naive.matting_matrix_dense((L @ Y.reshape(-1)).reshape(H, W), 1, 1e-2)
    A = np.eye(H * W) + 0.3 * L @ M @ L
    want = np.linalg.solve(A, X.reshape(-1))
    Z, _ = oracle.solve(X, Y, u, 1, 1, 0.3, 1e-2, max_iters=1000, tol=1e-13)
    np.testing.assert_allclose(Z.reshape(-1), want, atol=1e-9)


def test_exact_recovery_of_pan_consistent_truth():
    """Z* = alpha Y + beta with noiseless X = D B Z* and eps = 0 makes both terms of eq. (initialize_z_fast) zero,
    so the solve recovers Z*; with eps > 0 the error shrinks roughly linearly in eps."""
    H = W = 24
    c, n = 2, 5
    rng = rng_for(12)
    Y = rng.uniform(0, 1, (H, W))  # texture-rich: every window has positive variance
    u = scenes.gaussian_kernel(n, 1.0, cx=0.2, cy=-0.3)
    coef = [(0.7, 0.1), (-1.3, 2.0)]
    Zs = np.stack([a * Y + b for a, b in coef])
    X = np.stack([naive.conv_direct(z, u)[::c, ::c] for z in Zs])
    Z, _ = oracle.solve(X, Y, u, c, 1, 0.05, 0.0, max_iters=5000, tol=1e-13)
    np.testing.assert_allclose(Z, Zs, atol=1e-8)
    errs = []
    for eps in (1e-2, 1e-3):
        Ze, _ = oracle.solve(X, Y, u, c, 1, 0.05, eps, max_iters=5000, tol=1e-13)
        errs.append(np.abs(Ze - Zs).max())
    assert errs[1] < errs[0] / 5


@pytest.mark.parametrize("case", CASES[:3])
def test_objective_three_ways(case):
    H, W, c, n, r, lam, eps = case
    u, Y, X, rng = tiny_problem(*case)
    A, DB = naive.dense_system(u, c, Y, r, lam, eps)
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    Z = rng.standard_normal((2, H, W))
    f1 = oracle.objective(Z, X, prob)
    f2 = oracle.objective_levin(Z, X, prob)
    zf, xf = Z.reshape(2, -1), X.reshape(2, -1)
    f3 = [0.5 * z @ A @ z - (x @ DB) @ z + 0.5 * x @ x for z, x in zip(zf, xf)]
    np.testing.assert_allclose(f1, f3, rtol=1e-11)
    np.testing.assert_allclose(f2, f3, rtol=1e-10)


# --------------------------------------------------------------------------------------------- generator ---

def test_gaussian_kernel_unit_gain_and_peak():
    u = scenes.gaussian_kernel(9, 1.5, cx=0.0, cy=0.0)
    assert u.sum() == pytest.approx(1.0, abs=1e-14) and u.min() >= 0
    assert np.unravel_index(np.argmax(u), u.shape) == (4, 4)
    np.testing.assert_allclose(u, u.T, atol=1e-15)
    v = scenes.gaussian_kernel(9, 1.0, cx=0.9, cy=-1.1)
    assert np.unravel_index(np.argmax(v), v.shape) == (4 - 1, 4 + 1)  # row = y = -1, column = x = +1
    w = scenes.gaussian_kernel(17, 2.0, 1.4, theta=0.0)
    # wider along x (columns) than along y (rows)
    assert w[8, 8 + 3] > w[8 + 3, 8]


def test_scene_shapes_and_seeds():
    sc, st = scenes.config_scene(0, 0, side=64)
    assert sc.X.shape == (4, 16, 16) and sc.Y.shape == (64, 64) and sc.u.shape == (9, 9)
    assert sc.X.dtype == np.float32 and sc.Y.dtype == np.float32
    sc2, _ = scenes.config_scene(0, 0, side=64)
    np.testing.assert_array_equal(sc.X, sc2.X)
    sc3, _ = scenes.config_scene(0, 1, side=64)
    assert not np.array_equal(sc.X, sc3.X)
    assert st.max_iters == 50 and st.tol == 0.0 and st.r == 1


# ----------------------------------------------------------------- Fourier-domain preconditioner (PCG) ---

def dense_preconditioner(u, c, Y, r, lam, eps):
    """Dense P = (DB)^T DB + lambda * mbar * L^T L from explicit matrices, mbar the mean of the dense M's diagonal."""
    H, W = Y.shape
    B = naive.conv_matrix(u, H, W)
    D = naive.decimation_matrix(H, W, c)
    L = naive.laplacian_matrix(H, W)
    LY = (L @ Y.reshape(-1)).reshape(H, W)
    M = naive.matting_matrix_dense(LY, r, eps)
    mbar = float(np.mean(np.diag(M)))
    DB = D @ B
    return DB.T @ DB + lam * mbar * L.T @ L, mbar


@pytest.mark.parametrize("case", CASES)
def test_preconditioner_inverts_dense_P(case):
    """precond_apply is the exact inverse of the dense P (every aliasing group, including the one of K = 0),
    and mbar is the mean diagonal entry of the matting matrix assembled entry by entry."""
    H, W, c, n, r, lam, eps = case
    u, Y, X, rng = tiny_problem(*case)
    P, mbar = dense_preconditioner(u, c, Y, r, lam, eps)
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    assert abs(oracle.matting_diag_mean(prob) - mbar) < 1e-12 * max(1.0, mbar)
    V = rng.standard_normal((3, H, W))
    got = oracle.precond_apply((V.reshape(3, -1) @ P.T).reshape(3, H, W), prob, mbar)
    np.testing.assert_allclose(got, V, rtol=0, atol=1e-9 * np.abs(V).max())
    got2 = oracle.precond_apply(V, prob, mbar).reshape(3, -1) @ P.T
    np.testing.assert_allclose(got2, V.reshape(3, -1), rtol=0, atol=1e-9 * np.abs(V).max())


def test_laplacian_symbol_matches_dense_eigenvalues():
    H, W = 6, 8
    L = naive.laplacian_matrix(H, W)
    k1, k2 = 2, 3
    f = np.exp(2j * np.pi * (k1 * np.arange(H)[:, None] / H + k2 * np.arange(W)[None, :] / W)).reshape(-1)
    lam_k = oracle.laplacian_symbol(H, W)[k1, k2]
    np.testing.assert_allclose(L @ f, lam_k * f, atol=1e-12)


@pytest.mark.parametrize("case", CASES[:3])
def test_pcg_converges_to_dense_solve(case):
    H, W, c, n, r, lam, eps = case
    u, Y, X, _ = tiny_problem(*case)
    A, DB = naive.dense_system(u, c, Y, r, lam, eps)
    want = np.linalg.solve(A, (X.reshape(2, -1) @ DB).T).T
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    Z, its = oracle.pcg(prob, oracle.rhs(X, prob), max_iters=20 * H * W, tol=1e-13)
    np.testing.assert_allclose(Z.reshape(2, -1), want, rtol=0, atol=1e-8 * np.abs(want).max())
    assert np.all(its <= H * W)


def test_pcg_fixed_iterate_is_preconditioned_krylov_minimiser():
    """The k-th PCG iterate from 0 minimises the A-norm error over span{s0, (P^-1 A) s0, ..., (P^-1 A)^(k-1) s0},
    s0 = P^-1 b, with the dense P."""
    case = (8, 8, 2, 3, 1, 0.1, 1e-3)
    H, W, c, n, r, lam, eps = case
    u, Y, X, _ = tiny_problem(*case, N=1)
    A, DB = naive.dense_system(u, c, Y, r, lam, eps)
    P, _ = dense_preconditioner(u, c, Y, r, lam, eps)
    b = X.reshape(1, -1)[0] @ DB
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    Pinv_A = np.linalg.solve(P, A)
    for k in (1, 3, 6):
        K = np.empty((b.size, k))
        v = np.linalg.solve(P, b)
        for j in range(k):
            K[:, j] = v
            v = Pinv_A @ v
        Q, _ = np.linalg.qr(K)
        want = Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ b)
        got, its = oracle.pcg(prob, b.reshape(1, H, W), max_iters=k)
        assert its[0] == k
        np.testing.assert_allclose(got.reshape(-1), want, atol=1e-9 * np.abs(want).max())


def test_pcg_beats_cg_on_scene_recipe():
    """On a 64^2 crop-size scene of the 2048^2 recipe the preconditioner cuts the iterations to tol 1e-6."""
    sc, st = scenes.config_scene(1, 0, side=64)
    prob = Problem(u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=st.lam, eps=st.eps)
    b = oracle.rhs(sc.X[:1], prob)
    _, it_cg = oracle.cg(prob, b, max_iters=5000, tol=1e-6)
    _, it_pcg = oracle.pcg(prob, b, max_iters=5000, tol=1e-6)
    assert it_pcg[0] < 0.6 * it_cg[0], (it_pcg, it_cg)
