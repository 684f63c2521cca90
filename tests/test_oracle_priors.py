"""Pins for the oracle's prior family (oracle/priors.py): for every prior of the paper's comparison, the operator
against the dense matrix sum_d F_d^T M_{F_d Y} F_d built from circulant matrices assembled by loops and the
matting matrix of eq. (matting_matrix) assembled entry by entry; the LLP member against the LLP operator of the
main oracle; the LGC member against the explicit-difference form; the filters against their definitions; the
objective against per-window least squares; CG against a dense solve.
"""
import numpy as np
import pytest

import naive
import oracle
from oracle import lgc, priors
from oracle.llp import Problem


def rng_for(*key):
    return np.random.default_rng(np.random.SeedSequence([31, *key]))


def tiny(H, W, c, n, key=0):
    rng = rng_for(H, W, c, n, key)
    u = rng.uniform(0, 1, (n, n))
    u /= u.sum()
    Y = rng.uniform(0, 1, (H, W))
    X = rng.standard_normal((2, H // c, W // c))
    return u, Y, X, rng


def dense_filters(kind, u, H, W):
    """Circulant matrices of the prior's filters, from the paper's definitions, by loops."""
    if kind == "llp":
        return [naive.laplacian_matrix(H, W)]
    if kind == "lgc":
        mats = []
        for di, dj in ((0, 1), (1, 0)):
            G = np.zeros((H * W, H * W))
            for i in range(H):
                for j in range(W):
                    G[i * W + j, ((i + di) % H) * W + (j + dj) % W] += 1.0
                    G[i * W + j, i * W + j] -= 1.0
            mats.append(G)
        return mats
    if kind == "lpp":
        return [np.eye(H * W)]
    B = naive.conv_matrix(u, H, W)
    if kind == "lpf":
        return [B]
    if kind == "hpf":
        return [np.eye(H * W) - B]
    raise ValueError(kind)


def dense_prior_system(kind, u, c, Y, r, lam, eps):
    H, W = Y.shape
    DB = naive.decimation_matrix(H, W, c) @ naive.conv_matrix(u, H, W)
    A = DB.T @ DB
    for F in dense_filters(kind, u, H, W):
        FY = (F @ Y.reshape(-1)).reshape(H, W)
        A = A + lam * F.T @ naive.matting_matrix_dense(FY, r, eps) @ F
    return A, DB


CASES = [  # H, W, c, n, r, lam, eps
    (8, 8, 2, 3, 1, 0.1, 1e-3),
    (6, 9, 3, 3, 1, 0.05, 1e-2),
    (8, 12, 4, 5, 1, 0.2, 1e-3),
    (10, 10, 2, 5, 2, 0.3, 0.1),
]


def test_filters_follow_their_definitions():
    u = rng_for(1).uniform(0, 1, (5, 5))
    u /= u.sum()
    z = rng_for(2).standard_normal((7, 9))
    f = priors.prior_filters("lgc", u)
    np.testing.assert_allclose(oracle.blur(z, oracle.kernel_otf(f[0], 7, 9)), np.roll(z, -1, 1) - z, atol=1e-13)
    np.testing.assert_allclose(oracle.blur(z, oracle.kernel_otf(f[1], 7, 9)), np.roll(z, -1, 0) - z, atol=1e-13)
    np.testing.assert_allclose(oracle.blur(z, oracle.kernel_otf(priors.prior_filters("lpp", u)[0], 7, 9)), z,
                               atol=1e-13)
    hpf = priors.prior_filters("hpf", u)[0]
    np.testing.assert_allclose(hpf.sum(), 0.0, atol=1e-15)  # delta - u removes the mean: a high-pass
    np.testing.assert_allclose(oracle.blur(z, oracle.kernel_otf(hpf, 7, 9)), z - naive.conv_direct(z, u),
                               atol=1e-12)
    np.testing.assert_array_equal(priors.prior_filters("lpf", u)[0], u)


@pytest.mark.parametrize("kind", priors.KINDS)
@pytest.mark.parametrize("case", CASES[:3])
def test_operator_matches_dense_system(kind, case):
    H, W, c, n, r, lam, eps = case
    u, Y, _, rng = tiny(H, W, c, n)
    A, _ = dense_prior_system(kind, u, c, Y, r, lam, eps)
    prob = priors.PriorProblem(kind, u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    Z = rng.standard_normal((3, H, W))
    np.testing.assert_allclose(priors.apply_A_prior(Z, prob).reshape(3, -1), Z.reshape(3, -1) @ A.T, atol=1e-10)
    np.testing.assert_allclose(A, A.T, atol=1e-10)


@pytest.mark.parametrize("case", CASES)
def test_llp_and_lgc_members_match_their_own_oracles(case):
    H, W, c, n, r, lam, eps = case
    u, Y, _, rng = tiny(H, W, c, n, key=1)
    Z = rng.standard_normal((2, H, W))
    p_llp = priors.PriorProblem("llp", u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    np.testing.assert_allclose(priors.apply_prior(Z, p_llp),
                               oracle.apply_llp(Z, Problem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)), atol=1e-11)
    p_lgc = priors.PriorProblem("lgc", u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    np.testing.assert_allclose(priors.apply_prior(Z, p_lgc),
                               lgc.apply_lgc(Z, lgc.LgcProblem(u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)), atol=1e-11)


@pytest.mark.parametrize("kind", ["lgc", "hpf", "lpp"])
def test_objective_is_window_least_squares(kind):
    H, W, c, n, r, lam, eps = CASES[0]
    u, Y, X, rng = tiny(H, W, c, n, key=2)
    prob = priors.PriorProblem(kind, u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    Z = rng.standard_normal((2, H, W))
    DB = naive.decimation_matrix(H, W, c) @ naive.conv_matrix(u, H, W)
    got = priors.objective_prior(Z, X, prob)
    for i in range(2):
        res = DB @ Z[i].reshape(-1) - X[i].reshape(-1)
        want = 0.5 * float(res @ res)
        for F in dense_filters(kind, u, H, W):
            fz = (F @ Z[i].reshape(-1)).reshape(H, W)
            fy = (F @ Y.reshape(-1)).reshape(H, W)
            want += 0.5 * lam * naive.levin_penalty(fz, fy, r, eps)
        assert got[i] == pytest.approx(want, rel=1e-10)


@pytest.mark.parametrize("kind", priors.KINDS)
def test_cg_converges_to_dense_solve(kind):
    H, W, c, n, r, lam, eps = CASES[2]
    u, Y, X, _ = tiny(H, W, c, n, key=3)
    A, DB = dense_prior_system(kind, u, c, Y, r, lam, eps)
    prob = priors.PriorProblem(kind, u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
    b = (X.reshape(2, -1) @ DB).reshape(2, H, W)
    want = np.linalg.solve(A, b.reshape(2, -1).T).T
    z, its = priors.cg_prior(prob, b, max_iters=20 * H * W, tol=1e-13)
    np.testing.assert_allclose(z.reshape(2, -1), want, rtol=0, atol=1e-8 * np.abs(want).max())
    # from the solution itself, CG starts converged
    z2, its2 = priors.cg_prior(prob, b, z0=want.reshape(2, H, W), max_iters=5, tol=1e-9)
    assert np.all(its2 == 0)


def test_every_prior_annihilates_constants():
    """Each filter maps a constant plane to a constant plane and M 1 = 0 for every guide, so no prior constrains
    the mean of a band: the mean is fixed by the data term alone."""
    H, W, c, n, r, lam, eps = CASES[0]
    u, Y, _, _ = tiny(H, W, c, n, key=4)
    ones = np.ones((1, H, W))
    for kind in priors.KINDS:
        prob = priors.PriorProblem(kind, u=u, c=c, Y=Y, r=r, lam=lam, eps=eps)
        assert np.abs(priors.apply_prior(ones, prob)).max() < 1e-11, kind
