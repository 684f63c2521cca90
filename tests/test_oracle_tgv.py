"""Pins of oracle.tgv (Algorithm "Blur Kernel Estimation", Sec. III-A and App. A) against brute force, closed
forms and identities that do not reuse its code."""
import numpy as np
import pytest

import oracle
from oracle import tgv
from paper_2103_09943_amd import scenes


def rng_for(*key):
    return np.random.default_rng(np.random.SeedSequence([47, *key]))


def diff_matrices(n):
    """Explicit periodic forward-difference matrices on the n x n grid (row-major vectorisation)."""
    N = n * n
    Dh = np.zeros((N, N))
    Dv = np.zeros((N, N))
    for i in range(n):
        for j in range(n):
            k = i * n + j
            Dh[k, i * n + (j + 1) % n] += 1.0
            Dh[k, k] -= 1.0
            Dv[k, ((i + 1) % n) * n + j] += 1.0
            Dv[k, k] -= 1.0
    return Dh, Dv


@pytest.mark.parametrize("n", [3, 5, 8])
def test_gradients_match_explicit_matrices(n):
    rng = rng_for(1, n)
    u = rng.standard_normal((n, n))
    p = rng.standard_normal((2, n, n))
    g = rng.standard_normal((2, n, n))
    Dh, Dv = diff_matrices(n)
    got = tgv.grad(u)
    np.testing.assert_allclose(got[0].ravel(), Dh @ u.ravel(), atol=1e-12)
    np.testing.assert_allclose(got[1].ravel(), Dv @ u.ravel(), atol=1e-12)
    np.testing.assert_allclose(tgv.grad_adj(g).ravel(), Dh.T @ g[0].ravel() + Dv.T @ g[1].ravel(), atol=1e-12)
    E = tgv.sym_grad(p)
    mid = 0.5 * (Dv @ p[0].ravel() + Dh @ p[1].ravel())
    for k, want in enumerate([Dh @ p[0].ravel(), mid, mid, Dv @ p[1].ravel()]):
        np.testing.assert_allclose(E[k].ravel(), want, atol=1e-12)


def test_shrink2_is_the_prox_of_the_l2_norm():
    """x = shrink_2(e, t) minimises t ||x|| + 1/2 ||x - e||^2 at every point: compare with a dense search."""
    rng = rng_for(2)
    e = rng.standard_normal((2, 6)) * np.array([1.0, 0.2, 3.0, 0.01, 0.5, 2.0])
    t = 0.4
    x = tgv.shrink2(e, t)
    for k in range(e.shape[1]):
        def f(v):
            return t * np.linalg.norm(v) + 0.5 * np.sum((v - e[:, k]) ** 2)
        # the minimiser lies on the segment from 0 to e: scan it finely, then compare values
        s = np.linspace(0.0, 1.0, 200001)
        vals = t * s * np.linalg.norm(e[:, k]) + 0.5 * (1 - s) ** 2 * np.sum(e[:, k] ** 2)
        best = s[np.argmin(vals)] * e[:, k]
        assert f(x[:, k]) <= f(best) + 1e-10
        np.testing.assert_allclose(x[:, k], best, atol=1e-4 * max(1.0, np.linalg.norm(e[:, k])))


def test_simplex_projection():
    rng = rng_for(3)
    for trial in range(20):
        v = rng.standard_normal((5, 5)) * rng.uniform(0.01, 3.0)
        x = tgv.project_simplex(v)
        assert x.min() >= 0.0
        assert abs(x.sum() - 1.0) < 1e-12
        # the threshold found by bisection on sum(max(v - theta, 0)) = 1 gives the same point
        lo, hi = v.min() - 1.0, v.max()
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if np.maximum(v - mid, 0.0).sum() > 1.0:
                lo = mid
            else:
                hi = mid
        np.testing.assert_allclose(x, np.maximum(v - 0.5 * (lo + hi), 0.0), atol=1e-12)
        # and no random feasible point is closer to v
        for _ in range(50):
            q = rng.dirichlet(np.ones(25)).reshape(5, 5)
            assert np.sum((q - v) ** 2) >= np.sum((x - v) ** 2) - 1e-12


@pytest.mark.parametrize("n,c", [(3, 2), (5, 4), (7, 3)])
def test_E_is_decimated_convolution_of_pan(n, c):
    rng = rng_for(4, n, c)
    H = W = 6 * c
    Y = rng.uniform(0, 1, (H, W))
    u = rng.uniform(0, 1, (n, n))
    E = tgv.conv_matrix_E(Y, n, c)
    want = oracle.decimate(oracle.blur(Y[None], oracle.kernel_otf(u, H, W)), c)[0]
    np.testing.assert_allclose(E @ u.ravel(), want.ravel(), atol=1e-12)


def test_omega_is_regularised_least_squares():
    rng = rng_for(5)
    Xp = rng.uniform(0, 1, (4, 12, 12))
    Y = rng.uniform(0, 1, (48, 48))
    l, lam_w, c = 1, 3.0, 4
    om = tgv.estimate_omega(Xp, Y, c, l, lam_w)
    M = np.stack([tgv.circ_conv(x, tgv.box_kernel(2 * l + 1)).ravel() for x in Xp], axis=1)
    v = oracle.decimate(oracle.blur(Y[None], oracle.kernel_otf(tgv.box_kernel(c * l + 1), 48, 48)), c)[0].ravel()
    G = np.diff(np.eye(4), axis=0)
    want, *_ = np.linalg.lstsq(np.vstack([M, np.sqrt(lam_w) * G]), np.concatenate([v, np.zeros(3)]), rcond=None)
    np.testing.assert_allclose(om, want, atol=1e-10)
    # the box pre-blur on the LR grid is a true circular convolution (the oracle's FFT path agrees)
    np.testing.assert_allclose(tgv.circ_conv(Xp[0], tgv.box_kernel(3)),
                               oracle.blur(Xp[:1], oracle.kernel_otf(tgv.box_kernel(3), 12, 12))[0], atol=1e-12)


@pytest.mark.parametrize("n", [5, 9])
def test_up_step_cramer_matches_dense_minimiser(n):
    """eq. (u_p_solution) by Cramer's rule per frequency equals (i) a direct 3 x 3 complex solve per frequency and
    (ii) the minimiser of the (u, p) quadratic assembled from explicit difference matrices."""
    rng = rng_for(6, n)
    a1m1, a2m2, mu3 = 100.0, 0.6, 100.0
    x = rng.standard_normal((2, n, n))
    y = rng.standard_normal((4, n, n))
    y[2] = y[1]
    L1 = rng.standard_normal((2, n, n))
    L2 = rng.standard_normal((4, n, n))
    L2[2] = L2[1]
    z = rng.standard_normal((n, n))
    L3 = rng.standard_normal((n, n))
    B = tgv.up_rhs(x, y, z, L1, L2, L3, a1m1, a2m2, mu3)
    u, p1, p2 = tgv.up_solve(*B, a1m1, a2m2, mu3)
    # (i) per-frequency direct solve
    d1, d2, d3, d4, d5, d6 = tgv.up_blocks(n, a1m1, a2m2, mu3)
    F = [np.fft.fft2(b) for b in B]
    sol = np.zeros((3, n, n), complex)
    for k1 in range(n):
        for k2 in range(n):
            Mk = np.array([[d1[k1, k2], np.conj(d4[k1, k2]), np.conj(d5[k1, k2])],
                           [d4[k1, k2], d2[k1, k2], np.conj(d6[k1, k2])],
                           [d5[k1, k2], d6[k1, k2], d3[k1, k2]]])
            sol[:, k1, k2] = np.linalg.solve(Mk, [f[k1, k2] for f in F])
    for got, want in zip((u, p1, p2), sol):
        np.testing.assert_allclose(got, np.fft.ifft2(want).real, atol=1e-10)
    # (ii) the quadratic of the (u, p) step with the mu_3 coupling, minimised by dense least squares
    Dh, Dv = diff_matrices(n)
    N = n * n
    Z0 = np.zeros((N, N))
    I = np.eye(N)
    s1, s2 = np.sqrt(a1m1), np.sqrt(a2m2)
    rows = [  # residual blocks (operator on [u; p1; p2], target)
        (s1 * np.hstack([Dh, -I, Z0]), s1 * (x[0] - L1[0]).ravel()),
        (s1 * np.hstack([Dv, Z0, -I]), s1 * (x[1] - L1[1]).ravel()),
        (s2 * np.hstack([Z0, Dh, Z0]), s2 * (y[0] - L2[0]).ravel()),
        (s2 * np.hstack([Z0, 0.5 * Dv, 0.5 * Dh]), s2 * (y[1] - L2[1]).ravel()),
        (s2 * np.hstack([Z0, 0.5 * Dv, 0.5 * Dh]), s2 * (y[2] - L2[2]).ravel()),
        (s2 * np.hstack([Z0, Z0, Dv]), s2 * (y[3] - L2[3]).ravel()),
        (np.sqrt(mu3) * np.hstack([I, Z0, Z0]), np.sqrt(mu3) * (z - L3).ravel()),
    ]
    K = np.vstack([r[0] for r in rows])
    t = np.concatenate([r[1] for r in rows])
    want, *_ = np.linalg.lstsq(K, t, rcond=None)
    np.testing.assert_allclose(np.concatenate([u.ravel(), p1.ravel(), p2.ravel()]), want, atol=1e-9)


def test_z_step_is_regularised_least_squares():
    rng = rng_for(7)
    n, c = 5, 4
    Y = rng.uniform(0, 1, (32, 32))
    f = rng.standard_normal(64)
    E = tgv.conv_matrix_E(Y, n, c)
    ut, L3, mu3 = rng.standard_normal((n, n)), rng.standard_normal((n, n)), 7.0
    z, zs = tgv.z_update(tgv.z_prepare(E, mu3), E.T @ f, ut, L3, mu3)
    want, *_ = np.linalg.lstsq(np.vstack([E, np.sqrt(mu3) * np.eye(n * n)]),
                               np.concatenate([f, np.sqrt(mu3) * (ut + L3).ravel()]), rcond=None)
    np.testing.assert_allclose(zs.ravel(), want, atol=1e-10)
    assert z.min() >= 0.0 and abs(z.sum() - 1.0) < 1e-12


def recovery_scene():
    rng = np.random.default_rng(np.random.SeedSequence([47, 8]))
    u = scenes.gaussian_kernel(9, 1.6, 1.2, theta=0.4, cx=0.7, cy=-0.4)
    sc = scenes.make_scene(rng, 256, 256, 6, 4, u, pan_noise=0.0, ms_noise=0.0)
    return u, sc


def test_recovers_known_gaussian_kernel_on_noiseless_data():
    """Algorithm 1 with the paper's parameters (Sec. IV-C) on a noiseless synthetic scene (6 bands, 256^2 PAN,
    x4): the estimate lies in the simplex and is within eps_r (eq. relative_error_kernel) of the true kernel."""
    u, sc = recovery_scene()
    uh, info = tgv.estimate_kernel(sc.X, sc.Y, 4, tgv.TgvParams(n=9))
    assert uh.min() >= 0.0 and abs(uh.sum() - 1.0) < 1e-12
    assert info["iters"] < 10000
    assert tgv.relative_kernel_error(u, uh) < 5.0  # the uniform start is at 84%
    # with the exact spectral weights (regressed from the truth) the ADMM alone recovers the kernel closely
    w, *_ = np.linalg.lstsq(sc.Z.reshape(6, -1).T.astype(np.float64), sc.Y.ravel().astype(np.float64), rcond=None)
    uw, _ = tgv.estimate_kernel(sc.X, sc.Y, 4, tgv.TgvParams(n=9), omega=w)
    assert tgv.relative_kernel_error(u, uw) < 1.0


def test_recovers_motion_blur_kernel_of_the_paper():
    """The kernel of the paper's kernel-estimation experiment (Sec. IV-C: R = 9, sigma = 2, d = 3, theta =
    -13.7 degrees, peak at (1.392, 0.093), eq. blur_kernel_final) on a noiseless synthetic scene."""
    import math
    u = scenes.motion_blur_kernel(9, 2.0, 3.0, math.radians(-13.7), 1.392, 0.093)
    rng = np.random.default_rng(np.random.SeedSequence([47, 9]))
    sc = scenes.make_scene(rng, 256, 256, 6, 4, u, pan_noise=0.0, ms_noise=0.0)
    uh, _ = tgv.estimate_kernel(sc.X, sc.Y, 4, tgv.TgvParams(n=19))
    assert uh.min() >= 0.0 and abs(uh.sum() - 1.0) < 1e-12
    assert tgv.relative_kernel_error(u, uh) < 10.0
    w, *_ = np.linalg.lstsq(sc.Z.reshape(6, -1).T.astype(np.float64), sc.Y.ravel().astype(np.float64), rcond=None)
    uw, _ = tgv.estimate_kernel(sc.X, sc.Y, 4, tgv.TgvParams(n=19), omega=w)
    assert tgv.relative_kernel_error(u, uw) < 1.0
