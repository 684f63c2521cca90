"""GPU: the A, C step and the FFT Z step of Algorithm "Fast Pansharpening" (llp_polish) against the oracle's
steps in the paper's order (oracle.polish: eq. ac_h_compute, the guided output, eq. Z_solution), through the C ABI.

The library forms the same Z as Z0 + P1^{-1}(b - A Z0); the oracle forms A, C and Lhat explicitly.  Bar: relative
L2 <= 1e-5 per band (float32 against FP64 on the same float32 inputs).  Shapes cover every radix, odd band
counts and c = 1..4; the starts are a few CG iterations (far from the minimiser) and a converged solve.
"""
import numpy as np
import pytest

import oracle
from oracle import polish
from oracle.llp import Problem
from paper_2103_09943_amd import binding as B
from paper_2103_09943_amd import scenes

pytestmark = pytest.mark.gpu

SHAPES = [  # N, h, w, c, n, r
    (3, 24, 20, 2, 5, 1),
    (1, 14, 12, 4, 9, 1),
    (2, 16, 16, 4, 17, 2),
    (4, 64, 64, 4, 9, 1),
    (2, 30, 30, 1, 3, 1),
    (1, 8, 8, 3, 5, 1),
    (5, 32, 40, 4, 15, 2),
]


def f32(x):
    return float(np.float32(x))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def ctx(torch_dev):
    c = B.Context(0)
    yield c
    c.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_l2(got, want):
    got = got.reshape(got.shape[0], -1)
    want = want.reshape(want.shape[0], -1)
    return np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)


@pytest.mark.parametrize("shape", SHAPES)
def test_polish_matches_oracle(ctx, torch_dev, shape):
    N, h, w, c, n, r = shape
    rng = np.random.default_rng(np.random.SeedSequence([91, *shape]))
    X, Y, u, _ = scenes.random_problem(rng, N, h * c, w * c, c, n)
    lam, eps = 0.05, 1e-2
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=f32(lam), eps=f32(eps))
    z0, _ = oracle.cg(prob, oracle.rhs(X, prob), max_iters=5)  # a start far from the minimiser
    z0 = z0.astype(np.float32)
    got = ctx.polish(dev(torch_dev, z0), dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, u), r=r, lam=lam,
                     eps=eps)
    want = polish.polish(z0.astype(np.float64), X, prob)
    err = rel_l2(host(got), want)
    assert np.all(err < 1e-5), err
    # the round moved z0 by much more than the bar, so the comparison is not z0 against z0
    assert np.all(rel_l2(z0.astype(np.float64), want) > 1e-3)


def test_polish_after_solve_on_parity_scene(ctx, torch_dev):
    """The 256^2 x 4 parity scene: Algorithm Fast Pansharpening end to end (solve at tol 1e-6, then the round).
    The converged Z0 is nearly a fixed point; the round must match the oracle's and must not raise the objective
    of eq. (initialize_z_fast)."""
    sc, st = scenes.config_scene(0, 0)
    prob = Problem(u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=f32(st.lam), eps=f32(st.eps))
    args = (dev(torch_dev, sc.X), dev(torch_dev, sc.Y), dev(torch_dev, sc.u))
    Z0, rep, status = ctx.pansharpen(*args, r=st.r, lam=st.lam, eps=st.eps, max_iters=2000, tol=1e-6, precond=1)
    assert status == B.OK
    Z1 = ctx.polish(Z0, *args, r=st.r, lam=st.lam, eps=st.eps)
    z0 = host(Z0)
    want = polish.polish(z0, sc.X, prob)
    assert np.all(rel_l2(host(Z1), want) < 1e-5)
    f0 = oracle.objective(z0, sc.X, prob)
    f1 = oracle.objective(host(Z1), sc.X, prob)
    assert np.all(f1 <= f0 * (1 + 1e-6)), (f0, f1)
    # and from a rough start (20 iterations) the round lowers the objective clearly
    Zr, _, _ = ctx.pansharpen(*args, r=st.r, lam=st.lam, eps=st.eps, max_iters=20, tol=0.0)
    Zr1 = ctx.polish(Zr, *args, r=st.r, lam=st.lam, eps=st.eps)
    g0 = oracle.objective(host(Zr), sc.X, prob)
    g1 = oracle.objective(host(Zr1), sc.X, prob)
    assert np.all(g1 < g0), (g0, g1)
    assert np.all(rel_l2(host(Zr1), polish.polish(host(Zr), sc.X, prob)) < 1e-5)


def test_polish_refuses_unsupported(ctx, torch_dev):
    rng = np.random.default_rng(5)
    X, Y, u, _ = scenes.random_problem(rng, 1, 32, 32, 4, 5)
    z0 = np.zeros((1, 32, 32), np.float32)
    with pytest.raises(B.LlpError) as ei:  # r = 0: no window, no LLP weight for the Fourier solve
        ctx.polish(dev(torch_dev, z0), dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, u), r=0, lam=0.05,
                   eps=1e-2)
    assert ei.value.status == B.E_UNSUPPORTED
    with pytest.raises(B.LlpError) as ei:  # an LR side with a prime factor above 7
        X2, Y2, u2, _ = scenes.random_problem(rng, 1, 44, 44, 4, 5)
        ctx.polish(dev(torch_dev, np.zeros((1, 44, 44), np.float32)), dev(torch_dev, X2), dev(torch_dev, Y2),
                   dev(torch_dev, u2), r=1, lam=0.05, eps=1e-2)
    assert ei.value.status == B.E_UNSUPPORTED
