"""GPU: the compared priors (llp_apply_prior, llp_prior_pansharpen) against the oracle's prior family
(oracle/priors.py), through the C ABI; and the LLP solve with a motion-blur kernel (App. B).

Bars as for LLP: operators to relative L2 <= 1e-5 per band (float32 against FP64 on the same float32 inputs);
the CG iterate after a fixed iteration count to relative L2 <= 1e-5 per band; at a tolerance, the returned
HRMS's residual, re-evaluated by the oracle in FP64, within 1.5 tol (the library checks it with its float32
operator).  Shapes span several tiles with ragged edges, odd band counts, c = 1..4 and every filter.
"""
import numpy as np
import pytest

import oracle
from oracle import priors
from oracle.llp import Problem
from paper_2103_09943_amd import binding as B
from paper_2103_09943_amd import scenes

pytestmark = pytest.mark.gpu

KINDS = ["llp", "lgc", "lpp", "lpf", "hpf"]
SHAPES = [  # N, h, w, c, n, r
    (3, 24, 20, 4, 9, 1),    # 96 x 80: two tile columns, ragged
    (2, 30, 36, 2, 5, 2),
    (1, 13, 11, 3, 7, 1),    # ragged under the c = 3 tiles
    (2, 40, 72, 1, 3, 1),
    (1, 16, 16, 4, 17, 2),   # the largest filter the operator takes at r = 2
    (2, 20, 22, 2, 5, 3),    # a window radius without its own kernel instance
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


def case(shape, key):
    N, h, w, c, n, r = shape
    rng = np.random.default_rng(np.random.SeedSequence([47, key, *shape]))
    return scenes.random_problem(rng, N, h * c, w * c, c, n)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("shape", SHAPES)
def test_apply_prior_matches_oracle(ctx, torch_dev, kind, shape):
    N, h, w, c, n, r = shape
    X, Y, u, P = case(shape, 1)
    lam, eps = 0.05, 1e-2
    prob = priors.PriorProblem(kind, u=u, c=c, Y=Y, r=r, lam=f32(lam), eps=f32(eps))
    args = (dev(torch_dev, P), dev(torch_dev, Y), dev(torch_dev, u))
    got = ctx.apply_prior(kind, *args, c=c, r=r, lam=lam, eps=eps)
    err = rel_l2(host(got), priors.apply_prior(P, prob))
    assert np.all(err < 1e-5), (kind, shape, err)
    got = ctx.apply_prior(kind, *args, c=c, r=r, lam=lam, eps=eps, data_term=True)
    err = rel_l2(host(got), priors.apply_A_prior(P, prob))
    assert np.all(err < 1e-5), (kind, shape, err)


@pytest.mark.parametrize("shape", SHAPES[:3])
def test_llp_member_matches_the_llp_operator(ctx, torch_dev, shape):
    """The prior kernel with the Laplacian against the solve's own LLP operator (two independent kernels)."""
    N, h, w, c, n, r = shape
    X, Y, u, P = case(shape, 2)
    args = (dev(torch_dev, P), dev(torch_dev, Y), dev(torch_dev, u))
    a = ctx.apply_prior("llp", *args, c=c, r=r, lam=0.05, eps=1e-2, data_term=True)
    b = ctx.apply_A(*args, c=c, r=r, lam=0.05, eps=1e-2)
    assert np.all(rel_l2(host(a), host(b)) < 2e-6)


@pytest.mark.parametrize("kind", KINDS)
def test_fixed_iterations_match_oracle_cg(ctx, torch_dev, kind):
    shape = (3, 24, 20, 4, 9, 1)
    N, h, w, c, n, r = shape
    X, Y, u, _ = case(shape, 3)
    lam, eps, K = 0.05, 1e-2, 25
    prob = priors.PriorProblem(kind, u=u, c=c, Y=Y, r=r, lam=f32(lam), eps=f32(eps))
    Z, rep, status = ctx.prior_pansharpen(kind, dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, u), r=r,
                                          lam=lam, eps=eps, max_iters=K)
    assert status == B.OK and all(x["iters"] == K for x in rep), rep
    want, _ = priors.cg_prior(prob, oracle.rhs(X, prob), max_iters=K)
    err = rel_l2(host(Z), want)
    assert np.all(err < 1e-5), (kind, err)


@pytest.mark.parametrize("kind", ["lgc", "hpf", "lpp"])
def test_tolerance_on_parity_scene(ctx, torch_dev, kind):
    """The 256^2 x 4 scene (c 4, n 9, r 1) to tol 1e-5: every band converged, its residual re-evaluated in FP64 by
    the oracle within 1.5 tol; a restart from the returned HRMS stops at once."""
    sc, st = scenes.config_scene(0, 0)
    prob = priors.PriorProblem(kind, u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=f32(st.lam), eps=f32(st.eps))
    args = (dev(torch_dev, sc.X), dev(torch_dev, sc.Y), dev(torch_dev, sc.u))
    tol = 1e-5
    Z, rep, status = ctx.prior_pansharpen(kind, *args, r=st.r, lam=st.lam, eps=st.eps, max_iters=3000, tol=tol)
    assert status == B.OK, rep
    assert all(x["status"] == B.OK and x["true_rel_residual"] <= tol for x in rep), rep
    b = oracle.rhs(sc.X, prob).astype(np.float32).astype(np.float64)
    res = b - priors.apply_A_prior(host(Z), prob)
    rel = np.linalg.norm(res.reshape(4, -1), axis=1) / np.linalg.norm(b.reshape(4, -1), axis=1)
    assert np.all(rel <= 1.5 * tol), rel
    Z2, rep2, _ = ctx.prior_pansharpen(kind, *args, r=st.r, lam=st.lam, eps=st.eps, max_iters=3000, tol=tol,
                                       init=Z.clone())
    assert all(x["iters"] == 0 and x["status"] == B.OK for x in rep2), rep2
    assert torch_dev.equal(Z2, Z)


def test_priors_differ_and_llp_member_solves_like_the_llp_path(ctx, torch_dev):
    sc, st = scenes.config_scene(0, 0)
    args = (dev(torch_dev, sc.X), dev(torch_dev, sc.Y), dev(torch_dev, sc.u))
    kw = dict(r=st.r, lam=st.lam, eps=st.eps, max_iters=20)
    outs = {k: host(ctx.prior_pansharpen(k, *args, **kw)[0]) for k in KINDS}
    main = host(ctx.pansharpen(*args, **kw)[0])
    assert np.all(rel_l2(outs["llp"], main) < 1e-5)
    for a in KINDS:
        for b in KINDS:
            if a < b:
                assert np.all(rel_l2(outs[a], outs[b]) > 1e-4), (a, b)


def test_refusals(ctx, torch_dev):
    X, Y, u, P = case((1, 16, 16, 4, 9, 1), 4)
    args = (dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, u))
    with pytest.raises(B.LlpError) as ei:  # the preconditioner is for the LLP solve only
        shp = B.shape_of(*args)
        prm = B.Params(1, 0.05, 1e-2, 10, 0.0, 0, 1)
        out = torch_dev.empty((1, 64, 64), device="cuda")
        B._check(B.lib().llp_prior_pansharpen(ctx._h, shp, prm, 1, B._ptr(args[0]), B._ptr(args[1]),
                                              B._ptr(args[2]), None, B._ptr(out), None, None), "prior")
    assert ei.value.status == B.E_UNSUPPORTED
    with pytest.raises(B.LlpError) as ei:  # unknown prior
        shp = B.shape_of(*args)
        prm = B.Params(1, 0.05, 1e-2, 10, 0.0, 0, 0)
        B._check(B.lib().llp_prior_pansharpen(ctx._h, shp, prm, 7, B._ptr(args[0]), B._ptr(args[1]),
                                              B._ptr(args[2]), None, B._ptr(out), None, None), "prior")
    assert ei.value.status == B.E_ARG
    X2, Y2, u2, P2 = case((1, 16, 16, 4, 29, 2), 5)  # a 29 x 29 filter at r = 2: the tile does not fit in LDS
    with pytest.raises(B.LlpError) as ei:
        ctx.apply_prior("hpf", dev(torch_dev, P2), dev(torch_dev, Y2), dev(torch_dev, u2), c=4, r=2, lam=0.05,
                        eps=1e-2)
    assert ei.value.status == B.E_UNSUPPORTED


def test_motion_blur_kernel_solve(ctx, torch_dev):
    """The LLP solve (plain and preconditioned) on a scene blurred by the motion-blur kernel of App. B, against
    the oracle's CG at a fixed iteration count."""
    rng = np.random.default_rng(np.random.SeedSequence([53]))
    u = scenes.motion_blur_kernel(6, 1.2, 5.0, 0.6, 0.3, -0.2).astype(np.float32)
    Zt = rng.uniform(0, 1, (3, 128, 128))
    Y = Zt.mean(axis=0).astype(np.float32)
    prob = Problem(u=u, c=4, Y=Y, r=1, lam=f32(1e-2), eps=f32(1e-3))
    X = (oracle.decimate(oracle.blur(Zt, prob.otf), 4) + 0.01 * rng.standard_normal((3, 32, 32))).astype(np.float32)
    args = (dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, u))
    Z, rep, _ = ctx.pansharpen(*args, r=1, lam=1e-2, eps=1e-3, max_iters=30)
    want, _ = oracle.cg(prob, oracle.rhs(X, prob), max_iters=30)
    assert np.all(rel_l2(host(Z), want) < 1e-5)
    Zp, rep, _ = ctx.pansharpen(*args, r=1, lam=1e-2, eps=1e-3, max_iters=30, precond=1)
    wantp, _ = oracle.pcg(prob, oracle.rhs(X, prob), max_iters=30)
    assert np.all(rel_l2(host(Zp), wantp) < 1e-5)


def test_full_size_lgc_solve_sampled_bands(ctx, torch_dev):
    """The priors workload as the benchmark runs it: the 8-band 2048^2 scene (x4, 17-tap blur, r 2) under LGC to
    tol 1e-6; on two sampled bands the oracle re-evaluates the returned HRMS's residual in FP64."""
    sc, st = scenes.config_scene(1, 0)
    args = (dev(torch_dev, sc.X), dev(torch_dev, sc.Y), dev(torch_dev, sc.u))
    Z, rep, status = ctx.prior_pansharpen("lgc", *args, r=st.r, lam=st.lam, eps=st.eps, max_iters=st.max_iters,
                                          tol=st.tol)
    assert status == B.OK and all(x["true_rel_residual"] <= st.tol for x in rep), rep
    prob = priors.PriorProblem("lgc", u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=f32(st.lam), eps=f32(st.eps))
    for band in (0, 5):
        Zb = host(Z[band:band + 1])
        b = oracle.rhs(sc.X[band:band + 1], prob).astype(np.float32).astype(np.float64)
        res = b - priors.apply_A_prior(Zb, prob)
        rel = float(np.linalg.norm(res) / np.linalg.norm(b))
        assert rel <= 1.5 * st.tol, (band, rel)
