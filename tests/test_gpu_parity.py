"""GPU parity: every step of the HIP path against the FP64 oracle, through the C ABI.

Bars: operators (PAN statistics, right-hand side, A, objective) to relative L2 <= 1e-5 per band (FP32 against
FP64); the CG iterate after a fixed iteration count to relative L2 <= 1e-5 per band; at a residual tolerance of
1e-6, the objective of the returned HRMS within 1e-6 (relative) of the objective at the exact minimiser.
The oracle always receives the same float32-rounded inputs (and float32-rounded lambda, eps) as the library.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.llp import Problem
from paper_2103_09943_amd import binding as B
from paper_2103_09943_amd import scenes

pytestmark = pytest.mark.gpu


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


def rng_for(*key):
    return np.random.default_rng(np.random.SeedSequence([11, *key]))


def out_residual(prob, b, Z):
    """||f32(b) - A Z|| / ||f32(b)|| per band in FP64: the residual of a float32 HRMS against the float32-rounded
    right-hand side (the one the library holds)."""
    b32 = b.astype(np.float32).astype(np.float64)
    res = b32 - oracle.apply_A(Z, prob)
    N = b.shape[0]
    return np.linalg.norm(res.reshape(N, -1), axis=1) / np.linalg.norm(b32.reshape(N, -1), axis=1)


# ------------------------------------------------------------------------------------------ operators ---

OP_SHAPES = [  # N, h, w, c, n, r
    (4, 64, 64, 4, 9, 1),     # the 256^2 parity scene's shape
    (2, 16, 12, 4, 17, 2),
    (3, 24, 20, 2, 5, 1),     # odd band count
    (1, 7, 9, 3, 7, 2),       # ragged: tiles do not divide the image
    (2, 40, 40, 1, 3, 1),     # c = 1
    (1, 8, 8, 2, 1, 0),       # n = 1, r = 0
    (2, 34, 18, 4, 33, 4),    # largest kernel and window
    (1, 80, 48, 2, 11, 3),
    # shapes on the specialised kernels (c in {2, 4}, n in {9..17, 29}, r in {1, 2})
    (2, 20, 18, 2, 9, 1),
    (1, 16, 40, 2, 17, 2),
    (1, 12, 20, 4, 29, 1),
    (2, 24, 24, 4, 11, 2),
    (1, 9, 17, 4, 15, 1),     # ragged on both tile shapes
]


@pytest.mark.parametrize("shape", OP_SHAPES)
def test_pan_stats(ctx, torch_dev, shape):
    N, h, w, c, n, r = shape
    rng = rng_for(1, *shape)
    Y = rng.uniform(0, 1, (h * c, w * c)).astype(np.float32)
    eps = 1e-3
    G, mu, d = ctx.pan_stats(dev(torch_dev, Y), N=N, c=c, n=n, r=r, eps=eps)
    LY = oracle.laplacian(Y.astype(np.float64))
    omu, _, od = oracle.matting_stats(LY, r, f32(eps))
    np.testing.assert_allclose(host(G), LY, rtol=0, atol=1e-6 * np.abs(LY).max())
    np.testing.assert_allclose(host(mu), omu, rtol=0, atol=1e-6 * np.abs(LY).max())
    np.testing.assert_allclose(host(d), od, rtol=2e-6, atol=0)


@pytest.mark.parametrize("shape", OP_SHAPES)
def test_rhs(ctx, torch_dev, shape):
    N, h, w, c, n, r = shape
    rng = rng_for(2, *shape)
    X = rng.standard_normal((N, h, w)).astype(np.float32)
    u = rng.uniform(0, 1, (n, n))
    u = (u / u.sum()).astype(np.float32)
    b = ctx.rhs(dev(torch_dev, X), dev(torch_dev, u), c)
    prob = Problem(u=u, c=c, Y=np.zeros((h * c, w * c)), r=0, lam=0.0, eps=0.0)
    assert np.all(rel_l2(host(b), oracle.rhs(X, prob)) < 1e-6)


@pytest.mark.parametrize("shape", OP_SHAPES)
def test_apply_A(ctx, torch_dev, shape):
    N, h, w, c, n, r = shape
    rng = rng_for(3, *shape)
    X, Y, u, P = scenes.random_problem(rng, N, h * c, w * c, c, n)
    lam, eps = 0.05, 1e-3
    got = ctx.apply_A(dev(torch_dev, P), dev(torch_dev, Y), dev(torch_dev, u), c=c, r=r, lam=lam, eps=eps)
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=f32(lam), eps=f32(eps))
    err = rel_l2(host(got), oracle.apply_A(P, prob))
    assert np.all(err < 1e-5), err


@pytest.mark.parametrize("shape", OP_SHAPES)
def test_apply_data_and_llp_terms(ctx, torch_dev, shape):
    """The two terms of the matrix of eq. (Z_ini_matting) separately (llp_apply_data, llp_apply_llp)."""
    N, h, w, c, n, r = shape
    rng = rng_for(7, *shape)
    X, Y, u, P = scenes.random_problem(rng, N, h * c, w * c, c, n)
    lam, eps = 0.05, 1e-3
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=f32(lam), eps=f32(eps))
    Pd = dev(torch_dev, P)
    got_d = ctx.apply_data(Pd, dev(torch_dev, u), c=c, r=r)
    got_l = ctx.apply_llp(Pd, dev(torch_dev, Y), dev(torch_dev, u), c=c, r=r, lam=lam, eps=eps)
    # a window of one pixel (r = 0) gives M = 0: the LLP term is then 0 and is measured against ||A P||
    scale = np.linalg.norm(oracle.apply_A(P, prob).reshape(N, -1), axis=1)
    err_d = rel_l2(host(got_d), oracle.apply_data(P, prob))
    want_l = oracle.apply_llp(P, prob)
    err_l = (np.linalg.norm((host(got_l) - want_l).reshape(N, -1), axis=1)
             / np.maximum(np.linalg.norm(want_l.reshape(N, -1), axis=1), 1e-3 * scale))
    assert np.all(err_d < 1e-5), err_d
    assert np.all(err_l < 1e-5), err_l


@pytest.mark.parametrize("shape", OP_SHAPES[:4])
def test_objective(ctx, torch_dev, shape):
    N, h, w, c, n, r = shape
    rng = rng_for(4, *shape)
    X, Y, u, P = scenes.random_problem(rng, N, h * c, w * c, c, n)
    lam, eps = 0.05, 1e-3
    got = ctx.objective(dev(torch_dev, P), dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, u), r=r, lam=lam,
                        eps=eps)
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=f32(lam), eps=f32(eps))
    want = oracle.objective(P, X, prob)
    np.testing.assert_allclose(got, want, rtol=1e-6)


@pytest.fixture(scope="module")
def generic_ctx(torch_dev):
    import os
    os.environ["LLP_FORCE_GENERIC"] = "1"
    try:
        c = B.Context(0)
    finally:
        del os.environ["LLP_FORCE_GENERIC"]
    yield c
    c.close()


@pytest.mark.parametrize("shape", [(4, 64, 64, 4, 9, 1), (2, 24, 24, 4, 17, 2), (2, 20, 18, 2, 9, 1),
                                   (1, 12, 20, 4, 29, 1)])
def test_specialised_matches_generic(ctx, generic_ctx, torch_dev, shape):
    """The specialised kernels and the generic ones compute the same operator and the same CG iterates."""
    N, h, w, c, n, r = shape
    rng = rng_for(7, *shape)
    X, Y, u, P = scenes.random_problem(rng, N, h * c, w * c, c, n)
    d = {k: dev(torch_dev, v) for k, v in dict(X=X, Y=Y, u=u, P=P).items()}
    kw = dict(c=c, r=r, lam=0.05, eps=1e-3)
    a1 = host(ctx.apply_A(d["P"], d["Y"], d["u"], **kw))
    a2 = host(generic_ctx.apply_A(d["P"], d["Y"], d["u"], **kw))
    assert np.all(rel_l2(a1, a2) < 2e-6)
    skw = dict(r=r, lam=0.05, eps=1e-3, max_iters=25, tol=0.0)
    z1, _, _ = ctx.pansharpen(d["X"], d["Y"], d["u"], **skw)
    z2, _, _ = generic_ctx.pansharpen(d["X"], d["Y"], d["u"], **skw)
    assert np.all(rel_l2(host(z1), host(z2)) < 1e-5)


# ------------------------------------------------------------------------------------- the solve ---

@pytest.fixture(scope="module")
def scene0():
    sc, st = scenes.config_scene(0, 0)
    prob = Problem(u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=f32(st.lam), eps=f32(st.eps))
    b = oracle.rhs(sc.X, prob)
    return sc, st, prob, b


@pytest.fixture(scope="module")
def scene0_exact(scene0):
    sc, st, prob, b = scene0
    Z, _ = oracle.cg(prob, b, max_iters=5000, tol=1e-11)
    return Z


def run(ctx, torch, sc, st, **kw):
    args = dict(r=st.r, lam=st.lam, eps=st.eps, max_iters=st.max_iters, tol=st.tol)
    args.update(kw)
    return ctx.pansharpen(dev(torch, sc.X), dev(torch, sc.Y), dev(torch, sc.u), **args)


def test_cg_fixed_iterations_parity(ctx, torch_dev, scene0):
    """The 256^2 x 4 parity scene after exactly 50 iterations from Z = 0."""
    sc, st, prob, b = scene0
    Z, rep, status = run(ctx, torch_dev, sc, st)
    assert status == B.OK
    assert [r["iters"] for r in rep] == [50] * 4
    want, its = oracle.cg(prob, b, max_iters=50)
    assert list(its) == [50] * 4
    err = rel_l2(host(Z), want)
    assert np.all(err < 1e-5), err
    # the reported residuals and objective describe the returned iterate: out_rel_residual is the FP64 residual
    # of the float32 output (against the float32-rounded right-hand side the library holds), true_rel_residual
    # that of the iterate before the rounding (the same to a few float32 roundings at this residual level)
    true_rel = out_residual(prob, b, host(Z))
    np.testing.assert_allclose([r["out_rel_residual"] for r in rep], true_rel, rtol=1e-6)
    np.testing.assert_allclose([r["true_rel_residual"] for r in rep], true_rel, rtol=1e-3)
    np.testing.assert_allclose([r["objective"] for r in rep], oracle.objective(host(Z), sc.X, prob), rtol=1e-6)


def test_cg_tolerance_objective_parity(ctx, torch_dev, scene0, scene0_exact):
    """Run to ||b - A Z|| <= 1e-6 ||b||: the FP64 residual of the solver's iterate meets the tolerance, the
    float32 output's residual is what the oracle computes for it, and the objective matches the exact
    minimiser's to 1e-6."""
    sc, st, prob, b = scene0
    Z, rep, status = run(ctx, torch_dev, sc, st, max_iters=5000, tol=1e-6)
    assert status == B.OK
    assert all(r["true_rel_residual"] <= 1e-6 for r in rep), rep
    np.testing.assert_allclose([r["out_rel_residual"] for r in rep], out_residual(prob, b, host(Z)), rtol=1e-6)
    f_exact = oracle.objective(scene0_exact, sc.X, prob)
    f_gpu = oracle.objective(host(Z), sc.X, prob)
    assert np.all(np.abs(f_gpu - f_exact) / f_exact < 1e-6), (f_gpu, f_exact)
    np.testing.assert_allclose([r["objective"] for r in rep], f_gpu, rtol=1e-6)
    _, its = oracle.cg(prob, b, max_iters=5000, tol=1e-6)
    for r_, o in zip(rep, its):
        assert abs(r_["iters"] - o) <= max(8, 0.1 * o), (r_["iters"], o)


def test_warm_start_from_solution(ctx, torch_dev, scene0, scene0_exact):
    sc, st, prob, b = scene0
    init = dev(torch_dev, scene0_exact)
    Z, rep, status = run(ctx, torch_dev, sc, st, max_iters=5000, tol=1e-6, init=init)
    assert status == B.OK
    # the float32-rounded solution is a few float32 roundings away from meeting 1e-6: a few iterations remain
    assert all(r["iters"] <= 40 and r["true_rel_residual"] <= 1e-6 for r in rep), rep
    assert np.all(rel_l2(host(Z), scene0_exact) < 1e-5)


def test_deterministic(ctx, torch_dev, scene0):
    sc, st, _, _ = scene0
    Z1, r1, _ = run(ctx, torch_dev, sc, st)
    Z2, r2, _ = run(ctx, torch_dev, sc, st)
    assert torch_dev.equal(Z1, Z2)
    assert r1 == r2


def test_zero_iterations_and_zero_rhs(ctx, torch_dev, scene0):
    sc, st, _, _ = scene0
    Z, rep, status = run(ctx, torch_dev, sc, st, max_iters=0)
    assert status == B.OK and float(Z.abs().max()) == 0.0 and all(r["iters"] == 0 for r in rep)
    X0 = np.zeros_like(sc.X)
    Z, rep, status = ctx.pansharpen(dev(torch_dev, X0), dev(torch_dev, sc.Y), dev(torch_dev, sc.u), r=1, lam=0.01,
                                    eps=1e-3, max_iters=100, tol=1e-6)
    assert status == B.OK and float(Z.abs().max()) == 0.0 and all(r["iters"] == 0 for r in rep)


def test_not_converged_status(ctx, torch_dev, scene0):
    sc, st, _, _ = scene0
    Z, rep, status = run(ctx, torch_dev, sc, st, max_iters=3, tol=1e-6)
    assert status == B.NOT_CONVERGED
    assert all(r["iters"] == 3 and r["status"] == B.NOT_CONVERGED for r in rep)


def test_nonfinite_input(ctx, torch_dev, scene0):
    sc, st, _, _ = scene0
    Y = sc.Y.copy()
    Y[3, 7] = np.nan
    with pytest.raises(B.LlpError) as ei:
        ctx.pansharpen(dev(torch_dev, sc.X), dev(torch_dev, Y), dev(torch_dev, sc.u), r=1, lam=0.01, eps=1e-3,
                       max_iters=5, tol=0.0)
    assert ei.value.status == B.E_NONFINITE


@pytest.mark.parametrize("shape", [(1, 12, 10, 2, 5, 1), (3, 9, 9, 4, 13, 2), (2, 30, 30, 1, 3, 1)])
def test_small_shapes_fixed_iterations(ctx, torch_dev, shape):
    N, h, w, c, n, r = shape
    rng = rng_for(5, *shape)
    X, Y, u, _ = scenes.random_problem(rng, N, h * c, w * c, c, n)
    lam, eps = 0.05, 1e-2
    Z, rep, status = ctx.pansharpen(dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, u), r=r, lam=lam, eps=eps,
                                    max_iters=15, tol=0.0)
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=f32(lam), eps=f32(eps))
    want, _ = oracle.cg(prob, oracle.rhs(X, prob), max_iters=15)
    err = rel_l2(host(Z), want)
    assert np.all(err < 1e-5), err


# --------------------------------------------------------------------- full-size (2048^2 x 8) checks ---

@pytest.fixture(scope="module")
def scene1():
    return scenes.config_scene(1, 0)


def test_full_size_apply_sampled_bands(ctx, torch_dev, scene1):
    sc, st = scene1
    rng = rng_for(6)
    P = rng.standard_normal(sc.Z.shape).astype(np.float32)
    got = ctx.apply_A(dev(torch_dev, P), dev(torch_dev, sc.Y), dev(torch_dev, sc.u), c=sc.c, r=st.r, lam=st.lam,
                      eps=st.eps)
    prob = Problem(u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=f32(st.lam), eps=f32(st.eps))
    bands = [0, 5]
    want = oracle.apply_A(P[bands], prob)
    err = rel_l2(host(got[bands]), want)
    assert np.all(err < 1e-5), err


def test_full_size_solve_to_tolerance(ctx, torch_dev, scene1):
    """The 2048^2 x 8 scene to 1e-6: the returned HRMS has a small true residual (oracle-evaluated on sampled
    bands) and the reported objective is that of the returned HRMS."""
    sc, st = scene1
    Z, rep, status = run(ctx, torch_dev, sc, st)
    assert status == B.OK, rep
    assert all(r["true_rel_residual"] <= 1e-6 for r in rep), rep
    prob = Problem(u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=f32(st.lam), eps=f32(st.eps))
    bands = [1, 6]
    Zh = host(Z[bands])
    b = oracle.rhs(sc.X[bands], prob)
    np.testing.assert_allclose([rep[i]["out_rel_residual"] for i in bands], out_residual(prob, b, Zh), rtol=1e-5)
    f_out = oracle.objective(Zh, sc.X[bands], prob)
    np.testing.assert_allclose([rep[i]["objective"] for i in bands], f_out, rtol=1e-6)
    # the objective at the exact minimiser (FP64 CG to 1e-11, tests/golden/make_scene_objectives.py)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "scene_objectives.json")))
    for i, band in enumerate(bands):
        f_exact = gold["bands"][str(band)]["objective"]
        assert abs(f_out[i] - f_exact) / f_exact < 1e-6, (band, f_out[i], f_exact)
