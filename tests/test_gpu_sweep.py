"""GPU: the column-sweep operator variant (the LLP term, and for c = 4 the data term on the matrix cores inside the
sweep; for c = 2 a separate data-term launch) against the oracle.

The variant is forced with LLP_APPLY_VARIANT=2 (and segment lengths with LLP_SEG_ROWS) so that it is exercised
on small, ragged shapes too: strips of 52 (r = 2) or 56 (r = 1) output columns and segments of 32..96 rows,
neither dividing the image, plus images only a few segments tall.  Bars as in the other parity tests: the
operator to relative L2 <= 1e-5 per band, the CG iterate after a fixed count to 1e-5, and bit-identical results
between the single-scene and the batched launches of the same kernels.
"""
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


def make_ctx(seg_rows, dir_rows=None):
    env = {"LLP_APPLY_VARIANT": "2", "LLP_SEG_ROWS": str(seg_rows)}
    if dir_rows is not None:
        env["LLP_DIR_ROWS"] = str(dir_rows)
    os.environ.update(env)
    try:
        return B.Context(0)
    finally:
        for k in env:
            del os.environ[k]


@pytest.fixture(scope="module", params=[32, 96])
def sweep_ctx(request, torch_dev):
    c = make_ctx(request.param)
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


SHAPES = [  # N, h, w, c, n, r  (H = c h >= 3 (2r + 2) rows)
    (2, 20, 18, 2, 9, 1),
    (1, 16, 40, 2, 17, 2),
    (3, 24, 24, 4, 11, 2),
    (1, 9, 33, 4, 15, 1),     # W = 132: 3 strips, the last one ragged
    (5, 40, 16, 4, 17, 2),    # five bands: two waves of a workgroup idle
    (2, 64, 64, 4, 9, 1),
    (2, 20, 24, 4, 13, 1),    # n 13: the c = 4 classes with a 4 x 4 y neighbourhood
    (1, 16, 20, 4, 29, 2),    # n 29: an 8 x 8 neighbourhood, 16 K steps of the matrix-core product
]


@pytest.mark.parametrize("shape", SHAPES)
def test_sweep_apply_matches_oracle(sweep_ctx, torch_dev, shape):
    N, h, w, c, n, r = shape
    rng = np.random.default_rng(np.random.SeedSequence([61, *shape]))
    X, Y, u, P = scenes.random_problem(rng, N, h * c, w * c, c, n)
    lam, eps = 0.05, 1e-3
    got = sweep_ctx.apply_A(dev(torch_dev, P), dev(torch_dev, Y), dev(torch_dev, u), c=c, r=r, lam=lam, eps=eps)
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=f32(lam), eps=f32(eps))
    err = rel_l2(host(got), oracle.apply_A(P, prob))
    assert np.all(err < 1e-5), err


@pytest.mark.parametrize("shape", SHAPES)
def test_sweep_terms_match_oracle(sweep_ctx, torch_dev, shape):
    """The data term and the LLP term separately through the sweep's launch configuration."""
    N, h, w, c, n, r = shape
    rng = np.random.default_rng(np.random.SeedSequence([63, *shape]))
    X, Y, u, P = scenes.random_problem(rng, N, h * c, w * c, c, n)
    lam, eps = 0.05, 1e-3
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=f32(lam), eps=f32(eps))
    Pd = dev(torch_dev, P)
    err_d = rel_l2(host(sweep_ctx.apply_data(Pd, dev(torch_dev, u), c=c, r=r)), oracle.apply_data(P, prob))
    err_l = rel_l2(host(sweep_ctx.apply_llp(Pd, dev(torch_dev, Y), dev(torch_dev, u), c=c, r=r, lam=lam, eps=eps)),
                   oracle.apply_llp(P, prob))
    assert np.all(err_d < 1e-5), err_d
    assert np.all(err_l < 1e-5), err_l


@pytest.mark.parametrize("shape", SHAPES[:4])
def test_sweep_cg_matches_oracle(sweep_ctx, torch_dev, shape):
    N, h, w, c, n, r = shape
    rng = np.random.default_rng(np.random.SeedSequence([62, *shape]))
    X, Y, u, _ = scenes.random_problem(rng, N, h * c, w * c, c, n)
    lam, eps = 0.05, 1e-2
    Z, rep, status = sweep_ctx.pansharpen(dev(torch_dev, X), dev(torch_dev, Y), dev(torch_dev, u), r=r, lam=lam,
                                          eps=eps, max_iters=20, tol=0.0)
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=f32(lam), eps=f32(eps))
    want, _ = oracle.cg(prob, oracle.rhs(X, prob), max_iters=20)
    assert np.all(rel_l2(host(Z), want) < 1e-5)


def test_sweep_parity_scene_50_iterations(torch_dev):
    """The 256^2 x 4 parity scene after exactly 50 iterations, on the split kernels."""
    sc, st = scenes.config_scene(0, 0)
    prob = Problem(u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=f32(st.lam), eps=f32(st.eps))
    with make_ctx(64) as ctx:
        Z, rep, status = ctx.pansharpen(dev(torch_dev, sc.X), dev(torch_dev, sc.Y), dev(torch_dev, sc.u), r=st.r,
                                        lam=st.lam, eps=st.eps, max_iters=50, tol=0.0)
    want, _ = oracle.cg(prob, oracle.rhs(sc.X, prob), max_iters=50)
    assert status == B.OK and np.all(rel_l2(host(Z), want) < 1e-5)


def test_sweep_batch_matches_single(torch_dev):
    host_sc = [scenes.config_scene(2, s, side=side)[0] for s, side in enumerate([96, 128, 160, 104])]
    ds = [tuple(dev(torch_dev, a) for a in (sc.X, sc.Y, sc.u)) for sc in host_sc]
    kw = dict(r=1, lam=1e-2, eps=1e-3, max_iters=300, tol=1e-6)
    with make_ctx(32) as ctx:
        outs, reps, _ = ctx.pansharpen_batch(ds, **kw)
        for (X, Y, u), Z, rs in zip(ds, outs, reps):
            Zs, rs_s, _ = ctx.pansharpen(X, Y, u, **kw)
            assert torch_dev.equal(Z, Zs) and rs == rs_s


@pytest.mark.parametrize("shape", [(2, 40, 40, 4, 17, 2), (1, 48, 36, 4, 9, 1), (2, 40, 40, 2, 9, 1)])
def test_eight_row_update_tiles(torch_dev, shape):
    """The update kernel's 8-row tiles (8 waves of 512 threads, one LR row each): the CG iterate after a fixed
    count matches the oracle, and the batched launch reproduces the single-scene one bit for bit."""
    N, h, w, c, n, r = shape
    rng = np.random.default_rng(np.random.SeedSequence([63, *shape]))
    X, Y, u, _ = scenes.random_problem(rng, N, h * c, w * c, c, n)
    lam, eps = 0.05, 1e-2
    d = tuple(dev(torch_dev, a) for a in (X, Y, u))
    with make_ctx(32, dir_rows=8) as ctx:
        Z, _, _ = ctx.pansharpen(*d, r=r, lam=lam, eps=eps, max_iters=20, tol=0.0)
        outs, _, _ = ctx.pansharpen_batch([d, d], r=r, lam=lam, eps=eps, max_iters=20, tol=0.0)
    prob = Problem(u=u, c=c, Y=Y, r=r, lam=f32(lam), eps=f32(eps))
    want, _ = oracle.cg(prob, oracle.rhs(X, prob), max_iters=20)
    assert np.all(rel_l2(host(Z), want) < 1e-5)
    for o in outs:
        assert torch_dev.equal(o, Z)
