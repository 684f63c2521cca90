"""GPU: the batched solve (llp_pansharpen_batch) of many scenes of different sizes at once.

Every band of every scene is the same CG as a single-scene solve (the batched kernels run the same tile code in
the same order, and the reductions add in the same order), so the batch must reproduce the single-scene
results bit for bit, iteration counts included; the single-scene path itself is held to the FP64 oracle
elsewhere, and here once more directly on the batch (relative L2 <= 1e-5 per band after 50 iterations).
The scene mix follows the batch workload's recipe (PAN sides, 4 or 8 bands, kernels of 9..17 taps, r = 1) at
reduced sides, plus one scene whose (c, n) has no specialised kernels.
"""
import numpy as np
import pytest

import oracle
from oracle.llp import Problem
from paper_2103_09943_amd import binding as B
from paper_2103_09943_amd import scenes

pytestmark = pytest.mark.gpu

SIDES = [64, 96, 128, 72, 160, 100, 88, 64]
R, LAM, EPS = 1, 1e-2, 1e-3


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


def make_batch(seed_offset=0):
    """Host scenes: (X, Y, u, c) tuples."""
    out = []
    for s, side in enumerate(SIDES):
        sc, _ = scenes.config_scene(2, s + seed_offset, side=side)
        out.append((sc.X, sc.Y, sc.u, sc.c))
    rng = np.random.default_rng(np.random.SeedSequence([12, seed_offset]))
    X, Y, u, _ = scenes.random_problem(rng, 3, 40, 36, 2, 5)  # c = 2, n = 5: generic kernels
    out.append((X, Y, u, 2))
    return out


@pytest.fixture(scope="module")
def batch_host():
    return make_batch()


def to_dev(torch, batch):
    return [(dev(torch, X), dev(torch, Y), dev(torch, u)) for X, Y, u, _ in batch]


def single_solves(ctx, dscenes, **kw):
    outs, reps = [], []
    for X, Y, u in dscenes:
        Z, rep, _ = ctx.pansharpen(X, Y, u, r=R, lam=LAM, eps=EPS, **kw)
        outs.append(Z)
        reps.append(rep)
    return outs, reps


def assert_same(torch, got, want, grep, wrep):
    for i, (a, b) in enumerate(zip(got, want)):
        assert torch.equal(a, b), f"scene {i}: max |diff| {float((a - b).abs().max())}"
    assert grep == wrep


def test_batch_matches_single_fixed_iterations(ctx, torch_dev, batch_host):
    ds = to_dev(torch_dev, batch_host)
    outs, reps, status = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=30, tol=0.0)
    assert status == B.OK
    assert all(r["iters"] == 30 for rs in reps for r in rs)
    want, wreps = single_solves(ctx, ds, max_iters=30, tol=0.0)
    assert_same(torch_dev, outs, want, reps, wreps)


def test_batch_matches_single_to_tolerance(ctx, torch_dev, batch_host):
    ds = to_dev(torch_dev, batch_host)
    outs, reps, status = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=5000, tol=1e-6)
    assert status == B.OK
    assert all(r["true_rel_residual"] <= 1e-6 and r["status"] == B.OK for rs in reps for r in rs)
    its = sorted({r["iters"] for rs in reps for r in rs})
    assert len(its) > 3, its  # the bands stop at different iterations
    want, wreps = single_solves(ctx, ds, max_iters=5000, tol=1e-6)
    assert_same(torch_dev, outs, want, reps, wreps)


def test_batch_oracle_parity(ctx, torch_dev, batch_host):
    """Each scene of the batch after exactly 50 iterations against the FP64 oracle's CG."""
    ds = to_dev(torch_dev, batch_host)
    outs, reps, status = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=50, tol=0.0)
    assert status == B.OK
    for (X, Y, u, c), Z in zip(batch_host[:4] + batch_host[-1:], outs[:4] + outs[-1:]):
        prob = Problem(u=u, c=c, Y=Y, r=R, lam=f32(LAM), eps=f32(EPS))
        want, _ = oracle.cg(prob, oracle.rhs(X, prob), max_iters=50)
        err = rel_l2(host(Z), want)
        assert np.all(err < 1e-5), err


@pytest.mark.parametrize("flags", [B.BATCH_NO_GRAPH, B.BATCH_SERIAL])
def test_batch_flags_agree(ctx, torch_dev, batch_host, flags):
    ds = to_dev(torch_dev, batch_host)
    g_outs, g_reps, _ = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=200, tol=1e-5)
    outs, reps, _ = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=200, tol=1e-5, flags=flags)
    assert_same(torch_dev, outs, g_outs, reps, g_reps)


def test_batch_graph_reuse_new_inputs(ctx, torch_dev):
    """Same shapes, new inputs: the cached graph is replayed over the new scene table; eager device work
    between the calls; every call checked against single-scene solves."""
    for off in (100, 200, 100):
        batch = make_batch(off)
        ds = to_dev(torch_dev, batch)
        noise = torch_dev.randn(1 << 20, device="cuda")
        noise.mul_(2.0).sum().item()
        outs, reps, _ = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=300, tol=1e-6)
        want, wreps = single_solves(ctx, ds, max_iters=300, tol=1e-6)
        assert_same(torch_dev, outs, want, reps, wreps)


def test_batch_iteration_cap_not_multiple_of_chunk(ctx, torch_dev, batch_host):
    ds = to_dev(torch_dev, batch_host)
    outs, reps, status = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=13, tol=1e-6)
    assert status == B.NOT_CONVERGED
    assert all(r["iters"] == 13 and r["status"] == B.NOT_CONVERGED for rs in reps for r in rs)
    want, wreps = single_solves(ctx, ds, max_iters=13, tol=1e-6)
    assert_same(torch_dev, outs, want, reps, wreps)


def test_batch_warm_start(ctx, torch_dev, batch_host):
    ds = to_dev(torch_dev, batch_host)
    sol, cold, _ = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=5000, tol=1e-7)
    outs, reps, status = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=5000, tol=1e-6,
                                              inits=[z.clone() for z in sol])
    assert status == B.OK
    # from a converged start only the float32 rounding of the start is left to remove
    assert all(r["iters"] <= 8 and r["iters"] * 5 < c["iters"]
               for rs, cs in zip(reps, cold) for r, c in zip(rs, cs)), reps
    want, wreps = single_solves(ctx, ds, max_iters=5000, tol=1e-6, init=None)
    for a, b in zip(outs, want):
        assert np.all(rel_l2(host(a), host(b)) < 1e-5)


def test_batch_empty_and_zero_iterations(ctx, torch_dev, batch_host):
    outs, reps, status = ctx.pansharpen_batch([], r=R, lam=LAM, eps=EPS, max_iters=10)
    assert status == B.OK and outs == [] and reps == []
    ds = to_dev(torch_dev, batch_host)
    outs, reps, status = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=0)
    assert status == B.OK
    assert all(float(z.abs().max()) == 0.0 for z in outs)
    assert all(r["iters"] == 0 for rs in reps for r in rs)


def test_batch_nonfinite_scene(ctx, torch_dev, batch_host):
    ds = to_dev(torch_dev, batch_host)
    X, Y, u = ds[2]
    Y = Y.clone()
    Y[5, 5] = float("nan")
    ds[2] = (X, Y, u)
    with pytest.raises(B.LlpError) as ei:
        ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=5)
    assert ei.value.status == B.E_NONFINITE


def test_batch_timed_launches_agree(ctx, torch_dev, batch_host):
    """With kernel timing on, the batch runs its kernels eagerly between events: same results, times counted."""
    ds = to_dev(torch_dev, batch_host)
    g_outs, g_reps, _ = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=40, tol=1e-6)
    ctx.set_profiling(True)
    ctx.kernel_times(reset=True)
    try:
        outs, reps, _ = ctx.pansharpen_batch(ds, r=R, lam=LAM, eps=EPS, max_iters=40, tol=1e-6)
        kt = ctx.kernel_times(reset=True)
    finally:
        ctx.set_profiling(False)
    assert_same(torch_dev, outs, g_outs, reps, g_reps)
    assert kt["apply_launches"] > 0 and kt["apply_ms"] > 0 and kt["dir_ms"] > 0
