"""llp_apply_A_noalloc (the product with the matrix of eq. (Z_ini_matting) for callers that cannot allocate)
against llp_apply_A on the same inputs, and both against the FP64 oracle: two calls in a row, the second on a
smaller scene (the library's fixed device array then still holds the first call's contents), and the rejection
of a scene whose statistics do not fit the array."""
import numpy as np
import pytest

import oracle
from oracle.llp import Problem
from paper_2103_09943_amd import binding as B
from paper_2103_09943_amd import scenes

pytestmark = pytest.mark.gpu

# (N, h, w, c, n, r): a 512^2 scene, then a smaller ragged one whose H W is not a multiple of 64
CALLS = [(4, 128, 128, 4, 9, 2), (2, 37, 29, 2, 11, 1)]


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _rel(got, want):
    N = want.shape[0]
    return np.linalg.norm((got - want).reshape(N, -1), axis=1) / np.linalg.norm(want.reshape(N, -1), axis=1)


def test_noalloc_matches_apply_A():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = B.Context(0)
    try:
        lam, eps = 0.05, 1e-3
        for k, (N, h, w, c, n, r) in enumerate(CALLS):
            print(f"noalloc call {k}: N={N} h={h} w={w} c={c} n={n} r={r}", flush=True)
            rng = np.random.default_rng(np.random.SeedSequence([23, k, N, h, w, c, n, r]))
            X, Y, u, P = scenes.random_problem(rng, N, h * c, w * c, c, n)
            Pd, Yd, ud = _dev(torch, P), _dev(torch, Y), _dev(torch, u)
            out = torch.full_like(Pd, float("nan"))
            got = B.apply_A_noalloc(Pd, Yd, ud, c=c, r=r, lam=lam, eps=eps, out=out)
            ref = ctx.apply_A(Pd, Yd, ud, c=c, r=r, lam=lam, eps=eps)
            torch.cuda.synchronize()
            g = got.cpu().numpy().astype(np.float64)
            e = ref.cpu().numpy().astype(np.float64)
            assert np.all(np.isfinite(g))
            prob = Problem(u=u, c=c, Y=Y, r=r, lam=float(np.float32(lam)), eps=float(np.float32(eps)))
            want = oracle.apply_A(P, prob)
            # the same kernels in the same configuration as a fresh context's llp_apply_A
            assert np.all(_rel(g, e) < 1e-6), _rel(g, e)
            assert np.all(_rel(g, want) < 1e-5), _rel(g, want)
    finally:
        ctx.close()


def test_noalloc_rejects_oversized_scene():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    # 3 H W floats of PAN statistics for a 4096^2 scene exceed the array
    z = torch.zeros((1, 4096, 4096), device="cuda")
    pan = torch.zeros((4096, 4096), device="cuda")
    u = torch.full((9, 9), 1.0 / 81, device="cuda")
    with pytest.raises(B.LlpError) as ei:
        B.apply_A_noalloc(z, pan, u, c=4, r=1, lam=0.05, eps=1e-3, out=torch.empty_like(z))
    assert ei.value.status == B.E_UNSUPPORTED
