"""GPU: what the trained warm-start network gains over the solve without it.

The committed parameters (paper_2103_09943_amd/weights/cnn_warm_start.npy) were trained on the GPU by
paper_2103_09943_amd.train_cnn on 2000 synthetic 4-band 256^2 scenes against plain-solver outputs.  On held-out
8-band 512^2 scenes, the solve to the same tolerance must need fewer CG iterations from the network's estimate
than from Z = 0 and than from the bicubic upsampling alone, and reach the same objective.  The size of the gain is
a property of the trained weights (parity unpinned: training is stochastic); the bar here is a strict gain.
"""
import os

import numpy as np
import pytest

from paper_2103_09943_amd import binding as B
from paper_2103_09943_amd import scenes

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2103_09943_amd",
                       "weights", "cnn_warm_start.npy")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def test_trained_network_saves_iterations(torch_dev):
    assert os.path.exists(WEIGHTS), "trained parameters are missing"
    flat = np.load(WEIGHTS)
    host = [scenes.config_scene(3, s)[0] for s in range(2000, 2004)]
    ds = [tuple(torch_dev.from_numpy(a).cuda() for a in (sc.X, sc.Y, sc.u)) for sc in host]
    _, st = scenes.config_scene(3, 2000, side=64)
    kw = dict(r=st.r, lam=st.lam, eps=st.eps, max_iters=st.max_iters, tol=st.tol)
    bicubic = flat.copy()
    bicubic[-(32 * 9 + 1):] = 0.0
    with B.Context(0) as ctx:
        _, cold, _ = ctx.pansharpen_batch(ds, **kw)
        ctx.cnn_set_weights(bicubic)
        _, bic, _ = ctx.pansharpen_batch(ds, inits="cnn", **kw)
        ctx.cnn_set_weights(flat)
        _, net, status = ctx.pansharpen_batch(ds, inits="cnn", **kw)
    assert status == B.OK
    it = {k: np.mean([r["iters"] for rs in v for r in rs]) for k, v in
          dict(cold=cold, bicubic=bic, network=net).items()}
    assert it["network"] < it["bicubic"] < it["cold"], it
    assert it["network"] < 0.95 * it["cold"], it
    assert all(r["init"] == B.INIT_NET for rs in net for r in rs)
    for rs_n, rs_c in zip(net, cold):
        np.testing.assert_allclose([r["objective"] for r in rs_n], [r["objective"] for r in rs_c], rtol=1e-6)
