"""GPU: the launch-configuration autotuners (llp_autotune, llp_autotune_batch) and their JSON table.

The tuner must pick one of the configurations it timed, no slower than the default; solves after tuning still
meet the oracle bar (the tile shape changes only the order of float32 operations); a saved table reloads to the
same choice; a table made for another architecture or an unreadable one is refused.
"""
import json

import numpy as np
import pytest

import oracle
from oracle.llp import Problem
from paper_2103_09943_amd import binding as B
from paper_2103_09943_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel_l2(got, want):
    got = got.reshape(got.shape[0], -1)
    want = want.reshape(want.shape[0], -1)
    return np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)


@pytest.fixture(scope="module")
def scene(torch_dev):
    sc, st = scenes.config_scene(2, 3, side=192)
    return sc, st, tuple(dev(torch_dev, a) for a in (sc.X, sc.Y, sc.u))


def test_autotune_choice_and_parity(torch_dev, scene, tmp_path):
    sc, st, (X, Y, u) = scene
    with B.Context(0) as ctx:
        assert ctx.tune_count() == 0
        res = ctx.autotune(X, Y, u, r=st.r, lam=st.lam, eps=st.eps, iters=6)
        assert res["candidates"] >= 1 and res["fast"] == 1
        assert res["dir_rows"] in (4, 8) and res["apply_variant"] in (0, 1, 2) and res["seg_rows"] >= 32
        assert 0 < res["us_per_iter"] <= res["default_us_per_iter"]
        assert ctx.tune_count() == 1
        Z, rep, _ = ctx.pansharpen(X, Y, u, r=st.r, lam=st.lam, eps=st.eps, max_iters=40, tol=0.0)
        prob = Problem(u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=float(np.float32(st.lam)),
                       eps=float(np.float32(st.eps)))
        want, _ = oracle.cg(prob, oracle.rhs(sc.X, prob), max_iters=40)
        assert np.all(rel_l2(Z.cpu().numpy().astype(np.float64), want) < 1e-5)
        path = str(tmp_path / "tune.json")
        ctx.tune_save(path)
        rec = json.load(open(path))
        assert rec["arch"].startswith("gfx") and len(rec["entries"]) == 1
        e = rec["entries"][0]
        assert (e["dir_rows"], e["apply_variant"]) == (res["dir_rows"], res["apply_variant"])
    with B.Context(0) as ctx2:
        ctx2.tune_load(path)
        assert ctx2.tune_count() == 1
        Z2, _, _ = ctx2.pansharpen(X, Y, u, r=st.r, lam=st.lam, eps=st.eps, max_iters=40, tol=0.0)
        assert torch_dev.equal(Z, Z2)  # same configuration, same result bits
        ctx2.tune_clear()
        assert ctx2.tune_count() == 0


def test_tune_load_refuses_other_arch_and_garbage(torch_dev, tmp_path):
    other = tmp_path / "other.json"
    other.write_text(json.dumps({"arch": "gfx000", "entries": [
        {"c": 4, "R": 4, "r": 1, "bucket": 30, "fast": 1, "dir_rows": 4, "apply_variant": 1}]}))
    bad = tmp_path / "bad.json"
    bad.write_text('{"arch": "gfx950", "entries": [{"c": 4}]}')
    with B.Context(0) as ctx:
        with pytest.raises(B.LlpError) as ei:
            ctx.tune_load(str(other))
        assert ei.value.status == B.E_UNSUPPORTED
        with pytest.raises(B.LlpError) as ei:
            ctx.tune_load(str(bad))
        assert ei.value.status in (B.E_ARG, B.E_UNSUPPORTED)
        with pytest.raises(B.LlpError):
            ctx.tune_load(str(tmp_path / "missing.json"))
        assert ctx.tune_count() == 0


def test_batch_autotune_flag(torch_dev):
    """LLP_BATCH_AUTOTUNE tunes every class of the batch once, as batched entries; the batch still solves every
    band to the tolerance, to the objective of single-scene solves, and a repeat reproduces it bit for bit."""
    host = [scenes.config_scene(2, s, side=side)[0] for s, side in enumerate([96, 128, 160, 96])]
    ds = [tuple(dev(torch_dev, a) for a in (sc.X, sc.Y, sc.u)) for sc in host]
    kw = dict(r=1, lam=1e-2, eps=1e-3, max_iters=300, tol=1e-6)
    with B.Context(0) as ctx:
        outs, reps, _ = ctx.pansharpen_batch(ds, flags=B.BATCH_AUTOTUNE, **kw)
        n = ctx.tune_count()
        assert 1 <= n <= len(host)
        outs2, reps2, _ = ctx.pansharpen_batch(ds, flags=B.BATCH_AUTOTUNE, **kw)
        assert ctx.tune_count() == n  # nothing left to tune
        for a, b in zip(outs, outs2):
            assert torch_dev.equal(a, b)
        assert reps == reps2
        for (X, Y, u), rs in zip(ds, reps):
            _, rs_s, _ = ctx.pansharpen(X, Y, u, **kw)
            assert all(r["true_rel_residual"] <= 1e-6 for r in rs)
            np.testing.assert_allclose([r["objective"] for r in rs], [r["objective"] for r in rs_s], rtol=1e-6)


def test_autotune_batch_entry(torch_dev, scene, tmp_path):
    """llp_autotune_batch keeps a batched entry of the class (saved with "batched": 1) and leaves single-scene
    solves on their own choice; a batch after reloading the table reproduces the batch bit for bit, and its
    bands meet the oracle bar at a fixed iteration count."""
    sc, st, (X, Y, u) = scene
    with B.Context(0) as ctx:
        Zs0, _, _ = ctx.pansharpen(X, Y, u, r=st.r, lam=st.lam, eps=st.eps, max_iters=40, tol=0.0)
        res = ctx.autotune_batch(X, Y, u, r=st.r, lam=st.lam, eps=st.eps, iters=4, copies=4)
        assert res["fast"] == 1 and res["candidates"] >= 2
        assert res["dir_rows"] in (4, 8) and res["apply_variant"] in (0, 1, 2) and res["seg_rows"] >= 32
        assert 0 < res["us_per_iter"] <= res["default_us_per_iter"]
        assert ctx.tune_count() == 1
        Zs1, _, _ = ctx.pansharpen(X, Y, u, r=st.r, lam=st.lam, eps=st.eps, max_iters=40, tol=0.0)
        assert torch_dev.equal(Zs0, Zs1)  # single-scene solves do not use the batched entry
        outs, _, _ = ctx.pansharpen_batch([(X, Y, u)] * 2, r=st.r, lam=st.lam, eps=st.eps, max_iters=40, tol=0.0)
        prob = Problem(u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=float(np.float32(st.lam)),
                       eps=float(np.float32(st.eps)))
        want, _ = oracle.cg(prob, oracle.rhs(sc.X, prob), max_iters=40)
        for Z in outs:
            assert np.all(rel_l2(Z.cpu().numpy().astype(np.float64), want) < 1e-5)
        path = str(tmp_path / "tune_batch.json")
        ctx.tune_save(path)
        rec = json.load(open(path))
        assert [e["batched"] for e in rec["entries"]] == [1]
        assert rec["entries"][0]["apply_variant"] == res["apply_variant"]
    with B.Context(0) as ctx2:
        ctx2.tune_load(path)
        outs2, _, _ = ctx2.pansharpen_batch([(X, Y, u)] * 2, r=st.r, lam=st.lam, eps=st.eps, max_iters=40, tol=0.0)
        for a, b in zip(outs, outs2):
            assert torch_dev.equal(a, b)
