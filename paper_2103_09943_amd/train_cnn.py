"""Train the warm-start network on the GPU and measure what it saves.

    python -m paper_2103_09943_amd.train_cnn [--train 2000] [--eval 500] [--epochs 40] [--lr 2e-3] [--out PATH]

1. Synthetic training scenes (4 bands, 256^2 PAN, the batch workload's blur recipe) and their plain-solver HRMS
   (cold start, tolerance 1e-6) as targets.
2. Adam on the mean squared error of the network output against the normalised residual of the target over the
   bicubic upsampling, one scene per step, cosine-decayed step size; all forward and backward work runs in the
   library's kernels.
3. Held-out scenes (8 bands, 512^2) solved to 1e-6 from Z = 0, from the bicubic upsampling (the network with a
   zero last layer) and from the trained network: iterations per band and wall time of the batched solve.
The trained parameters are saved as a float32 .npy file, and a JSON summary next to it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import binding as B
from . import scenes

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "cnn_warm_start.npy")


def _gen(args):
    s, side = args
    sc, st = scenes.config_scene(3, s, side=side)
    return sc.X, sc.Y, sc.u


def generate(ids, side, workers):
    with ProcessPoolExecutor(workers) as ex:
        return list(ex.map(_gen, [(s, side) for s in ids], chunksize=8))


def to_dev(torch, host):
    return [tuple(torch.from_numpy(a).cuda() for a in sc) for sc in host]


def solve_all(ctx, ds, chunk, **kw):
    """Batched solves in chunks of scenes; returns outputs, per-scene reports, seconds."""
    import torch
    outs, reps = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(0, len(ds), chunk):
        o, r, _ = ctx.pansharpen_batch(ds[i:i + chunk], **kw)
        outs += o
        reps += r
    torch.cuda.synchronize()
    return outs, reps, time.perf_counter() - t0


def evaluate(ctx, ds, flat, chunk, settings):
    """Cold, bicubic and network starts on the same scenes (the network's weights restored at the end)."""
    kw = dict(r=settings.r, lam=settings.lam, eps=settings.eps, max_iters=settings.max_iters, tol=settings.tol)
    res = {}
    bicubic = flat.copy()
    n_last = 32 * 9 + 1
    bicubic[-n_last:] = 0.0
    for name, weights, init in (("cold", None, None), ("bicubic", bicubic, "cnn"), ("network", flat, "cnn")):
        if weights is not None:
            ctx.cnn_set_weights(weights)
        solve_all(ctx, ds[:min(chunk, len(ds))], chunk, inits=init, **kw)  # warm-up (graphs, workspaces)
        _, reps, secs = solve_all(ctx, ds, chunk, inits=init, **kw)
        its = [r["iters"] for rs in reps for r in rs]
        res[name] = {
            "seconds": secs,
            "iters_mean": float(np.mean(its)),
            "iters_min": int(np.min(its)),
            "iters_max": int(np.max(its)),
            "rejected_bands": int(sum(r["init"] == B.INIT_NET_REJECTED for rs in reps for r in rs)),
            "max_rel_residual": float(max(r["rel_residual"] for rs in reps for r in rs)),
        }
    ctx.cnn_set_weights(flat)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--eval", type=int, default=500)
    ap.add_argument("--train-side", type=int, default=None)
    ap.add_argument("--eval-side", type=int, default=None)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--chunk", type=int, default=128, help="scenes per batched solve")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args()
    import torch

    t0 = time.perf_counter()
    train_host = generate(range(args.train), args.train_side, args.workers)
    print(f"generated {len(train_host)} training scenes in {time.perf_counter() - t0:.1f} s", flush=True)
    _, st = scenes.config_scene(3, 0, side=64)
    ctx = B.Context(0)
    ctx.tune_load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "gfx950.json"))
    train = to_dev(torch, train_host)
    targets, treps, secs = solve_all(ctx, train, args.chunk, r=st.r, lam=st.lam, eps=st.eps,
                                     max_iters=st.max_iters, tol=st.tol)
    print(f"plain-solver targets: {secs:.1f} s, mean iterations "
          f"{np.mean([r['iters'] for rs in treps for r in rs]):.1f}", flush=True)

    flat = scenes.cnn_init_params(np.random.default_rng(np.random.SeedSequence([2103, 9943])), last_std=1e-3)
    ctx.cnn_set_weights(flat)
    steps = args.epochs * len(train)
    rng = np.random.default_rng(np.random.SeedSequence([2103, 1]))
    log = []
    step = 0
    t_train = time.perf_counter()
    for ep in range(args.epochs):
        losses = []
        for s in rng.permutation(len(train)):
            lr = args.lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * step / steps)))
            X, Y, _ = train[s]
            want = step % 50 == 0
            loss = ctx.cnn_train_step(X, Y, targets[s], c=4, lr=lr, want_loss=want)
            if want:
                losses.append(loss)
            step += 1
        torch.cuda.synchronize()
        log.append({"epoch": ep, "mean_sampled_loss": float(np.mean(losses)),
                    "seconds": time.perf_counter() - t_train})
        print(json.dumps(log[-1]), flush=True)
    train_secs = time.perf_counter() - t_train
    trained = ctx.cnn_get_weights()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, trained)
    del train, targets

    t0 = time.perf_counter()
    eval_host = generate(range(2000, 2000 + args.eval), args.eval_side, args.workers)
    print(f"generated {len(eval_host)} evaluation scenes in {time.perf_counter() - t0:.1f} s", flush=True)
    ev = to_dev(torch, eval_host)
    _, st_e = scenes.config_scene(3, 2000, side=64)
    res = evaluate(ctx, ev, trained, args.chunk, st_e)
    pxb = sum(X.shape[0] * Y.numel() for X, Y, _ in ev)
    summary = {
        "train_scenes": args.train, "train_shape": list(train_host[0][0].shape) + list(train_host[0][1].shape),
        "epochs": args.epochs, "train_steps": steps, "train_seconds": train_secs, "log": log,
        "eval_scenes": args.eval, "eval_shape": list(eval_host[0][0].shape) + list(eval_host[0][1].shape),
        "eval_mpixel_bands": pxb / 1e6,
        "results": {k: dict(v, mpixel_bands_per_s=pxb / v["seconds"] / 1e6) for k, v in res.items()},
    }
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps(summary["results"]), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
