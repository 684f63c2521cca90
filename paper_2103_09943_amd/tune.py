"""Build the launch-configuration table for the benchmark workloads on this device and save it as JSON.

    python -m paper_2103_09943_amd.tune [--out PATH]

Tunes the 16-band 4096^2 scene of the large workload and the 8-band 2048^2 scene (r 2, 17 taps), and one
synthetic scene of every (PAN side, kernel size) class of
the batch workload (sides 256..1024 in steps of 128, 9..17 taps, r 1), each for single-scene solves and for
batched solves (on a batch of copies of the scene).  The library keys the table by (c, n, r)
and the image area in half-octaves, and refuses a table made on another architecture.
"""
from __future__ import annotations

import argparse
import json
import os

from . import binding as B
from . import scenes

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "gfx950.json")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--iters", type=int, default=16)
    args = ap.parse_args()
    import numpy as np
    import torch

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()

    jobs = []
    sc, st = scenes.config_scene(4, 0)
    jobs.append(("16x4096^2 n17 r2", sc, st))
    sc, st = scenes.config_scene(1, 0)
    jobs.append(("8x2048^2 n17 r2", sc, st))
    for side in range(256, 1025, 128):
        for n in range(9, 18, 2):
            rng = np.random.default_rng(np.random.SeedSequence([7, side, n]))
            u = scenes.gaussian_kernel(n, 1.75)
            s2 = scenes.make_scene(rng, side, side, 4, 4, u)
            jobs.append((f"4x{side}^2 n{n} r1", s2, scenes.SolveSettings(r=1, lam=1e-2, eps=1e-3, max_iters=8,
                                                                          tol=0.0)))
    with B.Context(0) as ctx:
        for name, s, stt in jobs:
            d = (dev(s.X), dev(s.Y), dev(s.u))
            res = ctx.autotune(*d, r=stt.r, lam=stt.lam, eps=stt.eps, iters=args.iters)
            print(json.dumps({"scene": name, "mode": "single", **res}), flush=True)
            res = ctx.autotune_batch(*d, r=stt.r, lam=stt.lam, eps=stt.eps, iters=args.iters)
            print(json.dumps({"scene": name, "mode": "batched", **res}), flush=True)
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        ctx.tune_save(args.out)
    print(f"saved {args.out}", flush=True)


if __name__ == "__main__":
    main()
