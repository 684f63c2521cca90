"""Writes the objective of eq. (initialize_z_fast) at the exact minimiser for sampled bands of the 8-band
2048 x 2048 scene (tests/golden/scene_objectives.json).  Calls only the oracle: FP64 conjugate gradients on
eq. (Z_ini_matting) to a relative residual of 1e-11, then the objective of that solution.  The inputs are the
seeded scene rounded to float32, and lambda, eps rounded to float32, exactly as the library receives them.

Usage: python tests/golden/make_scene_objectives.py   (about 10 minutes per band on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.llp import Problem  # noqa: E402
from paper_2103_09943_amd import scenes  # noqa: E402

BANDS = [1, 6]


def main():
    sc, st = scenes.config_scene(1, 0)
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    prob = Problem(u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=f32(st.lam), eps=f32(st.eps))
    out = {"scene": "workload 1, scene 0 (8 bands, 2048^2 PAN, 17x17 anisotropic blur, r 2, lambda 1e-2, eps 1e-3)",
           "solver": "oracle.cg to relative residual 1e-11 (FP64)", "bands": {}}
    for band in BANDS:
        t0 = time.time()
        X = sc.X[band:band + 1]
        b = oracle.rhs(X, prob)
        Z, its = oracle.cg(prob, b, max_iters=20000, tol=1e-11)
        res = b - oracle.apply_A(Z, prob)
        rel = float(np.linalg.norm(res) / np.linalg.norm(b))
        obj = float(oracle.objective(Z, X, prob)[0])
        out["bands"][str(band)] = {"objective": obj, "iterations": int(its[0]), "rel_residual": rel}
        print(f"band {band}: {int(its[0])} iterations, residual {rel:.2e}, objective {obj!r} "
              f"({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "scene_objectives.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
