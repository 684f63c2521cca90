"""Workload for HBM-traffic counters: one calibration copy of known size, then CG iterations of the 8-band
2048 x 2048 scene (the benchmark workload).

Run it under a counter collector, e.g.
    rocprofv3 --pmc FETCH_SIZE -d OUT -o run -- python3 -m paper_2103_09943_amd.traffic_probe
The device copy of COPY_BYTES (read COPY_BYTES, write COPY_BYTES) gives the scale between the counters and
bytes; the per-dispatch counters of the iteration kernels are then divided by that scale.
"""
from __future__ import annotations

import argparse

COPY_BYTES = 256 * 1024 * 1024


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=10)
    args = ap.parse_args()
    import torch

    from paper_2103_09943_amd import binding as B
    from paper_2103_09943_amd import scenes

    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    sc, st = scenes.config_scene(1, 0)
    X = torch.from_numpy(sc.X).cuda()
    Y = torch.from_numpy(sc.Y).cuda()
    u = torch.from_numpy(sc.u).cuda()
    with B.Context(0) as ctx:
        ctx.pansharpen(X, Y, u, r=st.r, lam=st.lam, eps=st.eps, max_iters=args.iters, tol=0.0, report=False)
    torch.cuda.synchronize()
    print(f"traffic probe: copy {COPY_BYTES} B, {args.iters} CG iterations", flush=True)


if __name__ == "__main__":
    main()
