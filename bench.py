#!/usr/bin/env python3
"""Throughput of the LLP HRMS solve on one MI355X.

One step = one full call of the library on one synthetic scene with inputs already in HBM: PAN statistics,
right-hand sides, conjugate gradients from Z = 0 to ||r|| <= 1e-6 ||b|| for every band, the true residual and
the objective of the result.  The workload is the 8-band scene with a 2048 x 2048 PAN image and 512 x 512 LRMS
(x4), a 17 x 17 anisotropic Gaussian blur, window radius 2, lambda 1e-2, eps 1e-3.
With --workload batch, one step is one batched call (llp_pansharpen_batch) on 64 scenes of uneven sizes (PAN
side from {256, 384, ..., 1024}, 4 or 8 bands, 9..17-tap Gaussian blurs, r 1, tol 1e-6); the line also
carries the same scenes solved one after another (`serial_value`).  With --workload warmstart (500 held-out
8-band 512^2 scenes) or large (4 scenes of 16 bands at 4096^2, r 2), the batched solve starts from the trained
network's estimate and the line carries the same solve from Z = 0 (`plain_cold_value`).

Prints one JSON line.  `value` is HRMS Mpixel*bands per second (N*H*W / time per step).  `roofline` is the
dominant kernel's algorithmic HBM bytes over its measured launch time (HIP events on the solver's stream around
each launch, summed over the timed steps); `traffic` is that kernel's counter-measured HBM bytes per launch from
profiles/traffic_8x2048.json while the kernel sources match the record.  `cpu_baseline` is the FP64 CPU oracle on a bounded sample of the same
scene (its setup plus a few CG iterations, extrapolated to the GPU's iteration count).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_8x2048.json")


def measured_traffic(prefixes):
    """HBM bytes per launch of the kernels whose names start with one of `prefixes` (summed: the operator step
    may be two launches) from the committed counter record, or None if the kernel sources have changed since
    the counters were taken (or there is no record for them)."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_RECORD))
        h = hashlib.sha256()
        for f in rec["source_files"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest()[:16] != rec["source_hash"]:
            return None
        total, found = 0.0, False
        for name, v in rec["kernels"].items():
            if any(name.startswith(p) for p in prefixes):
                total += v["traffic_bytes"]
                found = True
        return total if found else None
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--side", type=int, default=None, help="PAN side override (same recipe, smaller scene)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["scene", "batch", "warmstart", "large"], default="scene")
    ap.add_argument("--scenes", type=int, default=0, help="batched workloads: use only the first scenes")
    return ap.parse_args()


def cpu_baseline(sc, st, gpu_iters, budget_s):
    """FP64 oracle on the host: setup (operator data + right-hand sides) plus as many CG iterations of all bands
    as fit in the budget, extrapolated to the GPU's per-band iteration count."""
    import numpy as np
    import oracle
    from oracle.llp import Problem

    t0 = time.perf_counter()
    prob = Problem(u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=float(np.float32(st.lam)), eps=float(np.float32(st.eps)))
    b = oracle.rhs(sc.X, prob)
    t_setup = time.perf_counter() - t0
    k = 0
    t1 = time.perf_counter()
    while True:
        oracle.cg(prob, b, max_iters=1)  # one iteration of every band (the first: same cost as any other)
        k += 1
        if time.perf_counter() - t1 > budget_s / 2 or k >= 50:
            break
    t_iter = (time.perf_counter() - t1) / k
    N, H, W = sc.Z.shape
    t_solve = t_setup + gpu_iters * t_iter
    return {
        "value": N * H * W / t_solve / 1e6,
        "unit": "Mpixel*bands/s",
        "cores": os.cpu_count(),
        "kind": "oracle",
        "sample": f"setup + {k} CG iteration(s) of all {N} bands at {H}x{W}, FP64 numpy/scipy.fft "
                  f"(fft workers = all cores); extrapolated to {gpu_iters} iterations "
                  f"({t_setup:.2f} s setup, {t_iter:.2f} s per iteration)",
    }


def load_tuning(ctx):
    """Load the committed launch-configuration table for this device, if there is one for its architecture."""
    from paper_2103_09943_amd import binding as B
    from paper_2103_09943_amd.tune import DEFAULT_PATH
    if not os.path.exists(DEFAULT_PATH):
        return "none"
    try:
        ctx.tune_load(DEFAULT_PATH)
    except B.LlpError as e:
        return f"not loaded ({e})"
    return f"{os.path.relpath(DEFAULT_PATH, ROOT)} ({ctx.tune_count()} classes)"


def _gen_scene(args):
    from paper_2103_09943_amd import scenes
    config, s = args
    sc, st = scenes.config_scene(config, s)
    return sc.X, sc.Y, sc.u, sc.c


def apply_bytes_model(HW, c, band_iters, busy_launches):
    """Algorithmic HBM bytes of k_apply and k_dir for one scene (float32), c = resolution gap:
      k_apply: read p, r and y (1/c^2 of a plane), write q          -> 12 + 4/c^2 per active pixel-band
               plus the PAN statistics G, mu, dinv once per launch  -> 12 per pixel
      k_dir:   read r, q, p, x; write r, p, x and y                 -> 28 + 4/c^2 per active pixel-band"""
    c2 = float(c * c)
    return ((12.0 + 4.0 / c2) * HW * band_iters + 12.0 * HW * busy_launches,
            (28.0 + 4.0 / c2) * HW * band_iters)


def cpu_baseline_batch(host, settings, reps, budget_s, weights=None):
    """FP64 oracle on the host, on a sample of the workload: the setup and two CG iterations of the first scenes
    that fit the budget (and, for network starts, the oracle network on a 64 x 64 crop of one band); per-pixel
    setup, per-pixel-band network and per-pixel-band iteration costs extrapolated to the whole workload at the
    GPU's iteration counts."""
    import numpy as np
    import oracle
    from oracle import cnn
    from oracle.llp import Problem

    t_setup = t_iter = 0.0
    px = pxb = 0
    used = 0
    for (X, Y, u, c) in host:
        t0 = time.perf_counter()
        prob = Problem(u=u, c=c, Y=Y, r=settings.r, lam=float(np.float32(settings.lam)),
                       eps=float(np.float32(settings.eps)))
        b = oracle.rhs(X, prob)
        t1 = time.perf_counter()
        oracle.cg(prob, b, max_iters=2)
        t2 = time.perf_counter()
        t_setup += t1 - t0
        t_iter += (t2 - t1) / 2
        px += Y.size
        pxb += X.shape[0] * Y.size
        used += 1
        if t_setup + 2 * t_iter > budget_s / 2:
            break
    t_net_px = 0.0
    if weights is not None:
        X, Y, u, c = host[0]
        crop = 64
        t0 = time.perf_counter()
        cnn.warm_start(cnn.unflatten(weights), X[:1, :crop // c, :crop // c], Y[:crop, :crop], c)
        t_net_px = (time.perf_counter() - t0) / (crop * crop)
    total_px = sum(Y.size for _, Y, _, _ in host)
    total_pxb_it = sum(r["iters"] * Y.size for (X, Y, u, c), rs in zip(host, reps) for r in rs)
    total_pxb = sum(X.shape[0] * Y.size for X, Y, u, c in host)
    t_solve = t_setup / px * total_px + t_iter / pxb * total_pxb_it + t_net_px * total_pxb
    net = " plus the network start (oracle forward timed on a 64x64 crop)" if weights is not None else ""
    return {
        "value": total_pxb / t_solve / 1e6,
        "unit": "Mpixel*bands/s",
        "cores": os.cpu_count(),
        "kind": "oracle",
        "sample": f"setup + 2 CG iterations of every band of the first {used} scene(s), FP64 numpy/scipy.fft "
                  f"(fft workers = all cores){net}; per-pixel costs extrapolated to all {len(host)} scenes at "
                  f"the GPU's iteration counts",
    }


WEIGHTS = os.path.join(ROOT, "paper_2103_09943_amd", "weights", "cnn_warm_start.npy")

# workload -> (generator config, scene ids, start of the timed solve, comparison leg)
BATCH_WORKLOADS = {
    "batch": (2, range(64), None, "serial"),
    "warmstart": (3, range(2000, 2500), "cnn", "cold"),
    "large": (4, range(4), "cnn", "cold"),
}


def describe(name, host, st, pxb):
    if name == "batch":
        return (f"batched plain LLP solve (cold start, one call), {len(host)} scenes, PAN side 256..1024, 4 or 8 "
                f"bands, 9..17-tap Gaussian blurs, x4, r={st.r}, lambda={st.lam}, eps={st.eps}, tol={st.tol}; "
                f"{pxb / 1e6:.1f} Mpixel*bands")
    X, Y, u, c = host[0]
    taps = sorted({h[2].shape[0] for h in host})
    return (f"batched LLP solve from the trained network's start (one call), {len(host)} held-out scenes of "
            f"{X.shape[0]} bands, PAN {Y.shape[0]}x{Y.shape[1]}, x{c}, Gaussian blurs of {taps} taps, r={st.r}, "
            f"lambda={st.lam}, eps={st.eps}, tol={st.tol}; {pxb / 1e6:.1f} Mpixel*bands")


def main_batch(args):
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np
    import torch

    from paper_2103_09943_amd import binding as B
    from paper_2103_09943_amd import scenes

    config, ids, init, compare = BATCH_WORKLOADS[args.workload]
    ids = list(ids)[: args.scenes] if args.scenes else list(ids)
    workers = max(1, min(8, os.cpu_count() or 1, len(ids)))
    with ProcessPoolExecutor(workers) as ex:
        host = list(ex.map(_gen_scene, [(config, s) for s in ids]))
    _, st = scenes.config_scene(config, ids[0], side=256)
    ds = [(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), torch.from_numpy(u).cuda()) for X, Y, u, _ in host]
    outs = [torch.empty((X.shape[0],) + Y.shape, dtype=torch.float32, device="cuda") for X, Y, u, _ in host]
    pxb = sum(X.shape[0] * Y.size for X, Y, u, _ in host)
    ctx = B.Context(0)
    tuned = load_tuning(ctx)
    weights = None
    if init == "cnn":
        if not os.path.exists(WEIGHTS):
            raise SystemExit(f"{WEIGHTS} is missing: train it with `python -m paper_2103_09943_amd.train_cnn`")
        weights = np.load(WEIGHTS)
        ctx.cnn_set_weights(weights)
    kw = dict(r=st.r, lam=st.lam, eps=st.eps, max_iters=st.max_iters, tol=st.tol, outs=outs)
    # classes missing from the table are tuned by the first call (warm-up)
    ctx.pansharpen_batch(ds, flags=B.BATCH_AUTOTUNE, inits=init, **kw)
    for _ in range(max(args.warmup - 1, 0)):
        ctx.pansharpen_batch(ds, inits=init, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, reps, status = ctx.pansharpen_batch(ds, inits=init, **kw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # comparison leg, one timed call after one untimed: the same scenes one after another, or from Z = 0
    cflags, cinit = (B.BATCH_SERIAL, init) if compare == "serial" else (0, None)
    ctx.pansharpen_batch(ds, flags=cflags, inits=cinit, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, creps, _ = ctx.pansharpen_batch(ds, flags=cflags, inits=cinit, **kw)
    torch.cuda.synchronize()
    cmp_s = time.perf_counter() - t1
    # one call with events around every class launch (eager launches of the same kernels)
    ctx.set_profiling(True)
    ctx.kernel_times(reset=True)
    _, preps, _ = ctx.pansharpen_batch(ds, inits=init, **kw)
    kt = ctx.kernel_times(reset=True)
    ctx.set_profiling(False)
    ctx.close()

    apply_b = dir_b = 0.0
    for (X, Y, u, c), rs in zip(host, preps):
        a, d = apply_bytes_model(Y.size, c, sum(r["iters"] for r in rs), max(r["iters"] for r in rs))
        apply_b += a
        dir_b += d
    apply_gbs = apply_b / (kt["apply_ms"] * 1e-3) / 1e9 if kt["apply_ms"] > 0 else 0.0
    dir_gbs = dir_b / (kt["dir_ms"] * 1e-3) / 1e9 if kt["dir_ms"] > 0 else 0.0
    dominant = "k_apply" if kt["apply_ms"] >= kt["dir_ms"] else "k_dir"
    dom = dict(k_apply=(apply_gbs, kt["apply_ms"], kt["apply_launches"]),
               k_dir=(dir_gbs, kt["dir_ms"], kt["dir_launches"]))[dominant]
    iters = [r["iters"] for rs in reps for r in rs]
    citers = [r["iters"] for rs in creps for r in rs]
    value = pxb / (elapsed / args.steps) / 1e6
    cfg = {
        "workload": describe(args.workload, host, st, pxb),
        "status": status,
        "tuning": tuned,
        "iters_min_mean_max": [min(iters), round(sum(iters) / len(iters), 1), max(iters)],
        "k_apply_gbs": round(apply_gbs, 1),
        "k_dir_gbs": round(dir_gbs, 1),
    }
    if compare == "serial":
        cfg["serial_value"] = round(pxb / cmp_s / 1e6, 3)
        cfg["batch_over_serial"] = round(cmp_s / (elapsed / args.steps), 3)
    else:
        cfg["plain_cold_value"] = round(pxb / cmp_s / 1e6, 3)
        cfg["warm_over_cold"] = round(cmp_s / (elapsed / args.steps), 3)
        cfg["cold_iters_min_mean_max"] = [min(citers), round(sum(citers) / len(citers), 1), max(citers)]
        cfg["network_starts_rejected"] = sum(r["init"] == B.INIT_NET_REJECTED for rs in reps for r in rs)
        cfg["weights"] = os.path.relpath(WEIGHTS, ROOT)
    line = {
        "metric": "HRMS Mpixel·channels/s at fixed residual tol, plain vs CNN warm-start",
        "value": round(value, 3),
        "unit": "Mpixel*bands/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if init is None else "f32 (network: bf16 products, f32 accumulation)",
        "data": "synthetic",
        "config": cfg,
        "roofline": {
            "bound": "hbm",
            "kernel": dominant + " (all kernel classes of the batch, eager launches with events)",
            "achieved": round(dom[0], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(dom[0] / HBM_PEAK_GBS, 4),
            "avg_launch_us": round(dom[1] / max(dom[2], 1) * 1e3, 2),
            "traffic": None,
        },
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batch(host, st, reps, args.cpu_seconds, weights)
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the per-band solves would shard "
              "across GPUs with no communication, but this program runs on one device.", file=sys.stderr)
        sys.exit(2)
    if args.workload != "scene":
        return main_batch(args)
    import numpy as np
    import torch

    from paper_2103_09943_amd import binding as B
    from paper_2103_09943_amd import scenes

    sc, st = scenes.config_scene(1, 0, side=args.side)
    N, H, W = sc.Z.shape
    X = torch.from_numpy(sc.X).cuda()
    Y = torch.from_numpy(sc.Y).cuda()
    u = torch.from_numpy(sc.u).cuda()
    out = torch.empty((N, H, W), dtype=torch.float32, device="cuda")
    ctx = B.Context(0)
    tuned = load_tuning(ctx)
    if tuned.startswith("none") or tuned.startswith("not"):
        res = ctx.autotune(X, Y, u, r=st.r, lam=st.lam, eps=st.eps, iters=8)  # part of the warm-up
        tuned = f"tuned in warm-up: dir_rows {res['dir_rows']}, apply_variant {res['apply_variant']}"
    kw = dict(r=st.r, lam=st.lam, eps=st.eps, max_iters=st.max_iters, tol=st.tol, out=out)

    for _ in range(args.warmup):
        ctx.pansharpen(X, Y, u, **kw)
    ctx.set_profiling(True)
    ctx.kernel_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(args.steps):
        _, rep, status = ctx.pansharpen(X, Y, u, **kw)
        reps.append(rep)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = ctx.kernel_times(reset=True)
    ctx.set_profiling(False)

    ms_per_step = elapsed / args.steps * 1e3
    value = N * H * W / (elapsed / args.steps) / 1e6
    iters = [r["iters"] for r in reps[-1]]
    HW = H * W
    band_iters = sum(sum(r["iters"] for r in rep) for rep in reps)
    launches = kt["apply_launches"]
    busy_launches = sum(max(r["iters"] for r in rep) for rep in reps)  # launches with at least one active band
    apply_bytes, dir_bytes = apply_bytes_model(HW, sc.c, band_iters, busy_launches)
    apply_gbs = apply_bytes / (kt["apply_ms"] * 1e-3) / 1e9 if kt["apply_ms"] > 0 else 0.0
    dir_gbs = dir_bytes / (kt["dir_ms"] * 1e-3) / 1e9 if kt["dir_ms"] > 0 else 0.0
    it_ms = kt["apply_ms"] + kt["dir_ms"]
    iter_gbs = (apply_bytes + dir_bytes) / (it_ms * 1e-3) / 1e9 if it_ms > 0 else 0.0
    dominant = "k_apply" if kt["apply_ms"] >= kt["dir_ms"] else "k_dir"
    # counter-measured HBM bytes per launch (8 x 2048^2 workload, all bands active) for the specialised kernels
    traffic = None
    if args.side is None:
        traffic = measured_traffic(("llp::k_llp<2, 1, 4, 8>",) if dominant == "k_apply"
                                   else ("llp::k_dir_fast<4, 8, 4, 2>",))
    dom = {
        "k_apply": dict(kernel="k_apply (q = A p: the column sweep k_llp, B^T D^T y on matrix cores + lambda "
                               "L^T M L p; p^T q, r^T q, q^T q)",
                        achieved=apply_gbs, ms=kt["apply_ms"], n=launches),
        "k_dir": dict(kernel="k_dir (x, r update; p = r + beta p; y = D B p; r^T r)", achieved=dir_gbs,
                      ms=kt["dir_ms"], n=kt["dir_launches"]),
    }[dominant]
    line = {
        "metric": "HRMS Mpixel·channels/s at fixed residual tol, plain vs CNN warm-start",
        "value": round(value, 3),
        "unit": "Mpixel*bands/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"plain LLP solve (cold start), 1 scene, {N} bands, PAN {H}x{W}, LRMS {H // sc.c}x{W // sc.c} "
                        f"(x{sc.c}), {sc.u.shape[0]}x{sc.u.shape[0]} anisotropic Gaussian blur, r={st.r}, "
                        f"lambda={st.lam}, eps={st.eps}, tol={st.tol}",
            "tuning": tuned,
            "iters_per_band": iters,
            "max_true_rel_residual": max(r["true_rel_residual"] for r in reps[-1]),
            "status": status,
            "ms_per_cg_iteration": round(it_ms / max(launches, 1), 4),
            "iteration_gbs": round(iter_gbs, 1),
            "iteration_frac": round(iter_gbs / HBM_PEAK_GBS, 4),
            "k_apply_gbs": round(apply_gbs, 1),
            "k_apply_avg_us": round(kt["apply_ms"] / max(launches, 1) * 1e3, 2),
            "k_dir_gbs": round(dir_gbs, 1),
            "k_dir_avg_us": round(kt["dir_ms"] / max(kt["dir_launches"], 1) * 1e3, 2),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom["kernel"],
            "achieved": round(dom["achieved"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(dom["achieved"] / HBM_PEAK_GBS, 4),
            "avg_launch_us": round(dom["ms"] / max(dom["n"], 1) * 1e3, 2),
            "traffic": round(traffic) if traffic is not None else None,
        },
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sc, st, int(statistics.median(iters)), args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
