#!/usr/bin/env python3
"""Throughput of the LLP HRMS solve on one MI355X.

Default workload (`large`): 4 synthetic scenes of 16 bands with a 4096 x 4096 PAN image and 1024 x 1024 LRMS (x4),
17 x 17 Gaussian blurs, window radius 2, lambda 1e-2, eps 1e-3, tolerance 1e-6 on the FP64 residual of every
band's iterate.  One step = one call of the library (llp_pansharpen_batch) on the 4 scenes with inputs already in
HBM: PAN statistics, right-hand sides, the warm-start network's estimate, the conjugate-gradient solve
preconditioned in the Fourier domain, FP64 residual replacement and verification, the reported residuals and
objective.  `value` is HRMS Mpixel*bands per second with the network start; `config.plain_cold_value` is the same
call from Z = 0 (the metric's plain leg), `config.cg_cold_value` the unpreconditioned solve from Z = 0.

Other workloads (--workload): `scene` (one 8-band 2048^2 scene, r 2; value from Z = 0; `config.polish_ms` times the
A, C and Z steps of Algorithm "Fast Pansharpening" on the solved HRMS), `batch` (64 scenes of
PAN side 256..1024, 4 or 8 bands, r 1; value from Z = 0), `warmstart` (500 held-out 8-band 512^2 scenes, network
start vs Z = 0), `priors` (the `scene` input solved under the compared priors of the paper's prior comparison:
value = the LGC prior to tol 1e-6 from Z = 0; HPF likewise, LLP/LPP/LPF at a fixed iteration count as legs),
`kernel_est` (Algorithm "Blur Kernel Estimation" on the `scene` input: a 29 x 29 kernel from the 8 LRMS bands and
PAN with the paper's parameters, to convergence; value = the scene's Mpixel*bands per second of estimation).

Prints one JSON line.  `roofline` is the kernel class with the most device time in one separately profiled step
(HIP events around every launch on the solver's stream; the timed steps carry no events): its algorithmic HBM
bytes (the model in `bytes_model` below) over its measured time.  `config.iteration_frac` is the same for all
iteration kernels together.  `traffic` is the dominant kernel's counter-measured HBM bytes per launch from the
profiles/ record while the kernel sources match it, else null.  `cpu_baseline` is the FP64 CPU oracle on a bounded
sample of the same workload, extrapolated.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
ROOT = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(ROOT, "paper_2103_09943_amd", "weights", "cnn_warm_start.npy")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_large.json")
METRIC = "HRMS Mpixel·channels/s at fixed residual tol, plain vs CNN warm-start"

# workload -> (generator config, scene ids, timed start, comparison start, description)
WORKLOADS = {
    "large": (4, range(4), "cnn", None),
    "scene": (1, range(1), None, None),
    "batch": (2, range(64), None, None),
    "warmstart": (3, range(2000, 2500), "cnn", None),
    "priors": (1, range(1), None, None),
    "kernel_est": (1, range(1), None, None),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="large")
    ap.add_argument("--scenes", type=int, default=0, help="use only the first scenes of the workload")
    ap.add_argument("--cpu-seconds", type=float, default=30.0, help="budget of the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the comparison legs and the profiled step")
    ap.add_argument("--profile-only", action="store_true",
                    help="skip the comparison legs but keep the profiled step (every call is then the same solve)")
    return ap.parse_args()


def _gen_scene(args):
    from paper_2103_09943_amd import scenes
    config, s = args
    sc, _ = scenes.config_scene(config, s)
    return sc.X, sc.Y, sc.u, sc.c


def bytes_model(kt, host, reps, precond):
    """Algorithmic HBM bytes of every kernel class over one call (float32 planes, c the resolution gap):
      operator (k_apply / sweep):   read p, r, y (1/c^2 of a plane); write q          12 + 4/c^2 per active px-band
                                    plus the PAN statistics G, mu, dinv per launch   12 per pixel
      plain update (k_dir mode 2):  read r, q, p, x; write r, p, x, y                 28 + 4/c^2
      direction (k_dir mode 3):     read s, p, x; write p, x, y                       20 + 4/c^2
      rows (forward, with update):  read r, q; write r, the spectrum                  16  (spectrum: 8 B per pixel pair)
      columns (group solve):        read and write the spectrum, read U               12  (8 + 8 + 8 B per pixel pair)
      rows (inverse):               read the spectrum and r; write s                  12
    Per scene: px-band iterations = H W * sum of band iterations; operator launches with an active band = the
    largest band iteration count."""
    out = {k: 0.0 for k in ("apply", "dir", "pc_rows", "pc_cols", "pc_rows_inv")}
    for (X, Y, u, c), rs in zip(host, reps):
        HW = Y.size
        band_iters = sum(r["iters"] for r in rs)
        busy = max(r["iters"] for r in rs)
        c2 = float(c * c)
        out["apply"] += (12.0 + 4.0 / c2) * HW * band_iters + 12.0 * HW * busy
        if precond:
            out["dir"] += (20.0 + 4.0 / c2) * HW * band_iters
            out["pc_rows"] += 16.0 * HW * band_iters
            out["pc_cols"] += 12.0 * HW * band_iters
            out["pc_rows_inv"] += 12.0 * HW * band_iters
        else:
            out["dir"] += (28.0 + 4.0 / c2) * HW * band_iters
    return out


KERNEL_NAMES = {
    "apply": "operator q = A p (column sweep k_llp_batch: B^T D^T y on matrix cores + lambda L^T M L p)",
    "dir": "direction kernel k_dir_fast_batch (x += alpha p, p = s + beta p, y = D B p)",
    "pc_rows": "k_pc_rows (r -= alpha q; forward row transforms of the band pairs)",
    "pc_cols": "k_pc_cols (column transforms, per-group solve of P, inverse column transforms)",
    "pc_rows_inv": "k_pc_rows_inv (inverse row transforms, s = P^-1 r, r^T s)",
}
# kernel names in the traffic record (namespace and template arguments, no parameter list)
PROF_PREFIX = {"pc_cols": "llp::k_pc_cols<", "pc_rows": "llp::k_pc_rows<", "pc_rows_inv": "llp::k_pc_rows_inv<",
               "dir": "llp::k_dir_fast_batch<", "apply": "llp::k_llp_batch<"}


def measured_traffic(kernel):
    """Counter-measured HBM bytes per launch of `kernel` from the committed record, or None if the kernel
    sources changed since the counters were taken (or the record has no such kernel)."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_RECORD))
        h = hashlib.sha256()
        for f in rec["source_files"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest()[:16] != rec["source_hash"]:
            return None
        for name, v in rec["kernels"].items():
            if name.startswith(PROF_PREFIX[kernel]):
                return v["traffic_bytes"]
    except (OSError, KeyError, ValueError):
        return None
    return None


def cpu_baseline(host, reps, settings, budget_s, net):
    """FP64 oracle on the host, on a bounded sample: for the first band of the first scene at full size, the
    scene set-up (operator data, right-hand side), one product with A and one with P^{-1} (one preconditioned
    iteration), and for network starts the oracle network on a 64 x 64 crop; per-pixel set-up, per-pixel-band
    iteration and network costs extrapolated to the whole workload at the GPU's iteration counts."""
    import numpy as np
    import oracle
    from oracle import cnn
    from oracle.llp import Problem

    X, Y, u, c = host[0]
    t0 = time.perf_counter()
    prob = Problem(u=u, c=c, Y=Y, r=settings.r, lam=float(np.float32(settings.lam)),
                   eps=float(np.float32(settings.eps)))
    b = oracle.rhs(X[:1], prob)
    mbar = oracle.matting_diag_mean(prob)
    t_setup = time.perf_counter() - t0
    t1 = time.perf_counter()
    q = oracle.apply_A(b, prob)
    s = oracle.precond_apply(b, prob, mbar)
    t_iter = time.perf_counter() - t1
    del q, s
    t_net = 0.0
    if net is not None:
        crop = 64
        t2 = time.perf_counter()
        cnn.warm_start(cnn.unflatten(net), X[:1, :crop // c, :crop // c], Y[:crop, :crop], c)
        t_net = (time.perf_counter() - t2) / (crop * crop)
    px = sum(Yh.size for _, Yh, _, _ in host)
    pxb = sum(Xh.shape[0] * Yh.size for Xh, Yh, _, _ in host)
    pxb_it = sum(r["iters"] * Yh.size for (Xh, Yh, _, _), rs in zip(host, reps) for r in rs)
    HW = Y.size
    t_solve = t_setup / HW * px + t_iter / HW * pxb_it + t_net * pxb
    return {
        "value": pxb / t_solve / 1e6,
        "unit": "Mpixel*bands/s",
        "cores": os.cpu_count(),
        "kind": "oracle",
        "sample": f"scene set-up plus one preconditioned iteration (A and P^-1 products) of one band at "
                  f"{Y.shape[0]}x{Y.shape[1]}, FP64 numpy/scipy (fft workers = all cores)"
                  + (", plus the oracle network on a 64x64 crop" if net is not None else "")
                  + f"; extrapolated to {len(host)} scene(s), {pxb / 1e6:.1f} Mpixel*bands at the GPU's iteration "
                    f"counts ({t_setup:.1f} s set-up, {t_iter:.1f} s per band-iteration at full size)",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the per-band solves would shard "
              "across GPUs with no communication, but this program runs on one device.", file=sys.stderr)
        sys.exit(2)
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np
    import torch

    from paper_2103_09943_amd import binding as B
    from paper_2103_09943_amd import scenes
    from paper_2103_09943_amd.tune import DEFAULT_PATH

    if args.workload == "priors":
        return run_priors(args)
    if args.workload == "kernel_est":
        return run_kernel_est(args)
    config, ids, init, _ = WORKLOADS[args.workload]
    ids = list(ids)[: args.scenes] if args.scenes else list(ids)
    t0 = time.time()
    workers = max(1, min(8, os.cpu_count() or 1, len(ids)))
    with ProcessPoolExecutor(workers) as ex:
        host = list(ex.map(_gen_scene, [(config, s) for s in ids]))
    _, st = scenes.config_scene(config, ids[0], side=256)
    log(f"{len(host)} scene(s) generated in {time.time() - t0:.0f} s")
    ds = [(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), torch.from_numpy(u).cuda()) for X, Y, u, _ in host]
    outs = [torch.empty((X.shape[0],) + Y.shape, dtype=torch.float32, device="cuda") for X, Y, u, _ in host]
    pxb = sum(X.shape[0] * Y.size for X, Y, u, _ in host)
    ctx = B.Context(0)
    tuned = "none"
    if os.path.exists(DEFAULT_PATH):
        ctx.tune_load(DEFAULT_PATH)
        tuned = f"{os.path.relpath(DEFAULT_PATH, ROOT)} ({ctx.tune_count()} classes)"
    net = None
    if init == "cnn":
        net = np.load(WEIGHTS)
        ctx.cnn_set_weights(net)
    kw = dict(r=st.r, lam=st.lam, eps=st.eps, max_iters=st.max_iters, tol=st.tol, outs=outs)

    def call(inits, precond, flags=0):
        return ctx.pansharpen_batch(ds, inits=inits, precond=precond, flags=flags, **kw)

    def timed(inits, precond, steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            _, reps, status = call(inits, precond)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps, reps, status

    for i in range(args.warmup):
        call(init, 1)
        log(f"warm-up step {i + 1}/{args.warmup} done")
    step_s, reps, status = timed(init, 1, args.steps)
    log(f"timed {args.steps} step(s): {step_s * 1e3:.1f} ms per step")
    value = pxb / step_s / 1e6
    iters = [r["iters"] for rs in reps for r in rs]
    cfg = {
        "workload": describe(args.workload, host, st, pxb),
        "solver": "conjugate gradients preconditioned in the Fourier domain (P = B^T D^T D B + lambda mbar L^T L), "
                  "FP64 residual replacement; tol on the FP64 residual of every band's iterate",
        "start": "warm-start network (bf16 MFMA), rejected band by band where no better than Z = 0"
                 if init == "cnn" else "Z = 0",
        "status": status,
        "tuning": tuned,
        "iters_min_mean_max": [min(iters), round(float(np.mean(iters)), 1), max(iters)],
        "max_true_rel_residual": max(r["true_rel_residual"] for rs in reps for r in rs),
        "max_out_rel_residual": max(r["out_rel_residual"] for rs in reps for r in rs),
    }
    roofline = None
    if not args.no_legs:
        if init == "cnn" and not args.profile_only:
            call(None, 1)
            cold_s, creps, _ = timed(None, 1, 1)
            citers = [r["iters"] for rs in creps for r in rs]
            cfg["plain_cold_value"] = round(pxb / cold_s / 1e6, 3)
            cfg["warm_over_cold"] = round(cold_s / step_s, 3)
            cfg["cold_iters_min_mean_max"] = [min(citers), round(float(np.mean(citers)), 1), max(citers)]
            cfg["network_starts_rejected"] = sum(r["init"] == B.INIT_NET_REJECTED for rs in reps for r in rs)
            log(f"cold preconditioned leg: {cold_s * 1e3:.1f} ms")
        if not args.profile_only:
            call(None, 0)
            cg_s, greps, _ = timed(None, 0, 1)
            giters = [r["iters"] for rs in greps for r in rs]
            cfg["cg_cold_value"] = round(pxb / cg_s / 1e6, 3)
            cfg["cg_cold_iters_min_mean_max"] = [min(giters), round(float(np.mean(giters)), 1), max(giters)]
            log(f"unpreconditioned cold leg: {cg_s * 1e3:.1f} ms")
        if len(ds) == 1 and not args.profile_only:
            # the A, C step and the FFT Z step of Algorithm "Fast Pansharpening" on the solved HRMS (llp_polish)
            X0, Y0, u0 = ds[0]
            z0 = outs[0].clone()
            ctx.polish(z0, X0, Y0, u0, r=st.r, lam=st.lam, eps=st.eps)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(5):
                ctx.polish(z0, X0, Y0, u0, r=st.r, lam=st.lam, eps=st.eps)
            torch.cuda.synchronize()
            pol = (time.perf_counter() - t) / 5
            cfg["polish_ms"] = round(pol * 1e3, 3)
            cfg["polish_value"] = round(pxb / pol / 1e6, 1)
            log(f"A,C and Z step (llp_polish): {pol * 1e3:.2f} ms")
        # one profiled step (events around every launch): per-kernel device times
        ctx.set_profiling(True)
        ctx.kernel_times(reset=True)
        _, preps, _ = call(init, 1)
        kt = ctx.kernel_times(reset=True)
        ctx.set_profiling(False)
        model = bytes_model(kt, host, preps, True)
        per = {}
        for k in model:
            ms, n = kt[f"{k}_ms"], kt[f"{k}_launches"]
            if ms > 0 and n > 0:
                per[k] = dict(gbs=model[k] / (ms * 1e-3) / 1e9, ms=ms, n=n)
        for k, v in per.items():
            cfg[f"{k}_gbs"] = round(v["gbs"], 1)
            cfg[f"{k}_avg_us"] = round(v["ms"] / v["n"] * 1e3, 1)
        it_bytes = sum(model[k] for k in per)
        it_ms = sum(v["ms"] for v in per.values())
        cfg["iteration_gbs"] = round(it_bytes / (it_ms * 1e-3) / 1e9, 1)
        cfg["iteration_frac"] = round(it_bytes / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        cfg["ref_ms_per_step"] = round(kt["ref_ms"], 2)
        dom = max(per, key=lambda k: per[k]["ms"])
        d = per[dom]
        traffic = measured_traffic(dom) if args.workload == "large" and not args.scenes else None
        roofline = {
            "bound": "hbm",
            "kernel": KERNEL_NAMES[dom],
            "achieved": round(d["gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(d["gbs"] / HBM_PEAK_GBS, 4),
            "avg_launch_us": round(d["ms"] / d["n"] * 1e3, 1),
            "traffic": round(traffic) if traffic is not None else None,
        }
    ctx.close()
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpixel*bands/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if init is None else "f32 (network: bf16 products, f32 accumulation)",
        "data": "synthetic",
        "config": cfg,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(host, reps, st, args.cpu_seconds, net)
    print(json.dumps(line), flush=True)


def prior_bytes_model(kind, HW, c, reps):
    """Algorithmic HBM bytes of the prior solve's kernel classes over one call (float32 planes):
      operator (k_prior_apply):    read p, r, y (1/c^2 of a plane); write q          12 + 4/c^2 per active px-band
                                   plus per filter its guide, window means, dinv    12 per pixel and launch
      plain update (k_dir mode 2): read r, q, p, x; write r, p, x, y                 28 + 4/c^2"""
    nf = 2 if kind == "lgc" else 1
    band_iters = sum(r["iters"] for r in reps)
    busy = max(r["iters"] for r in reps)
    c2 = float(c * c)
    return {"apply": (12.0 + 4.0 / c2) * HW * band_iters + 12.0 * nf * HW * busy,
            "dir": (28.0 + 4.0 / c2) * HW * band_iters}


def run_priors(args):
    """The `priors` workload: one 8-band 2048^2 scene (x4, 17-tap blur, r 2) under the compared priors."""
    import numpy as np
    import torch

    from paper_2103_09943_amd import binding as B
    from paper_2103_09943_amd import scenes

    sc, st = scenes.config_scene(1, 0)
    ds = (torch.from_numpy(sc.X).cuda(), torch.from_numpy(sc.Y).cuda(), torch.from_numpy(sc.u).cuda())
    N, H, W = sc.X.shape[0], sc.Y.shape[0], sc.Y.shape[1]
    pxb = N * H * W
    out = torch.empty((N, H, W), dtype=torch.float32, device="cuda")
    ctx = B.Context(0)
    kw = dict(r=st.r, lam=st.lam, eps=st.eps, out=out)

    def timed(kind, steps, **k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            _, reps, status = ctx.prior_pansharpen(kind, *ds, **kw, **k)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps, reps, status

    tolkw = dict(max_iters=st.max_iters, tol=st.tol)
    for i in range(args.warmup):
        ctx.prior_pansharpen("lgc", *ds, **kw, **tolkw)
        log(f"warm-up step {i + 1}/{args.warmup} done")
    step_s, reps, status = timed("lgc", args.steps, **tolkw)
    log(f"timed {args.steps} step(s): {step_s * 1e3:.1f} ms per step")
    iters = [r["iters"] for r in reps]
    cfg = {
        "workload": f"1 scene of 8 bands, PAN 2048x2048, LRMS 512x512 (x4), Gaussian blur of 17 taps, r={st.r}, "
                    f"lambda={st.lam}, eps={st.eps}; the LGC prior (eq. reg2_lgc) in place of LLP, tol={st.tol} on "
                    f"the float32-operator residual; {pxb / 1e6:.1f} Mpixel*bands per step",
        "solver": "plain conjugate gradients, float32 vectors, FP64 dot products, true-residual check and restart",
        "start": "Z = 0",
        "status": status,
        "iters_min_mean_max": [min(iters), round(float(np.mean(iters)), 1), max(iters)],
        "max_true_rel_residual": max(r["true_rel_residual"] for r in reps),
    }
    roofline = None
    if not args.no_legs:
        legs = {}
        s_h, r_h, st_h = timed("hpf", 1, **tolkw)
        legs["hpf"] = {"value": round(pxb / s_h / 1e6, 3), "ms": round(s_h * 1e3, 1), "status": st_h,
                       "iters_max": max(r["iters"] for r in r_h)}
        K = 20
        for kind in ("llp", "lpp", "lpf"):  # residual floors of the float32 operator above 1e-6: fixed count
            s_k, r_k, _ = timed(kind, 1, max_iters=K, tol=0.0)
            legs[kind] = {"ms_per_iteration": round(s_k / K * 1e3, 2), "iters": K}
        s_l, _, _ = timed("lgc", 1, max_iters=K, tol=0.0)
        legs["lgc"] = {"ms_per_iteration": round(s_l / K * 1e3, 2), "iters": K}
        cfg["legs"] = legs
        ctx.set_profiling(True)
        ctx.kernel_times(reset=True)
        _, preps, _ = ctx.prior_pansharpen("lgc", *ds, **kw, **tolkw)
        kt = ctx.kernel_times(reset=True)
        ctx.set_profiling(False)
        model = prior_bytes_model("lgc", H * W, sc.c, preps)
        per = {}
        for k in model:
            ms, n = kt[f"{k}_ms"], kt[f"{k}_launches"]
            if ms > 0 and n > 0:
                per[k] = dict(gbs=model[k] / (ms * 1e-3) / 1e9, ms=ms, n=n)
        for k, v in per.items():
            cfg[f"{k}_gbs"] = round(v["gbs"], 1)
            cfg[f"{k}_avg_us"] = round(v["ms"] / v["n"] * 1e3, 1)
        dom = max(per, key=lambda k: per[k]["ms"])
        d = per[dom]
        roofline = {
            "bound": "hbm",
            "kernel": {"apply": "k_prior_apply<3, 2> (q = A p under LGC: two gradient filters, window sums in LDS, "
                                "B^T D^T y, CG dot products)",
                       "dir": "k_dir_fast (x, r, p update and D B p)"}[dom],
            "achieved": round(d["gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(d["gbs"] / HBM_PEAK_GBS, 4),
            "avg_launch_us": round(d["ms"] / d["n"] * 1e3, 1),
            "traffic": None,
        }
    ctx.close()
    line = {
        "metric": METRIC,
        "value": round(pxb / step_s / 1e6, 3),
        "unit": "Mpixel*bands/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": cfg,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline_priors(sc, st, reps)
    print(json.dumps(line), flush=True)


def cpu_baseline_priors(sc, st, reps):
    """FP64 oracle (oracle/priors.py) on a bounded sample: the LGC scene set-up and one product with A for one
    band at full size, extrapolated to every band at the GPU's iteration counts."""
    import numpy as np
    import oracle
    from oracle import priors

    t0 = time.perf_counter()
    prob = priors.PriorProblem("lgc", u=sc.u, c=sc.c, Y=sc.Y, r=st.r, lam=float(np.float32(st.lam)),
                               eps=float(np.float32(st.eps)))
    b = oracle.rhs(sc.X[:1], prob)
    t_setup = time.perf_counter() - t0
    t1 = time.perf_counter()
    priors.apply_A_prior(b, prob)
    t_iter = time.perf_counter() - t1
    N = sc.X.shape[0]
    band_iters = sum(r["iters"] for r in reps)
    t_solve = t_setup + t_iter * band_iters
    pxb = N * sc.Y.size
    return {
        "value": pxb / t_solve / 1e6,
        "unit": "Mpixel*bands/s",
        "cores": os.cpu_count(),
        "kind": "oracle",
        "sample": f"LGC scene set-up plus one product with A of one band at {sc.Y.shape[0]}x{sc.Y.shape[1]}, FP64 "
                  f"numpy/scipy; extrapolated to {N} bands at the GPU's {band_iters} band-iterations "
                  f"({t_setup:.1f} s set-up, {t_iter:.1f} s per band-iteration)",
    }


KE_N = 29  # the paper's kernel size (Sec. IV-C)
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector


def run_kernel_est(args):
    """The `kernel_est` workload: Algorithm 1 on the 8-band 2048^2 scene (x4), n = 29, the paper's parameters.
    The GADMM runs in one workgroup by design (its iterates are n x n); its roofline fraction is given against the
    chip's FP64 vector peak and, in config, against one compute unit's share of it."""
    import numpy as np
    import torch

    from paper_2103_09943_amd import binding as B
    from paper_2103_09943_amd import scenes

    sc, _ = scenes.config_scene(1, 0)
    X = torch.from_numpy(sc.X).cuda()
    Y = torch.from_numpy(sc.Y).cuda()
    N, H, W = sc.X.shape[0], sc.Y.shape[0], sc.Y.shape[1]
    pxb = N * H * W
    ctx = B.Context(0)

    def run(t_max, steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            k, om, rep = ctx.estimate_kernel(X, Y, sc.c, n=KE_N, t_max=t_max)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps, k, rep

    for i in range(args.warmup):
        run(10000, 1)
        log(f"warm-up step {i + 1}/{args.warmup} done")
    step_s, kern, rep = run(10000, args.steps)
    log(f"timed {args.steps} step(s): {step_s * 1e3:.1f} ms per step")
    setup_s, _, _ = run(0, 2)
    it = rep["iters"]
    n2 = KE_N * KE_N
    # flops of one GADMM iteration: the product with the n^2 x n^2 inverse, twelve n x n DFT passes (complex
    # multiply-adds over n terms), the per-frequency Cramer solves and the element-wise steps
    flops_iter = 2.0 * n2 * n2 + 12 * n2 * KE_N * 8.0 + n2 * 400.0
    gadmm_s = max(step_s - setup_s, 1e-9)
    achieved = flops_iter * it / gadmm_s / 1e12
    u_true = sc.u
    k = kern.cpu().numpy().astype(np.float64)
    R = (KE_N - 1) // 2
    pad = np.zeros((KE_N, KE_N))
    nt = u_true.shape[0]
    o = R - (nt - 1) // 2
    pad[o:o + nt, o:o + nt] = u_true
    cfg = {
        "workload": f"Algorithm 1 (blur-kernel estimation) on 1 scene of 8 bands, PAN 2048x2048, LRMS 512x512 (x4): "
                    f"a {KE_N}x{KE_N} kernel, the paper's parameters (l 1, lambda_w 10, alpha 1 / 0.006, mu 100, "
                    f"rho 0.5, threshold 1e-5); {pxb / 1e6:.1f} Mpixel*bands per step",
        "gadmm_iters": it,
        "setup_ms": round(setup_s * 1e3, 2),
        "gadmm_ms": round(gadmm_s * 1e3, 2),
        "gadmm_us_per_iter": round(gadmm_s / max(it, 1) * 1e6, 2),
        "gadmm_gflops": round(achieved * 1e3, 1),
        "gadmm_frac_of_one_cu": round(achieved / (FP64_PEAK_TFLOPS / 256.0), 4),
        "kernel_rel_error_pct": round(float(100.0 * np.linalg.norm(k - pad) / np.linalg.norm(pad)), 2),
    }
    ctx.close()
    line = {
        "metric": METRIC,
        "value": round(pxb / step_s / 1e6, 3),
        "unit": "Mpixel*bands/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": {"bound": "alu", "kernel": "k_ke_gadmm (one workgroup: the n x n GADMM iterates in LDS)",
                     "achieved": round(achieved, 5), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_PEAK_TFLOPS, 6), "traffic": None},
    }
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline_kernel_est(sc, it, pxb)
    print(json.dumps(line), flush=True)


def cpu_baseline_kernel_est(sc, iters, pxb):
    """The oracle's Algorithm 1 (oracle/tgv.py) on the same scene: the set-up alone (omega, E, the Cholesky factor
    of E^T E + mu_3 I; t_max = 0) and the set-up with 200 GADMM iterations, each the faster of two runs; the
    difference gives the time per iteration, extrapolated to the GPU's iteration count."""
    from oracle import tgv

    def timed(t_max):
        best = None
        for _ in range(2):
            t0 = time.perf_counter()
            tgv.estimate_kernel(sc.X, sc.Y, sc.c, tgv.TgvParams(n=KE_N, t_max=t_max, th=0.0))
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    K = 200
    t_setup = timed(0)
    t_iter = max(timed(K) - t_setup, 0.0) / K
    t = t_setup + t_iter * iters
    return {"value": pxb / t / 1e6, "unit": "Mpixel*bands/s", "cores": os.cpu_count(), "kind": "oracle",
            "sample": f"the oracle's set-up ({t_setup:.1f} s: omega, E, the Cholesky factor) and {K} GADMM iterations "
                      f"({t_iter * 1e3:.2f} ms each), the faster of two runs each, extrapolated to the GPU's "
                      f"{iters} iterations"}


def describe(name, host, st, pxb):
    X, Y, u, c = host[0]
    taps = sorted({h[2].shape[0] for h in host})
    sides = sorted({h[1].shape[0] for h in host})
    what = {"large": "4 scenes of 16 bands, PAN 4096x4096, LRMS 1024x1024",
            "scene": "1 scene of 8 bands, PAN 2048x2048, LRMS 512x512",
            "batch": f"{len(host)} scenes of 4 or 8 bands, PAN sides {sides}",
            "warmstart": f"{len(host)} held-out scenes of 8 bands, PAN 512x512"}[name]
    return (f"{what} (x{c}), Gaussian blurs of {taps} taps, r={st.r}, lambda={st.lam}, eps={st.eps}, "
            f"tol={st.tol} on the FP64 residual; {pxb / 1e6:.1f} Mpixel*bands per step")


if __name__ == "__main__":
    main()
