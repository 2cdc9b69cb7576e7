#!/usr/bin/env python3
"""Benchmark of the stochastic-CSC hot path on one MI355X.

Workload (default ``online``): online learning over a stream of synthetic
100 x 100 images (1/f^2 fields, contrast normalised) in mini-batches of 20,
K = 100 filters of 11 x 11, sampling rate p = 0.1, lambda = 1, 20 proximal-
gradient iterations per code update, FP64 surrogates.  One step = one
mini-batch through the whole hot path: selection, gather, 20 x (synthesis +
masked residual, adjoint at the selected coordinates + soft-threshold),
upsampling, non-zero lists, power iteration for L_d, surrogate accumulation
(C_bar, B_bar), the surrogate product and the projected filter update.
The ``batch`` workload is 10 images 100 x 100 with one batch filter update per
outer iteration instead.

Metric: selected code-coordinate updates per second = sum over the timed
steps of (iterations x |S|) / wall time, with the inputs resident in HBM.
Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12
PEAK_HBM = 8.0e12

WORKLOADS = {
    "online": dict(N=20, H=100, W=100, K=100, m=11, p=0.1, lam=1.0, T=20, cfg=3,
                   name="online SOCSC: mini-batches of 20 images 100x100 (1/f^2), K=100 filters 11x11, "
                        "p=0.1, lambda=1, 20 ISTA iterations, FP64 surrogates"),
    "batch": dict(N=10, H=100, W=100, K=100, m=11, p=0.1, lam=1.0, T=20, cfg=2,
                  name="batch SBCSC: 10 images 100x100 (1/f^2), K=100 filters 11x11, p=0.1, lambda=1, "
                       "20 ISTA iterations + 1 projected filter step"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="online")
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="fp32")
    ap.add_argument("--p", type=float, default=None, help="override the sampling rate")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(w, budget_s):
    """Time the FP64 oracle's code step on a bounded sample of the same workload."""
    import oracle
    import scsc_inputs as si

    try:
        from threadpoolctl import threadpool_info

        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = 1
    d = si.filters(w["cfg"], w["K"], w["m"]).astype(np.float32).astype(np.float64)
    Lz = oracle.lipschitz_code(d, max(w["H"], w["W"]))
    t0 = time.perf_counter()
    updates = 0
    n = 0
    while n < w["N"]:
        x = si.field(w["cfg"], n, w["H"], w["W"]).astype(np.float32).astype(np.float64)
        z, S = oracle.code_step(x, d, np.zeros((w["K"], w["H"], w["W"])), w["lam"], w["p"], 1, 1, w["T"],
                                step=1.0 / Lz, image_index=n)
        updates += int(S.sum()) * w["T"]
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {
        "value": updates / el,
        "unit": "updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "code step (%d ISTA iterations, p=%g) of %d of the %d images of the first batch, "
                  "FP64 NumPy, %.1f s; filter step not included" % (w["T"], w["p"], n, w["N"], el),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the method's hot path is measured on one MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        return 2
    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd import _lib
    from paper_1909_00145_amd.drivers import BatchLearner, OnlineLearner
    from paper_1909_00145_amd.ops import Context, Images

    w = dict(WORKLOADS[args.workload])
    if args.p is not None:
        w["p"] = args.p
    torch.cuda.set_device(0)
    ctx = Context(0)
    K, m = w["K"], w["m"]
    im = Images.uniform(w["N"], w["H"], w["W"])
    d = torch.from_numpy(si.filters(w["cfg"], K, m).astype(np.float32)).cuda()
    total_steps = args.warmup + args.steps
    if args.workload == "online":
        xs = torch.from_numpy(np.stack([si.stream_batch(w["cfg"], t, w["N"], w["H"], w["W"]).astype(np.float32)
                                        .reshape(-1) for t in range(1, total_steps + 1)])).cuda()
        learner = OnlineLearner(ctx, im, d, w["lam"], w["p"], n_code_iter=w["T"], precision=args.precision)

        def step(i):
            return learner.step(xs[i])
    else:
        x = torch.from_numpy(si.batch(w["cfg"], w["N"], w["H"], w["W"]).astype(np.float32).reshape(-1)).cuda()
        learner = BatchLearner(ctx, im, x, d, w["lam"], w["p"], n_code_iter=w["T"], precision=args.precision)

        def step(i):
            return learner.step()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    ctx.lib.csc_profile_enable(ctx.h, 1)
    sampled = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, total_steps):
        st, _ = step(i)
        sampled += st.sampled
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kernels = {}
    import ctypes as C

    for ci, name in enumerate(_lib.KERNEL_CLASSES):
        n = C.c_int64()
        ms = C.c_double()
        ctx.lib.csc_profile_read(ctx.h, ci, C.byref(n), C.byref(ms))
        if n.value:
            kernels[name] = {"launches": int(n.value), "avg_us": 1e3 * ms.value / n.value, "total_ms": ms.value}
    ctx.lib.csc_profile_enable(ctx.h, 0)

    updates = sampled * w["T"]
    value = updates / el
    # roofline of the dominant kernel class
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    avg_s = kernels[dom]["avg_us"] * 1e-6
    M = m * m
    if dom == "adjoint":
        per_launch = (sampled / args.steps) * (2 * M + 4)
        roof = {"bound": "alu", "achieved": per_launch / avg_s / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                "unit": "TFLOP/s"}
    elif dom == "sur_mv":
        per_launch = 8.0 * (K * M) ** 2
        roof = {"bound": "hbm", "achieved": per_launch / avg_s / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    else:
        roof = {"bound": "unmodelled", "achieved": None, "peak": None, "unit": None}
    if roof["achieved"] is not None:
        roof["frac"] = roof["achieved"] / roof["peak"]
    else:
        roof["frac"] = None
    roof["kernel"] = dom
    roof["traffic"] = None

    out = {
        "metric": "sampled code-coord updates/sec",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": w["name"], "images_per_step": w["N"], "height": w["H"], "width": w["W"],
                   "K": K, "filter": m, "p": w["p"], "lambda": w["lam"], "ista_iters": w["T"],
                   "precision": args.precision},
        "roofline": roof,
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
