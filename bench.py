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
Prints one JSON line.  Beside the headline it carries:
* ``fp32_plain``: the same steps with FP32 operands (the metric's comparison);
* ``time_to_objective``: online learning over 100 mini-batches in both
  precisions, with the training time until a held-out objective reaches FP32's
  final one;
* ``ragged``: code steps of the 256-image ragged batch (sides in [64, 512]) in
  both precisions, with per-kernel rooflines;
* ``unrolled``: forward and backward through 10 unrolled layers on 32 images
  128 x 128 with K = 256, both precisions, with the dense adjoint's roofline;
* ``hold_vs_project``: on the batch workload, the objective against training
  time with the unselected codes zeroed (eq. 4) and held (the randomization
  paragraph of Sec. 3.1);
* ``inpainting``: the reconstruction PSNR from half of the pixels (Sec. 4) with
  filters learned online;
* ``solver_compare``: ISTA against the paper's ADMM on one mini-batch;
* ``paper_reference``: the paper's own CPU timings, with their hardware;
* ``cpu_baseline``: the FP64 oracle's code step on the host cores.
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
PEAK_FP64_VECTOR = 78.6e12
PEAK_BF16_MFMA = 2.5e15
PEAK_HBM = 8.0e12
# LDS: 128 bytes per clock per CU (256 CUs, 2.4 GHz); one FP64 product of the lag pass is an
# 8-byte atomic read-modify-write in LDS (8 bytes read, 8 written), so 8 products per clock per CU
PEAK_LDS_BYTES = 256 * 2.4e9 * 128
PEAK_LAG_PRODUCTS = PEAK_LDS_BYTES / 16

# HBM bytes per launch of each kernel class's main kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes scaled by a 512 MiB copy (read x 2.000, write x 1.000), valid only for the kernel source
# they were taken on (first 16 hex digits of its SHA-256).  Keyed by (workload, kernel class,
# precision): (source, digest, bytes read, bytes written), taken on the launch variant with the
# most dispatches in the per-class timing pass (the tuned one; named after each entry).  The
# BF16 synthesis and adjoint are taken on their full-batch launches (the per-class timing pass
# launches those; the eager headline splits the batch over three streams).
TRAFFIC = {
    ("online", "synth", "bf16"): ("kernels_mfma.hip", "a5c6d6ec6d723eb8", 18.56e6, 0.8036e6),  # k_synth_mfma<11, 1> (full batch)
    ("online", "adjoint", "bf16"): ("kernels_code.hip", "41c438702764e40d", 20.98e6, 10.64e6),  # k_adjoint_shrink_mfma<11, true> (full batch)
    ("online", "corr", "bf16"): ("kernels_dict.hip", "5dba40135f457554", 27.01e6, 4.067e6),  # k_corr_fm<11>
    ("online", "sur_expand", "bf16"): ("kernels_sur.hip", "d57f51a0e58c130e", 772.5e6, 653.2e6),  # k_sur_expand<11>
    ("online", "power", "bf16"): ("kernels_sur.hip", "d57f51a0e58c130e", 18.22e6, 0.6944e6),  # k_lag_matvec<11>
    ("online", "synth", "fp32"): ("kernels_code.hip", "41c438702764e40d", 18.07e6, 0.802e6),  # k_synth<11, true, 16, 8, 4>
    ("online", "adjoint", "fp32"): ("kernels_code.hip", "41c438702764e40d", 20.93e6, 10.63e6),  # k_adjoint_shrink<11>
    ("online", "corr", "fp32"): ("kernels_dict.hip", "5dba40135f457554", 27.01e6, 4.067e6),  # k_corr_fm<11>
    ("online", "sur_expand", "fp32"): ("kernels_sur.hip", "d57f51a0e58c130e", 772.5e6, 653.2e6),  # k_sur_expand<11>
    ("online", "power", "fp32"): ("kernels_sur.hip", "d57f51a0e58c130e", 18.22e6, 0.6944e6),  # k_lag_matvec<11>
    ("batch", "synth", "bf16"): ("kernels_mfma.hip", "a5c6d6ec6d723eb8", 9.634e6, 0.4036e6),  # k_synth_mfma<11, 2> (full batch)
    ("batch", "adjoint", "bf16"): ("kernels_code.hip", "41c438702764e40d", 10.91e6, 5.289e6),  # k_adjoint_shrink_mfma<11, true> (full batch)
    ("batch", "power", "bf16"): ("kernels_sur.hip", "d57f51a0e58c130e", 18.22e6, 0.6944e6),  # k_lag_matvec<11>
    ("batch", "corr", "bf16"): ("kernels_mfma.hip", "a5c6d6ec6d723eb8", 7.659e6, 23.72e6),  # k_corr_mfma<11>
    ("batch", "synth", "fp32"): ("kernels_code.hip", "41c438702764e40d", 9.881e6, 0.4031e6),  # k_synth<11, true, 16, 8, 4>
    ("batch", "adjoint", "fp32"): ("kernels_code.hip", "41c438702764e40d", 10.91e6, 5.289e6),  # k_adjoint_shrink<11>
    ("batch", "power", "fp32"): ("kernels_sur.hip", "d57f51a0e58c130e", 18.22e6, 0.6944e6),  # k_lag_matvec<11>
    ("batch", "corr", "fp32"): ("kernels_dict.hip", "5dba40135f457554", 13.77e6, 4.067e6),  # k_corr_fm<11>
    ("ragged", "synth", "bf16"): ("kernels_mfma.hip", "a5c6d6ec6d723eb8", 1845e6, 85.04e6),  # k_synth_mfma<11, 1> (full batch)
    ("ragged", "adjoint", "bf16"): ("kernels_code.hip", "41c438702764e40d", 2170e6, 1349e6),  # k_adjoint_shrink_mfma<11, true> (full batch)
    ("ragged", "gather", "bf16"): ("kernels_code.hip", "41c438702764e40d", 9798e6, 184.7e6),  # k_gather_selected
    ("ragged", "scatter", "bf16"): ("kernels_code.hip", "41c438702764e40d", 1920e6, 8765e6),  # k_scatter_dense
    ("ragged", "synth", "fp32"): ("kernels_code.hip", "41c438702764e40d", 3462e6, 129.1e6),  # k_synth<11, true, 16, 8, 4>
    ("ragged", "adjoint", "fp32"): ("kernels_code.hip", "41c438702764e40d", 2224e6, 1404e6),  # k_adjoint_shrink<11>
    ("ragged", "gather", "fp32"): ("kernels_code.hip", "41c438702764e40d", 9798e6, 184.7e6),  # k_gather_selected
    ("ragged", "scatter", "fp32"): ("kernels_code.hip", "41c438702764e40d", 1921e6, 8766e6),  # k_scatter_dense
}


# The paper's own timings (end-to-end CPU wall times on a Core i7 PC with Matlab built-in
# functions, ADMM code solver; no GPU figures, no precision stated).  Context, not the target.
PAPER_REFERENCE = {
    "hardware": "Core i7 PC, Matlab built-in functions (the mini-batch study single-core)",
    "sbcsc_fruit": "10 images 100x100, K=100 filters 11x11, p=0.1: 170 s for 14 outer iterations of 10 ADMM "
                   "iterations each (Heide et al. 2015: 350 s); per outer iteration about 6x faster than the "
                   "non-subsampled spatial solver and about 2x faster than Fourier-domain ADMM",
    "socsc_fruit": "the 10 training images, one per iteration: 70 s (Liu et al. 2018: 440 s)",
    "minibatch": "1000 patches 100x100, K=400: mini-batches of 20 reach a comparable objective about 10x sooner "
                 "than single images",
    "derived_updates_per_s": 8.2e5,
    "derived_note": "not printed in the paper: 1e6 sampled coordinates per outer iteration x 10 ADMM iterations "
                    "x 14 outer iterations in 170 s, whole pipeline",
}


def traffic_for(cls, workload, precision):
    """Calibrated HBM bytes per launch, or None when the kernel changed since the counters were taken."""
    import hashlib

    key = (workload, cls, precision)
    if key not in TRAFFIC:
        return None
    src, sha, rd, wr = TRAFFIC[key]
    path = os.path.join(ROOT, "paper_1909_00145_amd", "csrc", src)
    try:
        cur = hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    return rd + wr if cur == sha else None

WORKLOADS = {
    "online": dict(N=20, H=100, W=100, K=100, m=11, p=0.1, lam=1.0, T=20, cfg=3,
                   name="online SOCSC: mini-batches of 20 images 100x100 (1/f^2), K=100 filters 11x11, "
                        "p=0.1, lambda=1, 20 ISTA iterations, FP64 surrogates"),
    "batch": dict(N=10, H=100, W=100, K=100, m=11, p=0.1, lam=1.0, T=20, cfg=2,
                  name="batch SBCSC: 10 images 100x100 (1/f^2), K=100 filters 11x11, p=0.1, lambda=1, "
                       "20 ISTA iterations + 1 projected filter step"),
    "ragged": dict(N=256, H=None, W=None, K=100, m=11, p=0.1, lam=0.5, T=30, cfg=4,
                   name="ragged code step: 256 images with sides uniform in [64, 512] (1/f^2), K=100 filters "
                        "11x11, p=0.1, lambda=0.5, 30 ISTA iterations in one batch"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the first five code steps of a new shape tune the launch variants (the synthesis
    # alone, then a screening of the split pairs and one call per finalist), so the
    # default warm-up covers them
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="online")
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="bf16",
                    help="bf16: MFMA operands in BF16 with FP32 accumulation (the configured path); "
                         "fp32: plain FP32")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the timed run of the other precision (FP32 plain next to BF16)")
    ap.add_argument("--p", type=float, default=None, help="override the sampling rate")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="launch the code step's iterations one by one (the default): the library then splits "
                         "them over three streams")
    ap.add_argument("--graph", action="store_true",
                    help="replay the code step's iterations and the power iteration from HIP graphs, on one stream")
    ap.add_argument("--no-tto", action="store_true",
                    help="skip the time-to-objective comparison of online learning, FP32 against BF16 "
                         "(100 mini-batches each; a few seconds)")
    ap.add_argument("--tto-batches", type=int, default=100, help="mini-batches of the time-to-objective run")
    ap.add_argument("--tto-study", action="store_true",
                    help="also run the study of the held-out objective during online learning (p = 0.1 and 1 on "
                         "streams with 2 px, 8 px and no local contrast normalisation; about a minute)")
    ap.add_argument("--no-ragged", action="store_true",
                    help="skip the ragged-batch leg (256 images with sides in [64, 512], one code step per timed "
                         "step in BF16 and FP32 with per-kernel rooflines; about 20 s)")
    ap.add_argument("--ragged-steps", type=int, default=2, help="timed code steps of the ragged leg per precision")
    ap.add_argument("--no-lag-pairs", action="store_true",
                    help="skip the replay of the online steps that counts the lag pass's products (its roofline)")
    ap.add_argument("--no-unrolled", action="store_true",
                    help="skip the differentiation leg (10 unrolled layers on 32 images 128x128, K=256, forward "
                         "and backward in BF16 and FP32; a few seconds)")
    ap.add_argument("--no-hold-compare", action="store_true",
                    help="skip the batch-workload comparison of the objective against training time with the "
                         "unselected codes held (HOLD) and zeroed (PROJECT); about a second on one GPU")
    ap.add_argument("--hold-iters", type=int, default=60, help="outer iterations of the HOLD/PROJECT comparison")
    ap.add_argument("--no-inpaint", action="store_true",
                    help="skip the inpainting leg (10 synthetic 256x256 images, 50 %% observed, lambda 0.4, "
                         "50 iterations, 5 trials, with filters learned online); a few seconds")
    ap.add_argument("--inpaint-train", type=int, default=60, help="mini-batches of online learning before inpainting")
    ap.add_argument("--no-solver-compare", action="store_true",
                    help="skip the code-solver comparison on one mini-batch: ISTA against the paper's ADMM "
                         "(rho = 10 lambda, alpha = 1.8, 5 CG iterations per step), FP32")
    ap.add_argument("--eta-sweep", default="",
                    help="comma-separated mini-batch sizes: online learning of an over-complete dictionary "
                         "(--sweep-K filters) over the same --sweep-samples images for each size, with the "
                         "held-out objective against training time (e.g. 1,5,20,50)")
    ap.add_argument("--sweep-K", type=int, default=400)
    ap.add_argument("--sweep-samples", type=int, default=200)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many MiB 3 times (a traffic-counter "
                         "calibration kernel of known size; outside the timed region)")
    return ap.parse_args()


def cpu_baseline(w, budget_s, sizes):
    """Time the FP64 oracle's code step on a bounded sample of the same workload,
    once with the BLAS pool at its default size and once with one thread.

    sizes: (H, W) of the images of one step, in order; image n of the sample is
    image n of the step.  Each pass codes images until it has run for budget_s / 2
    or the step's images are done.  The oracle's filter step is not timed: its
    dense surrogate and code matrices (about 1 GB per image at this size) take
    minutes per mini-batch."""
    import platform

    import oracle
    import scsc_inputs as si

    try:
        from threadpoolctl import threadpool_info, threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_info = threadpool_limits = None
    blas = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1]) if threadpool_info else 1
    host_cores = len(os.sched_getaffinity(0))
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next(ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name"))
    except (OSError, StopIteration):
        pass
    d = si.filters(w["cfg"], w["K"], w["m"]).astype(np.float32).astype(np.float64)
    Lz = oracle.lipschitz_code(d, int(max(max(hw) for hw in sizes)))
    xs = [si.field(w["cfg"], n, int(H), int(W)).astype(np.float32).astype(np.float64)
          for n, (H, W) in enumerate(sizes)]

    def run():
        t0 = time.perf_counter()
        updates = n = 0
        while n < len(sizes):
            H, W = xs[n].shape
            z, S = oracle.code_step(xs[n], d, np.zeros((w["K"], H, W)), w["lam"], w["p"], 1, 1, w["T"],
                                    step=1.0 / Lz, image_index=n)
            updates += int(S.sum()) * w["T"]
            n += 1
            if time.perf_counter() - t0 > budget_s / 2:
                break
        el = time.perf_counter() - t0
        return updates / el, n, el

    v_all, n_all, el_all = run()
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            v_one, n_one, el_one = run()
    else:  # pragma: no cover
        v_one, n_one, el_one = None, 0, 0.0
    return {
        "value": v_all,
        "unit": "updates/s",
        "cores": min(blas, host_cores),
        "kind": "oracle",
        "sample": "code step (%d ISTA iterations, p=%g) of %d of the %d images of one step, FP64 NumPy, "
                  "%.1f s with the BLAS pool at %d threads; filter step not included"
                  % (w["T"], w["p"], n_all, len(sizes), el_all, blas),
        "value_1thread": v_one,
        "sample_1thread": "the same code step of %d images with the BLAS pool at 1 thread, %.1f s" % (n_one, el_one),
        "cpu_model": model,
        "host_cores": host_cores,
        "os_cpu_count": os.cpu_count(),
        "blas_threads": blas,
    }


def online_curve(ctx, w, xs, him, held, precision, p, n_batches, lcn_note="", full=False):
    """Online learning from the workload's initial filters over the mini-batches xs,
    with the held-out objective (eq. 1, FP64) after every mini-batch, clock stopped.
    The held-out codes come from the training's own code update (rate p, w["T"] FP32
    iterations from zero, one fixed sample: draw 0, which no training step uses).
    Returns [(training seconds, F)] starting with the initial filters at 0 s, and
    with full=True also the held-out objective with codes over every coordinate
    (p = 1, 300 iterations) at the start and the end, and L_z of the final filters."""
    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd.drivers import OnlineLearner
    from paper_1909_00145_amd.ops import Images

    K, m, N, H, W = w["K"], w["m"], w["N"], w["H"], w["W"]
    im = Images.uniform(N, H, W)
    d = torch.from_numpy(si.filters(w["cfg"], K, m).astype(np.float32)).cuda()
    learner = OnlineLearner(ctx, im, d, w["lam"], p, n_code_iter=w["T"], precision=precision)
    extra = [learner.evaluate(him, held, n_iter=300, p=1.0)[0]] if full else []
    elapsed, curve = 0.0, [(0.0, learner.evaluate(him, held, n_iter=w["T"], p=p)[0])]
    for t in range(n_batches):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        learner.step(xs[t])
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        curve.append((elapsed, learner.evaluate(him, held, n_iter=w["T"], p=p)[0]))
    if full:
        extra.append(learner.evaluate(him, held, n_iter=300, p=1.0)[0])
        extra.append(ctx.lipschitz_code(learner.d, max(H, W)))
    return curve, extra


def time_to_objective(ctx, w, n_batches):
    """Online learning over a stream of n_batches mini-batches in FP32 and in BF16,
    from the same filters on the same stream.

    The stream has the online workload's shape and settings, with 1/f^2 fields that
    are only z-scored: on the locally contrast-normalised stream of the headline
    (2 px windows) the held-out objective falls for one mini-batch and then rises,
    at any sampling rate, so no time to an objective can be read off it
    (``--tto-study`` runs both streams).  After every mini-batch the held-out
    objective (eq. 1, FP64) is evaluated with the clock stopped, on 20 held-out
    images whose codes come from the code update the learner trains with (p and T
    of the workload, from zero, FP32, one fixed sample).  The target F* is the
    lowest held-out objective FP32 reaches; each precision reports the training
    time until its held-out objective first reaches F* (1 + 1e-3), and the two final
    objectives are compared (equal within 1e-3 relative)."""
    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd.ops import Images

    N, H, W = w["N"], w["H"], w["W"]
    xs = torch.from_numpy(np.stack([si.stream_batch(w["cfg"], t, N, H, W, lcn_sigma=None).astype(np.float32)
                                    .reshape(-1) for t in range(1, n_batches + 1)])).cuda()
    held = torch.from_numpy(si.batch(33, 20, H, W, lcn_sigma=None).astype(np.float32).reshape(-1)).cuda()
    him = Images.uniform(20, H, W)
    curves, full = {}, {}
    for prec in ("fp32", "bf16"):
        curves[prec], full[prec] = online_curve(ctx, w, xs, him, held, prec, w["p"], n_batches, full=True)
    best = min(range(1, n_batches + 1), key=lambda i: curves["fp32"][i][1])
    target = curves["fp32"][best][1]
    out = {"stream": "%d mini-batches of %d images %dx%d, 1/f^2 fields z-scored without local contrast "
                     "normalisation (cfg %d); K=%d, p=%g, lambda=%g, %d ISTA iterations"
                     % (n_batches, N, H, W, w["cfg"], w["K"], w["p"], w["lam"], w["T"]),
           "target_F": target, "target_mini_batch_fp32": best, "tolerance": 1e-3, "mini_batches": n_batches,
           "eval": "held-out 20 images 100x100 (cfg 33, same generator): codes from zero by the training's code "
                   "update (p=%g, %d FP32 iterations, one fixed sample), objective of eq. (1) in FP64, lambda=%g"
                   % (w["p"], w["T"], w["lam"]),
           "criterion": "first mini-batch whose held-out objective is <= F* (1 + 1e-3), F* = the lowest one "
                        "FP32 reaches over the run"}
    ref = [F for _, F in curves["fp32"]]
    for prec, curve in curves.items():
        hit = next((i for i in range(1, len(curve)) if curve[i][1] <= target * (1.0 + 1e-3)), None)
        out[prec] = {"seconds": curve[hit][0] if hit is not None else None,
                     "mini_batches": hit,
                     "initial_F": curve[0][1], "min_F": min(F for _, F in curve[1:]), "final_F": curve[-1][1],
                     "train_seconds": curve[-1][0],
                     "final_rel_diff_from_fp32": abs(curve[-1][1] - ref[-1]) / abs(ref[-1]),
                     "max_rel_dev_from_fp32": max(abs(F - r) / abs(r) for (_, F), r in zip(curve, ref)),
                     "F_after": {str(t): round(curve[t][1], 3) for t in (1, 2, 5, 10, 20, 50, 100)
                                 if t < len(curve)},
                     "heldout_p1_300iters_initial_final": [round(v, 3) for v in full[prec][:2]],
                     "final_L_z": full[prec][2]}
    if out["fp32"]["seconds"] and out["bf16"]["seconds"]:
        out["fp32_over_bf16_time"] = out["fp32"]["seconds"] / out["bf16"]["seconds"]
    out["fp32_over_bf16_time_per_mini_batch"] = out["fp32"]["train_seconds"] / out["bf16"]["train_seconds"]
    return out


def tto_study(ctx, w, n_batches):
    """Why the held-out objective of online learning rises on the default stream:
    FP32 online learning from the same filters for p = 0.1 and p = 1, on streams
    whose local contrast normalisation uses Gaussian windows of 2 px (the default),
    8 px, or none.  Reports the held-out objective under the training's code update
    and with codes over every coordinate (p = 1, 300 iterations), and L_z of the
    final filters (how coherent the dictionary has become)."""
    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd.ops import Images

    N, H, W = w["N"], w["H"], w["W"]
    him = Images.uniform(20, H, W)
    out = {"mini_batches": n_batches, "precision": "fp32",
           "L_z_initial": ctx.lipschitz_code(
               torch.from_numpy(si.filters(w["cfg"], w["K"], w["m"]).astype(np.float32)).cuda(), max(H, W))}
    for sig in (2.0, 8.0, None):
        xs = torch.from_numpy(np.stack([si.stream_batch(w["cfg"], t, N, H, W, lcn_sigma=sig).astype(np.float32)
                                        .reshape(-1) for t in range(1, n_batches + 1)])).cuda()
        held = torch.from_numpy(si.batch(33, 20, H, W, lcn_sigma=sig).astype(np.float32).reshape(-1)).cuda()
        for p in (w["p"], 1.0):
            curve, full = online_curve(ctx, w, xs, him, held, "fp32", p, n_batches, full=True)
            progress("study: stream lcn=%s p=%g done" % (sig, p))
            out["lcn_%s_p%g" % ("none" if sig is None else "%gpx" % sig, p)] = {
                "F_after": {str(t): round(curve[t][1], 1) for t in (0, 1, 2, 5, 10, 20, 50, 100) if t < len(curve)},
                "heldout_p1_300iters_initial_final": [round(v, 1) for v in full[:2]],
                "final_L_z": round(full[2], 1)}
        del xs, held
    return out


def hold_vs_project(ctx, w, n_outer, precision):
    """Batch learning (Alg. 1) on the batch workload with the unselected codes
    zeroed (PROJECT, eq. 4) and held (HOLD, Sec. 3.1), from the same filters and
    the same samples.  After every outer iteration the objective of eq. (1) over
    the batch is evaluated with the clock stopped; reports both curves against
    training time and the objectives at the time the faster mode finishes."""
    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd.drivers import BatchLearner
    from paper_1909_00145_amd.ops import Images

    K, m, N, H, W = w["K"], w["m"], w["N"], w["H"], w["W"]
    im = Images.uniform(N, H, W)
    x = torch.from_numpy(si.batch(w["cfg"], N, H, W).astype(np.float32).reshape(-1)).cuda()
    curves = {}
    for mode in ("project", "hold"):
        d = torch.from_numpy(si.filters(w["cfg"], K, m).astype(np.float32)).cuda()
        learner = BatchLearner(ctx, im, x, d, w["lam"], w["p"], n_code_iter=w["T"], precision=precision,
                               hold=mode == "hold")
        elapsed, curve = 0.0, []
        for _ in range(n_outer):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            learner.step()
            torch.cuda.synchronize()
            elapsed += time.perf_counter() - t0
            curve.append((elapsed, learner.objective()[0]))
        curves[mode] = curve

    def at(curve, t):
        """Objective of the last evaluation at or before time t."""
        F = curve[0][1]
        for el, f in curve:
            if el <= t:
                F = f
        return F

    t_eq = min(c[-1][0] for c in curves.values())
    out = {"workload": w["name"], "precision": precision, "outer_iterations": n_outer,
           "eval": "objective of eq. (1) over the batch after each outer iteration (clock stopped)",
           "equal_time_s": t_eq}
    for mode, c in curves.items():
        out[mode] = {"train_seconds": c[-1][0], "ms_per_outer": 1e3 * c[-1][0] / n_outer, "final_F": c[-1][1],
                     "F_at_equal_time": at(c, t_eq), "F_every_10": [round(f, 2) for _, f in c[9::10]]}
    return out


def inpainting(ctx, w, n_train, precision):
    """Inpainting as in Sec. 4: 10 held-out synthetic 256 x 256 images, each pixel
    observed with probability 0.5, codes of the masked problem over every
    coordinate (lambda = 0.4, 50 iterations from zero), reconstruction D z.  PSNR
    (peak = the original's dynamic range, all pixels) averaged over the images
    and 5 observation masks, for the filters after n_train mini-batches of online
    learning (the online workload's stream and settings), for the initial filters,
    and for filling the unobserved pixels with zeros.  The reconstruction time is the
    median over the timed reconstructions (and per filter set: the code sparsity, and
    so the work, differs between them), after six untimed ones that settle the
    launch-variant tuning of the 256 x 256 batch."""
    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd.drivers import OnlineLearner, inpaint, psnr
    from paper_1909_00145_amd.ops import Images

    K, m, N, H, W = w["K"], w["m"], w["N"], w["H"], w["W"]
    d0 = torch.from_numpy(si.filters(w["cfg"], K, m).astype(np.float32)).cuda()
    learner = OnlineLearner(ctx, Images.uniform(N, H, W), d0.clone(), w["lam"], w["p"], n_code_iter=w["T"],
                            precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(1, n_train + 1):
        learner.step(torch.from_numpy(si.stream_batch(w["cfg"], t, N, H, W).astype(np.float32).reshape(-1)).cuda())
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    NT, HT, WT, trials, lam, iters = 10, 256, 256, 5, 0.4, 50
    im = Images.uniform(NT, HT, WT)
    x = torch.from_numpy(si.batch(33, NT, HT, WT).astype(np.float32).reshape(-1)).cuda()
    res = {"learned": [], "initial": [], "zero_fill": []}
    times, by = [], {"learned": [], "initial": []}
    # the first five code steps of this shape tune its launch variants: untimed
    W0 = torch.from_numpy(np.stack([si.observation_mask(50, n, HT, WT) for n in range(NT)]).reshape(-1)).cuda()
    for _ in range(6):
        inpaint(ctx, im, x, W0, d0, lam, iters, precision=precision)
    for tr in range(trials):
        Wm = torch.from_numpy(np.stack([si.observation_mask(50 + tr, n, HT, WT) for n in range(NT)])
                              .reshape(-1)).cuda()
        res["zero_fill"] += psnr(im, x * Wm, x)
        for name, d in (("learned", learner.d), ("initial", d0)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xh, _ = inpaint(ctx, im, x, Wm, d, lam, iters, precision=precision)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            by[name].append(times[-1])
            res[name] += psnr(im, xh, x)
    return {"images": "%d held-out synthetic %dx%d fields (1/f^2)" % (NT, HT, WT), "observed": 0.5,
            "lambda": lam, "iterations": iters, "trials": trials, "precision": precision,
            "train": "%d online mini-batches (%.2f s)" % (n_train, train_s),
            "psnr_db": {k: round(float(np.mean(v)), 3) for k, v in res.items()},
            "ms_per_reconstruction": round(1e3 * float(np.median(times)), 1),
            "ms_per_reconstruction_by_filters": {k: round(1e3 * float(np.median(v)), 1) for k, v in by.items()}}


def eta_sweep(ctx, w, K, etas, n_samples, precision):
    """Mini-batch size sweep of online learning (Alg. 2 with mini-batches of eta
    images; the over-complete experiment of Sec. 4): for each eta, K filters from
    the same initial bank learn from the same stream of n_samples images.  About ten
    times per run the held-out objective (20 images, codes from zero at p = 1, 50
    FP32 iterations) is evaluated with the clock stopped."""
    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd.drivers import OnlineLearner
    from paper_1909_00145_amd.ops import Images

    m, H, W = w["m"], w["H"], w["W"]
    stream = si.batch(w["cfg"], n_samples, H, W).astype(np.float32)
    held = torch.from_numpy(si.batch(33, 20, H, W).astype(np.float32).reshape(-1)).cuda()
    him = Images.uniform(20, H, W)
    out = {"K": K, "m": m, "images": "%dx%d" % (H, W), "samples": n_samples, "precision": precision,
           "eval": "held-out objective of eq. (1): 20 images, codes from zero at p = 1, 50 FP32 iterations"}
    for eta in etas:
        im = Images.uniform(eta, H, W)
        d = torch.from_numpy(si.filters(w["cfg"], K, m).astype(np.float32)).cuda()
        learner = OnlineLearner(ctx, im, d, w["lam"], w["p"], n_code_iter=w["T"], precision=precision)
        steps = n_samples // eta
        every = max(1, steps // 10)
        elapsed, curve = 0.0, []
        for t in range(steps):
            x = torch.from_numpy(stream[t * eta:(t + 1) * eta].reshape(-1)).cuda()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            learner.step(x)
            torch.cuda.synchronize()
            elapsed += time.perf_counter() - t0
            if (t + 1) % every == 0 or t == steps - 1:
                curve.append(((t + 1) * eta, round(elapsed, 4), round(learner.evaluate(him, held)[0], 2)))
        out["eta_%d" % eta] = {"steps": steps, "ms_per_step": round(1e3 * elapsed / steps, 2),
                               "train_seconds": round(elapsed, 3), "final_F": curve[-1][2],
                               "curve_samples_seconds_F": curve}
        del learner
        torch.cuda.empty_cache()
    return out


def solver_compare(ctx, w):
    """Code solvers on one mini-batch of the online workload from zero codes, FP32:
    ISTA (the path's solver) for several iteration counts against the paper's ADMM
    (Sec. 3.2: rho = 10 lambda, alpha = 1.8, CG for the quadratic substep) for
    several ADMM iteration counts.  Reports the time of each code update and the
    objective of eq. (1) over the batch of the codes it returns (p = 0.1 sample)."""
    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd.ops import Images

    K, m, N, H, W = w["K"], w["m"], w["N"], w["H"], w["W"]
    im = Images.uniform(N, H, W)
    x = torch.from_numpy(si.stream_batch(w["cfg"], 1, N, H, W).astype(np.float32).reshape(-1)).cuda()
    d = torch.from_numpy(si.filters(w["cfg"], K, m).astype(np.float32)).cuda()
    z = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")

    def timed(fn):
        fn()  # first call sizes the workspaces
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0)

    out = {"batch": "%d images %dx%d, K=%d, %dx%d, p=%g, lambda=%g, from zero codes, FP32" % (N, H, W, K, m, m,
                                                                                             w["p"], w["lam"]),
           "objective": "eq. (1) over the batch"}
    for T in (5, 10, 20, 40):
        def run():
            z.zero_()
            ctx.code_step(im, x, d, z, w["lam"], w["p"], 1, 1, T)
        ms = timed(run)
        out["ista_%d" % T] = {"ms": round(ms, 2), "F": round(ctx.objective(im, x, d, z, w["lam"])[0], 2)}
    for n_admm in (2, 5, 10, 20):
        def run():
            z.zero_()
            ctx.code_step_admm(im, x, d, z, w["lam"], w["p"], 1, 1, n_admm, 5)
        ms = timed(run)
        out["admm_%d" % n_admm] = {"ms": round(ms, 2), "F": round(ctx.objective(im, x, d, z, w["lam"])[0], 2)}
    return out


def progress(msg):
    """One line per finished leg on stderr (the JSON result goes to stdout at the end)."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def workload_inputs(wname, w, n_steps):
    """Batch geometry and device-resident inputs of a workload (generated before any timing)."""
    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd.ops import Images

    if wname == "ragged":
        im = Images(si.ragged_sizes(w["cfg"], w["N"], 64, 512))
    else:
        im = Images.uniform(w["N"], w["H"], w["W"])
    if wname == "online":
        x = torch.from_numpy(np.stack([si.stream_batch(w["cfg"], t, w["N"], w["H"], w["W"]).astype(np.float32)
                                       .reshape(-1) for t in range(1, n_steps + 1)])).cuda()
    elif wname == "ragged":
        x = torch.from_numpy(im.pack([si.field(w["cfg"], n, int(H), int(Wd)).astype(np.float32)
                                      for n, (H, Wd) in enumerate(im.hw)])).cuda()
    else:
        x = torch.from_numpy(si.batch(w["cfg"], w["N"], w["H"], w["W"]).astype(np.float32).reshape(-1)).cuda()
    return im, x


def timed_run(ctx, wname, w, im, x, precision, graph, profile, warmup, steps):
    """Warm-up and timed steps of a workload in one precision, from the initial filters.

    graph: replay the code step's iterations from a HIP graph; profile: time every
    kernel class with HIP events that its kernels record at their own start and end on
    the library's stream (which needs eager launches to attribute the code step's
    kernels)."""
    import ctypes as C

    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd import _lib
    from paper_1909_00145_amd.drivers import BatchLearner, OnlineLearner

    K, m = w["K"], w["m"]
    ctx.set_graph(graph)
    d = torch.from_numpy(si.filters(w["cfg"], K, m).astype(np.float32)).cuda()
    if wname == "online":
        learner = OnlineLearner(ctx, im, d, w["lam"], w["p"], n_code_iter=w["T"], precision=precision)

        def step(i):
            return learner.step(x[i])
    elif wname == "ragged":
        z = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")

        def step(i):
            st = ctx.code_step(im, x, d, z, w["lam"], w["p"], w["cfg"], i + 1, w["T"], precision=precision,
                               stats=True)
            return st, None
    else:
        learner = BatchLearner(ctx, im, x, d, w["lam"], w["p"], n_code_iter=w["T"], precision=precision)

        def step(i):
            return learner.step()

    # timing on (one stream, full-batch launches) already for the warm-up, so that it runs
    # the timed pass's launch configuration; enabling again clears the counters
    ctx.lib.csc_profile_enable(ctx.h, 1 if profile else 0)
    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    ctx.lib.csc_profile_enable(ctx.h, 1 if profile else 0)
    r = {"sampled": 0, "nnz_iter": 0, "nnz_dict": 0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, warmup + steps):
        st, _ = step(i)
        r["sampled"] += st.sampled
        r["nnz_iter"] += st.nnz_iter_sum
        r["nnz_dict"] += st.nnz
    torch.cuda.synchronize()
    r["el"] = time.perf_counter() - t0
    kernels = {}
    for ci, name in enumerate(_lib.KERNEL_CLASSES):
        n = C.c_int64()
        ms = C.c_double()
        ctx.lib.csc_profile_read(ctx.h, ci, C.byref(n), C.byref(ms))
        if n.value:
            kernels[name] = {"launches": int(n.value), "avg_us": 1e3 * ms.value / n.value, "total_ms": ms.value}
    ctx.lib.csc_profile_enable(ctx.h, 0)
    r["kernels"] = kernels
    return r


def lag_pairs(z, im, K, m):
    """Products of the lag pass over codes z (packed [K][H][W] per image): every pair of a
    non-zero code at pixel q and one at q + delta, for the lags delta = (dy, dx) with dy > 0,
    or dy = 0 and dx >= 0, inside the window (|dx|, dy <= m - 1), both pixels in the image.
    The per-pixel counts are formed on the device; the pairs are summed on the host in
    integers, a batch of equal-sized images at a time."""
    import torch

    r = m - 1
    groups = {}
    base = 0
    for H, Wd in im.hw:
        H, Wd = int(H), int(Wd)
        groups.setdefault((H, Wd), []).append(base)
        base += K * H * Wd
    total = 0
    for (H, Wd), bases in groups.items():
        if len(bases) > 1 and all(b1 - b0 == K * H * Wd for b0, b1 in zip(bases, bases[1:])):
            n = (z[bases[0]:bases[0] + len(bases) * K * H * Wd].view(len(bases), K, H, Wd) != 0).sum(1)
        else:
            n = torch.stack([(z[b:b + K * H * Wd].view(K, H, Wd) != 0).sum(0) for b in bases])
        n = n.cpu().numpy().astype(np.int64)
        for dy in range(0, min(r, H - 1) + 1):
            for dx in range(-r, r + 1):
                if (dy == 0 and dx < 0) or abs(dx) >= Wd:
                    continue
                xa, xb = max(0, -dx), Wd - max(0, dx)
                total += int((n[:, 0:H - dy, xa:xb] * n[:, dy:H, xa + dx:xb + dx]).sum())
    return float(total)


def lag_pair_count(ctx, w, im, x, precision, warmup, steps):
    """Products of the lag pass summed over the timed steps, from a replay of the same
    online steps that writes every mini-batch's codes (the FP64 atomics of the surrogate
    sums may round the filters differently in the last bit, so the count can differ from
    the timed run's by the few codes that sit at the threshold)."""
    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd.drivers import OnlineLearner

    K, m = w["K"], w["m"]
    ctx.set_graph(False)
    d = torch.from_numpy(si.filters(w["cfg"], K, m).astype(np.float32)).cuda()
    learner = OnlineLearner(ctx, im, d, w["lam"], w["p"], n_code_iter=w["T"], precision=precision, keep_codes=True)
    total = 0.0
    for i in range(warmup + steps):
        learner.step(x[i])
        if i >= warmup:
            total += lag_pairs(learner.z, im, K, m)
    return total


def rooflines(wname, w, im, precision, res, kernels, steps):
    """Roofline object of the dominant modelled kernel class and the fractions of all
    modelled classes, from the algorithmic work of the timed steps (res) and the
    per-class event averages (kernels)."""
    K, m = w["K"], w["m"]
    sampled, nnz_iter, nnz_dict = res["sampled"], res["nnz_iter"], res["nnz_dict"]
    M = m * m
    c = m // 2
    L2 = (2 * m - 1) ** 2
    n_power = 20
    bf16 = precision == "bf16"
    mm_peak = PEAK_BF16_MFMA if bf16 else PEAK_FP32_VECTOR
    mm_bound = "mfma" if bf16 else "alu"
    # Algorithmic work of every timed launch of a kernel class, summed over the timed steps.
    work = {
        # one dot product of M taps per selected coordinate, then u = z + eta g and the shrink
        "adjoint": (mm_bound, (2 * M + 3) * sampled * w["T"], mm_peak),
        # M multiply-adds per non-zero code entering a synthesis
        "synth": (mm_bound, 2 * M * nnz_iter, mm_peak),
        # M multiply-adds per non-zero code of one correlation (B_bar = Z^T x, FP32 in both precisions)
        "corr": ("alu", 2 * M * nnz_dict, PEAK_FP32_VECTOR),
        # K^2 M^2 FP64 multiply-adds per product with the lag-sum normal matrix (20 per step)
        "power": ("alu64", 2.0 * K * K * M * M * n_power * steps, PEAK_FP64_VECTOR),
        # one pass over the blocks (k, k2 >= k) of the FP64 lag-layout matrix (the rest is their transpose)
        "sur_mv": ("hbm", 8.0 * (K * (K + 1) // 2) * M * M * steps, PEAK_HBM),
        # read-modify-write of the stored blocks (k <= k2) of C_bar plus their lag sums and the
        # 4 c^2 (2m - 1) band sums that can be non-zero
        "sur_expand": ("hbm", (K * (K + 1) // 2) * (16.0 * M * M + 8.0 * (L2 + 4 * c * c * (2 * m - 1)))
                       * steps, PEAK_HBM),
        # gather: the K planes of z read once (a Bernoulli(p) sample touches nearly every 64-byte
        # sector), the selection words, offsets and counts; the gathered pairs are not counted,
        # so this is a lower bound
        "gather": ("hbm", (4.0 * K + 4.0 * ((K + 31) // 32) + 6.0) * im.n_pix * steps, PEAK_HBM),
        # scatter: the K planes of z written once, the offsets and counts, and the list entries
        "scatter": ("hbm", (4.0 * K + 6.0) * im.n_pix * steps + 8.0 * nnz_dict, PEAK_HBM),
    }
    if "lag_pairs" in res:
        # one FP64 product (an 8-byte LDS atomic read-modify-write) per pair of non-zero codes at
        # a lag of the half window; the class also holds the tiled sum and the band sums
        work["sur_lag"] = ("lds", res["lag_pairs"], PEAK_LAG_PRODUCTS)
    # MFMA work the BF16 kernels execute per launch (dense tiles, padded shapes), 16x16x32 = 16384 flop
    executed = {}
    if bf16:
        tiles = sum(((int(H) + 15) // 16) * ((int(Wd) + 15) // 16) for H, Wd in im.hw)
        executed["synth"] = tiles * ((K + 7) // 8) * ((m + 3) // 4) * (16 + 2 * c) * 16384.0
        executed["adjoint"] = tiles * ((K + 15) // 16) * 16 * ((M + 31) // 32) * 16384.0
    if wname == "ragged":
        # code steps only
        work = {k: work[k] for k in ("adjoint", "synth", "gather", "scatter")}
    elif wname != "online":
        # batch filter step: one residual synthesis and one gradient correlation; lag-sum power iteration
        work.pop("sur_mv")
        work.pop("sur_expand")
        work["synth"] = (mm_bound, 2 * M * (nnz_iter + nnz_dict), mm_peak)
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    modelled = [k for k in kernels if k in work]
    # the headline roofline stays on a kernel with a flop or byte model
    headline = [k for k in modelled if work[k][0] != "lds"]
    pick = dom if dom in headline else max(headline, key=lambda k: kernels[k]["total_ms"])

    def roof_of(k):
        bound, total_work, peak = work[k]
        avg_s = kernels[k]["avg_us"] * 1e-6
        per_launch = total_work / kernels[k]["launches"]
        if bound == "hbm":
            r = {"bound": "hbm", "achieved": per_launch / avg_s / 1e9, "peak": peak / 1e9, "unit": "GB/s"}
        elif bound == "lds":
            r = {"bound": "lds", "achieved": per_launch / avg_s / 1e9, "peak": peak / 1e9,
                 "unit": "Gproducts/s"}
        else:
            r = {"bound": "alu" if bound == "alu64" else bound, "achieved": per_launch / avg_s / 1e12,
                 "peak": peak / 1e12, "unit": "TFLOP/s"}
            if bound == "alu64":
                r["precision"] = "fp64"
        r["frac"] = r["achieved"] / r["peak"]
        r["traffic"] = traffic_for(k, wname, precision)
        r["kernel"] = k
        r["per_launch_work"] = per_launch
        r["avg_launch_us"] = kernels[k]["avg_us"]
        if k in executed:
            r["executed_mfma_tflops"] = executed[k] / avg_s / 1e12
            r["executed_mfma_frac"] = executed[k] / avg_s / PEAK_BF16_MFMA
        return r

    roof = roof_of(pick)
    if dom != pick:
        roof["dominant_unmodelled"] = dom
    others = {}
    for k in modelled:
        r = roof_of(k)
        others[k] = {key: r[key] for key in ("bound", "achieved", "peak", "unit", "frac", "per_launch_work",
                                             "traffic", "executed_mfma_frac")
                     if key in r}
    return roof, others


def ragged_leg(ctx, steps, warmup):
    """One code step of the ragged batch (256 images, sides uniform in [64, 512], K = 100,
    T = 30) per timed step, BF16 and FP32 plain, with eager launches (the code step split
    over three streams; the warm-up covers the tuning of the split); then the same steps
    on one stream with every kernel class timed by kernel-recorded HIP events, for the
    per-class roofline fractions."""
    import torch

    w = WORKLOADS["ragged"]
    im, x = workload_inputs("ragged", w, 0)
    out = {"workload": w["name"], "pixels": im.n_pix, "steps": steps, "warmup": warmup, "graph": False}
    for prec in ("bf16", "fp32"):
        res = timed_run(ctx, "ragged", w, im, x, prec, False, False, warmup, steps)
        progress("ragged %s timed" % prec)
        prof = timed_run(ctx, "ragged", w, im, x, prec, False, True, 1, steps)
        roof, others = rooflines("ragged", w, im, prec, prof, prof["kernels"], steps)
        out[prec] = {"value": res["sampled"] * w["T"] / res["el"], "unit": "updates/s",
                     "ms_per_step": 1e3 * res["el"] / steps,
                     "roofline": roof, "roofline_all": others,
                     "kernels_avg_us": {k: round(v["avg_us"], 1) for k, v in prof["kernels"].items()}}
        torch.cuda.empty_cache()
        progress("ragged %s: %.1f ms per step" % (prec, out[prec]["ms_per_step"]))
    return out


def unrolled_leg(ctx, reps=2):
    """Differentiation workload: 10 unrolled subsampled-ISTA layers (p = 0.2, lambda =
    0.5, step 1/L_z) on 32 images 128 x 128 with K = 256 filters 11 x 11, loss
    1/2 sum ||x - D z_10||^2, one forward and backward pass through the torch
    Functions per timed run, in BF16 and FP32, with a checkpoint at every layer and
    every 5 layers.  Then a profiled pass for the per-class kernel times; the dense
    adjoint correlation (the layer's D^T r at every coordinate) is the real dense
    contraction here, so its roofline is reported on the matrix cores in BF16."""
    import torch

    import scsc_inputs as si
    from paper_1909_00145_amd import _lib
    from paper_1909_00145_amd.autograd import synthesis, unrolled_ista
    from paper_1909_00145_amd.ops import Images

    N, H, W, K, m, p, lam, T, cfg = 32, 128, 128, 256, 11, 0.2, 0.5, 10, 5
    im = Images.uniform(N, H, W)
    x0 = torch.from_numpy(si.batch(cfg, N, H, W).astype(np.float32).reshape(-1)).cuda()
    d0 = torch.from_numpy(si.filters(cfg, K, m).astype(np.float32)).cuda()
    mask = ctx.mask(im, K, p, cfg, 1)
    eta = 1.0 / ctx.lipschitz_code(d0, max(H, W))
    sampled = int(mask.sum())
    M, MP = m * m, 32 * ((m * m + 31) // 32)
    out = {"workload": "%d images %dx%d, K=%d filters %dx%d, p=%g, lambda=%g, %d unrolled layers, loss "
                       "1/2 sum ||x - D z_T||^2, forward + backward" % (N, H, W, K, m, m, p, lam, T),
           "sampled": sampled}

    def run(prec, every):
        x = x0.clone().requires_grad_(True)
        d = d0.clone().requires_grad_(True)
        z0 = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")
        zT = unrolled_ista(ctx, im, x, d, z0, mask, eta, lam, T, checkpoint_every=every, precision=prec)
        e = x - synthesis(ctx, im, zT, d, precision=prec)
        loss = 0.5 * (e * e).sum()
        loss.backward()
        return float(loss.detach())

    import ctypes as C

    for prec in ("bf16", "fp32"):
        res = {}
        for every in (1, 5):
            run(prec, every)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                loss = run(prec, every)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / reps
            res["checkpoint_every_%d" % every] = {"ms_fwd_bwd": round(ms, 2), "loss": loss,
                                                  "layer_updates_per_s": T * sampled / (ms * 1e-3)}
            torch.cuda.empty_cache()
        ctx.lib.csc_profile_enable(ctx.h, 1)
        run(prec, 1)
        torch.cuda.synchronize()
        kern = {}
        for ci, name in enumerate(_lib.KERNEL_CLASSES):
            n = C.c_int64()
            t = C.c_double()
            ctx.lib.csc_profile_read(ctx.h, ci, C.byref(n), C.byref(t))
            if n.value:
                kern[name] = {"launches": int(n.value), "avg_us": round(1e3 * t.value / n.value, 1)}
        ctx.lib.csc_profile_enable(ctx.h, 0)
        res["kernels"] = kern
        if "dense" in kern:
            avg = kern["dense"]["avg_us"] * 1e-6
            if prec == "bf16":
                # executed: the GEMM over 32-padded taps and 16-padded filters; algorithmic: 2 M K per pixel
                ex = 2.0 * (16 * ((K + 15) // 16)) * MP * im.n_pix
                res["roofline_dense_adjoint"] = {
                    "bound": "mfma", "achieved": 2.0 * M * K * im.n_pix / avg / 1e12, "peak": PEAK_BF16_MFMA / 1e12,
                    "unit": "TFLOP/s", "frac": 2.0 * M * K * im.n_pix / avg / PEAK_BF16_MFMA,
                    "executed_mfma_frac": ex / avg / PEAK_BF16_MFMA, "avg_launch_us": kern["dense"]["avg_us"]}
            else:
                res["roofline_dense_adjoint"] = {
                    "bound": "alu", "achieved": 2.0 * M * K * im.n_pix / avg / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                    "unit": "TFLOP/s", "frac": 2.0 * M * K * im.n_pix / avg / PEAK_FP32_VECTOR,
                    "avg_launch_us": kern["dense"]["avg_us"]}
        out[prec] = res
        progress("unrolled %s: %.1f ms per forward and backward" % (prec, res["checkpoint_every_1"]["ms_fwd_bwd"]))
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the method's hot path is measured on one MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        return 2
    import torch

    from paper_1909_00145_amd.ops import Context

    w = dict(WORKLOADS[args.workload])
    if args.p is not None:
        w["p"] = args.p
    torch.cuda.set_device(0)
    ctx = Context(0)
    K, m = w["K"], w["m"]
    total_steps = args.warmup + args.steps
    im, x = workload_inputs(args.workload, w, total_steps)

    # Eager launches by default: they let the library split the code step over three
    # streams, which beats graph replay on one stream for every workload (online 3.55
    # against 4.24 ms, batch 2.49 against 2.57 ms, ragged 196 against 225 ms per step).
    graph = args.graph and not args.eager
    # the headline run (no event timing), then the same steps eagerly with every kernel
    # class timed by HIP events that its kernels record at their start and end, for the
    # per-kernel figures and the roofline
    res = timed_run(ctx, args.workload, w, im, x, args.precision, graph, False, args.warmup, args.steps)
    el = res["el"]
    progress("headline %s: %.3f ms per step" % (args.precision, 1e3 * el / args.steps))
    prof = timed_run(ctx, args.workload, w, im, x, args.precision, False, True, args.warmup, args.steps)
    kernels = prof["kernels"]
    if (prof["sampled"], prof["nnz_iter"], prof["nnz_dict"]) != (res["sampled"], res["nnz_iter"], res["nnz_dict"]):
        raise RuntimeError("the profiled pass did not repeat the headline run's work")
    if args.workload == "online" and not args.no_lag_pairs:
        res["lag_pairs"] = lag_pair_count(ctx, w, im, x, args.precision, args.warmup, args.steps)

    if args.copy_probe_mb > 0:
        nb = args.copy_probe_mb << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    updates = res["sampled"] * w["T"]
    value = updates / el
    roof, others = rooflines(args.workload, w, im, args.precision, res, kernels, args.steps)
    bf16 = args.precision == "bf16"
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
                   "pixels_per_step": im.n_pix, "graph": graph,
                   "K": K, "filter": m, "p": w["p"], "lambda": w["lam"], "ista_iters": w["T"],
                   "precision": args.precision},
        "roofline": roof,
        "roofline_all": others,
        "kernels": kernels,
        "kernels_note": "per-class averages from an eager pass of the same steps on one stream, timed with "
                        "HIP events that each class's kernels record at their own start and end (%.2f ms per "
                        "step in that pass)" % (1e3 * prof["el"] / args.steps),
        "code_density": res["nnz_dict"] / (args.steps * K * im.n_pix),
    }
    if not args.no_compare:
        other = "fp32" if bf16 else "bf16"
        r2 = timed_run(ctx, args.workload, w, im, x, other, graph, False, args.warmup, args.steps)
        p2 = timed_run(ctx, args.workload, w, im, x, other, False, True, args.warmup, args.steps)
        out["fp32_plain" if other == "fp32" else "bf16"] = {
            "value": r2["sampled"] * w["T"] / r2["el"], "unit": "updates/s",
            "ms_per_step": 1e3 * r2["el"] / args.steps,
            "code_density": r2["nnz_dict"] / (args.steps * K * im.n_pix),
            "kernels_avg_us": {k: round(v["avg_us"], 1) for k, v in p2["kernels"].items()}}
    if not args.no_tto:
        out["time_to_objective"] = time_to_objective(ctx, WORKLOADS["online"], args.tto_batches)
        progress("time to objective done")
    if args.tto_study:
        out["tto_study"] = tto_study(ctx, WORKLOADS["online"], args.tto_batches)
        progress("time-to-objective study done")
    if args.workload == "online" and not args.no_ragged:
        out["ragged"] = ragged_leg(ctx, args.ragged_steps, 6)
        progress("ragged leg done")
    if args.workload == "online" and not args.no_unrolled:
        out["unrolled"] = unrolled_leg(ctx)
    if not args.no_hold_compare:
        out["hold_vs_project"] = hold_vs_project(ctx, WORKLOADS["batch"], args.hold_iters, args.precision)
        progress("hold/project comparison done")
    if not args.no_inpaint:
        out["inpainting"] = inpainting(ctx, WORKLOADS["online"], args.inpaint_train, args.precision)
        other = "fp32" if args.precision == "bf16" else "bf16"
        ip2 = inpainting(ctx, WORKLOADS["online"], args.inpaint_train, other)
        out["inpainting"]["other_precision"] = {k: ip2[k] for k in ("precision", "psnr_db", "ms_per_reconstruction",
                                                                    "ms_per_reconstruction_by_filters")}
        progress("inpainting done")
    if not args.no_solver_compare:
        out["solver_compare"] = solver_compare(ctx, WORKLOADS["online"])
        progress("solver comparison done")
    if args.eta_sweep:
        out["eta_sweep"] = eta_sweep(ctx, WORKLOADS["online"], args.sweep_K,
                                     [int(v) for v in args.eta_sweep.split(",")], args.sweep_samples, args.precision)
    out["paper_reference"] = PAPER_REFERENCE
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, [tuple(hw) for hw in im.hw])
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
