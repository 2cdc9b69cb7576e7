"""Shared helpers of the GPU parity tests: seeded inputs in both precisions and
the normwise error metric.  Inputs come from ``scsc_inputs``; the oracle gets
the FP32-rounded values in FP64 so both sides start from identical data."""

from __future__ import annotations

import sys

import numpy as np
import torch

import scsc_inputs as si


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((got - ref).ravel())
    return float(num / den) if den > 0 else float(num)


def f32(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def make_problem(cfg: int, hw, K: int, m: int, with_W: bool = False):
    """Images (list of FP32-exact float64 arrays), filters, optional masks."""
    xs = [f32(si.field(cfg, i, int(H), int(W))) for i, (H, W) in enumerate(hw)]
    d = f32(si.filters(cfg, K, m))
    Ws = [si.observation_mask(cfg, i, int(H), int(W)) for i, (H, W) in enumerate(hw)] if with_W else None
    return xs, d, Ws


def to_dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def packed(im, arrays, dtype=torch.float32):
    return to_dev(im.pack(arrays), dtype)
