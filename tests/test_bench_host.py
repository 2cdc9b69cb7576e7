"""Host-side checks of bench.py (no GPU): the module loads with its tables, the
traffic table names sources that exist, and more than one GPU is refused."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_module_tables():
    sys.path.insert(0, ROOT)
    import bench

    assert bench.PAPER_REFERENCE["derived_updates_per_s"] > 0
    for (wl, cls, prec), (src, sha, rd, wr) in bench.TRAFFIC.items():
        assert wl in bench.WORKLOADS and prec in ("bf16", "fp32")
        assert os.path.exists(os.path.join(ROOT, "paper_1909_00145_amd", "csrc", src))
        assert len(sha) == 16 and rd > 0 and wr > 0
    for wl in ("online", "ragged"):
        for prec in ("bf16", "fp32"):
            for cls in ("synth", "adjoint"):
                assert (wl, cls, prec) in bench.TRAFFIC
    for name in ("time_to_objective", "tto_study", "ragged_leg", "unrolled_leg", "cpu_baseline", "rooflines"):
        assert callable(getattr(bench, name))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_lag_pair_count_matches_brute_force():
    """The lag pass's product count, against a loop over every pair of non-zero codes."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch

    import bench

    class Im:
        hw = [(9, 13), (6, 4)]

    K, m = 3, 5
    rng = np.random.default_rng(4)
    parts = [(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.3)).astype(np.float32) for H, W in Im.hw]
    z = torch.from_numpy(np.concatenate([p.ravel() for p in parts]))
    want = 0
    for p in parts:
        nz = list(zip(*np.nonzero(p)))
        for (_, y, x) in nz:
            for (_, y2, x2) in nz:
                dy, dx = y2 - y, x2 - x
                if 0 <= dy <= m - 1 and abs(dx) <= m - 1 and (dy > 0 or dx >= 0):
                    want += 1
    assert bench.lag_pairs(z, Im, K, m) == want
