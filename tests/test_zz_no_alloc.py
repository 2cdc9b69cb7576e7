"""The allocation-free objective (csc_objective_noalloc) against csc_objective and
the FP64 oracle, through the C ABI.

Two calls in a row on the shared scratch array, the second on a smaller batch,
each against csc_objective on the same inputs (the same kernels in the same
order, so the results are bit-identical) and the oracle to 1e-12; the handle's
cached geometry is left alone; a batch beyond the scratch limit is rejected
before any work.
"""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import f32, make_problem, packed, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1909_00145_amd.ops import Context

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return Context(0)


def problem(cfg, hw, K, m, with_W, density=0.05):
    from paper_1909_00145_amd.ops import Images

    xs, d, Ws = make_problem(cfg, hw, K, m, with_W)
    rng = np.random.default_rng(cfg)
    zs = [f32(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < density)) for H, W in hw]
    im = Images(hw)
    dev = (packed(im, xs), to_dev(d), packed(im, zs), packed(im, Ws, torch.uint8) if Ws else None)
    return im, xs, d, zs, Ws, dev


@pytest.mark.parametrize("first,second", [
    (([(40, 33), (16, 50), (70, 9)], 12, 11, 0.7, True), ([(21, 18)], 5, 3, 0.3, False)),
    (([(100, 100)] * 4, 100, 11, 1.0, False), ([(17, 30), (1, 40)], 33, 7, 0.5, True)),
])
def test_two_calls_match_the_allocating_entry_point(ctx, first, second):
    for cfg, (hw, K, m, lam, with_W) in enumerate([first, second], start=11):
        say("objective_noalloc", hw, K, m, with_W)
        im, xs, d, zs, Ws, (xg, dg, zg, Wg) = problem(cfg, hw, K, m, with_W)
        F, data, l1 = ctx.objective(im, xg, dg, zg, lam, W=Wg, noalloc=True)
        Fa, dataa, l1a = ctx.objective(im, xg, dg, zg, lam, W=Wg)
        assert (F, data, l1) == (Fa, dataa, l1a)
        Fr, datar, l1r = oracle.objective(xs, d, zs, lam, Ws)
        assert abs(data - datar) <= 1e-12 * datar
        assert abs(l1 - l1r) <= 1e-12 * l1r
        assert abs(F - Fr) <= 1e-12 * Fr


def test_cached_geometry_is_untouched(ctx):
    say("objective_noalloc between two allocating calls")
    im1, _, _, _, _, (x1, d1, z1, _) = problem(21, [(48, 40), (33, 20)], 8, 5, False)
    im2, _, _, _, _, (x2, d2, z2, _) = problem(22, [(64, 64)], 8, 5, False)
    before = ctx.objective(im1, x1, d1, z1, 0.4)
    other = ctx.objective(im2, x2, d2, z2, 0.4, noalloc=True)
    after = ctx.objective(im1, x1, d1, z1, 0.4)
    assert before == after
    assert other == ctx.objective(im2, x2, d2, z2, 0.4)


def test_batch_beyond_the_scratch_limit_is_rejected(ctx):
    from paper_1909_00145_amd import _lib
    from paper_1909_00145_amd.ops import Images

    # 512 x 512 tiles of 16 x 16: the tile records and the partial sums alone fill
    # the 8 MiB array, so the image and result slots no longer fit
    hw = [(8192, 8192)]
    say("objective_noalloc beyond the limit", hw)
    im = Images(hw)
    x = torch.zeros(im.n_pix, device="cuda")
    z = torch.zeros(im.n_pix, device="cuda")
    d = torch.zeros((1, 3, 3), device="cuda")
    with pytest.raises(_lib.CSCError) as e:
        ctx.objective(im, x, d, z, 0.5, noalloc=True)
    assert e.value.status == _lib.CSC_EINVAL
    assert "limit" in str(e.value)
    # the allocating entry point takes the same batch
    F, _, _ = ctx.objective(im, x, d, z, 0.5)
    assert F == 0.0
