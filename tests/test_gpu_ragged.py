"""Full-size ragged batch: 256 images with sides uniform in [64, 512], K = 100,
11 x 11 filters, p = 0.1, lambda = 0.5, 30 iterations, in one code-step call
(the launch configuration of the ragged bench workload).  The smallest images
are checked against the oracle one by one; graph replay and BF16 are checked on
the same batch."""

import numpy as np
import pytest
import torch

import oracle
import scsc_inputs as si
from gpu_helpers import f32, rel_err, say

pytestmark = pytest.mark.gpu

CFG, N, K, M_SIDE, P, LAM, T = 4, 256, 100, 11, 0.1, 0.5, 30


@pytest.fixture(scope="module")
def batch():
    from paper_1909_00145_amd.ops import Context, Images

    torch.cuda.set_device(0)
    hw = si.ragged_sizes(CFG, N, 64, 512)
    im = Images(hw)
    xs = [f32(si.field(CFG, n, int(H), int(W))) for n, (H, W) in enumerate(hw)]
    x = torch.from_numpy(im.pack([a.astype(np.float32) for a in xs])).cuda()
    d = f32(si.filters(CFG, K, M_SIDE))
    ctx = Context(0)
    yield ctx, im, xs, x, d
    ctx.close()


def _run(ctx, im, x, d, precision="fp32"):
    z = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")
    st = ctx.code_step(im, x, torch.from_numpy(d.astype(np.float32)).cuda(), z, LAM, P, CFG, 1, T,
                       precision=precision, stats=True)
    return z, st


def test_ragged_full_size_fp32(batch):
    ctx, im, xs, x, d = batch
    say("ragged full size: pixels", im.n_pix)
    z, st = _run(ctx, im, x, d)
    say("  sampled", st.sampled, "nnz", st.nnz)
    assert 0.09 * K * im.n_pix < st.sampled < 0.11 * K * im.n_pix
    got = im.unpack(z.cpu().numpy(), K)
    Lz = oracle.lipschitz_code(d, im.max_side)
    assert abs(st.L_z - Lz) <= 1e-12 * Lz
    order = np.argsort(im.sizes)[:2]
    for n in order:
        H, W = im.hw[n]
        ref, _ = oracle.code_step(xs[n], d, np.zeros((K, H, W)), LAM, P, CFG, 1, T, step=1.0 / Lz, image_index=int(n))
        err = rel_err(got[n], ref)
        say("  image", int(n), (int(H), int(W)), "rel err", err)
        assert err < 1e-5


def test_ragged_graph_and_bf16(batch):
    ctx, im, xs, x, d = batch
    from paper_1909_00145_amd.ops import Context

    say("ragged graph replay")
    z_ref, _ = _run(ctx, im, x, d)
    g = Context(0)
    try:
        g.set_graph(True)
        for _ in range(3):  # tune, capture, replay
            zg, _ = _run(g, im, x, d)
            assert torch.equal(zg, z_ref)
    finally:
        g.close()
    say("ragged bf16")
    zb, _ = _run(ctx, im, x, d, "bf16")
    err = rel_err(zb.cpu().numpy(), z_ref.cpu().numpy())
    say("  bf16 vs fp32 rel err", err)
    assert err < 2e-2
