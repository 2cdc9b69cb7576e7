"""Full-size ragged batch: 256 images with sides uniform in [64, 512], K = 100,
11 x 11 filters, p = 0.1, lambda = 0.5, 30 iterations, in one code-step call
(the launch configuration of the ragged bench workload), in FP32 and in BF16.

Images are checked against the oracle one by one: the two smallest, the
largest (500 x 489), the last one packed (its lists end the buffers) and two
of median size, each in FP32 (normwise 1e-5) and in BF16 (2e-2).  Graph replay
is checked on the same batch."""

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
    say("ragged full size: pixels", im.n_pix)
    out = {}
    for prec in ("fp32", "bf16"):
        z, st = _run(ctx, im, x, d, prec)
        say("  ", prec, "sampled", st.sampled, "nnz", st.nnz)
        # keep the checked images only (the whole batch's codes are 8.3 GB)
        imgs = {n: z[K * int(im.offsets[n]) : K * int(im.offsets[n + 1])].cpu().numpy()
                .reshape(K, int(im.hw[n][0]), int(im.hw[n][1])) for n in _picks()}
        out[prec] = (imgs, st)
        del z
    yield ctx, im, xs, x, d, out
    ctx.close()


def _run(ctx, im, x, d, precision="fp32"):
    z = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")
    st = ctx.code_step(im, x, torch.from_numpy(d.astype(np.float32)).cuda(), z, LAM, P, CFG, 1, T,
                       precision=precision, stats=True)
    return z, st


def _picks():
    hw = si.ragged_sizes(CFG, N, 64, 512)
    order = np.argsort(hw[:, 0] * hw[:, 1], kind="stable")
    return [int(order[0]), int(order[1]), int(order[-1]), N - 1, int(order[N // 2]), int(order[N // 2 + 1])]


def test_ragged_full_size_statistics(batch):
    ctx, im, xs, x, d, out = batch
    Lz = oracle.lipschitz_code(d, im.max_side)
    for prec in ("fp32", "bf16"):
        st = out[prec][1]
        assert 0.09 * K * im.n_pix < st.sampled < 0.11 * K * im.n_pix
        assert abs(st.L_z - Lz) <= 1e-12 * Lz


@pytest.mark.parametrize("n", _picks())
def test_ragged_full_size_image_against_oracle(batch, n):
    ctx, im, xs, x, d, out = batch
    H, W = (int(v) for v in im.hw[n])
    say("ragged image", n, (H, W), "against the oracle")
    Lz = oracle.lipschitz_code(d, im.max_side)
    ref, S = oracle.code_step(xs[n], d, np.zeros((K, H, W)), LAM, P, CFG, 1, T, step=1.0 / Lz, image_index=n)
    for prec, tol in (("fp32", 1e-5), ("bf16", 2e-2)):
        got = out[prec][0][n]
        err = rel_err(got, ref)
        say("  ", prec, "rel err", err)
        assert err < tol
        assert not np.any(got[~S]), "codes off the sample must be zero"


def test_ragged_graph_replay(batch):
    ctx, im, xs, x, d, out = batch
    from paper_1909_00145_amd.ops import Context

    say("ragged graph replay")
    z_eager, _ = _run(ctx, im, x, d)
    for n, a in out["fp32"][0].items():  # eager launches repeat the first run bit for bit
        o = K * int(im.offsets[n])
        assert np.array_equal(z_eager[o : o + a.size].cpu().numpy(), a.ravel())
    g = Context(0)
    try:
        g.set_graph(True)
        for _ in range(3):  # tune, capture, replay
            zg, _ = _run(g, im, x, d)
            assert torch.equal(zg, z_eager)
    finally:
        g.close()
