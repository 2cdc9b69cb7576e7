"""GPU parity of inpainting (reconstruction from observed pixels, Sec. 4) against
the FP64 oracle: the reconstruction to 1e-5 (FP32) and 2e-2 (BF16) normwise,
the PSNR to 1e-3 dB, and the unobserved pixels never read (same bits when they
change)."""

import numpy as np
import pytest
import torch

import oracle
import scsc_inputs as si
from tests.gpu_helpers import f32, packed, rel_err, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1909_00145_amd.ops import Context

    torch.cuda.set_device(0)
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("hw,K,m,precision,tol", [([(40, 36), (23, 50)], 8, 5, "fp32", 1e-5),
                                                  ([(48, 40)], 16, 11, "fp32", 1e-5),
                                                  ([(48, 40)], 16, 11, "bf16", 2e-2)])
def test_inpaint_matches_oracle(ctx, hw, K, m, precision, tol):
    from paper_1909_00145_amd.drivers import inpaint, psnr
    from paper_1909_00145_amd.ops import Images

    say("inpaint", hw, K, m, precision)
    im = Images(hw)
    xs = [f32(si.field(7, i, H, W)) for i, (H, W) in enumerate(hw)]
    Ws = [si.observation_mask(41, i, H, W, 0.5) for i, (H, W) in enumerate(hw)]
    d = f32(oracle.project_ball(si.filters(7, K, m)))
    x = packed(im, xs)
    Wg = packed(im, Ws, torch.uint8)
    xh, _ = inpaint(ctx, im, x, Wg, to_dev(d), 0.4, 30, precision=precision)
    got = im.unpack(xh.cpu().numpy(), 1)
    Lz = oracle.lipschitz_code(d, im.max_side)
    refs = [oracle.inpaint(xi, Wi, d, 0.4, 30, step=1.0 / Lz)[0] for xi, Wi in zip(xs, Ws)]
    err = rel_err(np.concatenate([g.ravel() for g in got]), np.concatenate([r.ravel() for r in refs]))
    p_gpu = psnr(im, xh, x)
    p_ref = [oracle.psnr(r, xi) for r, xi in zip(refs, xs)]
    say("  rel err", err, "psnr", p_gpu, p_ref)
    assert err < tol
    if precision == "fp32":
        np.testing.assert_allclose(p_gpu, p_ref, rtol=0, atol=1e-3)
    # the unobserved pixels are not used
    x2 = packed(im, [np.where(Wi != 0, xi, 1e6) for xi, Wi in zip(xs, Ws)])
    xh2, _ = inpaint(ctx, im, x2, Wg, to_dev(d), 0.4, 30, precision=precision)
    np.testing.assert_array_equal(xh2.cpu().numpy(), xh.cpu().numpy())
