"""The code step with eager launches runs three parts of a batch (two for two
images; split between images) on the handle's stream and its side streams, with
its synthesis and adjoint variants tuned on the first calls (FP32 and BF16).  Every call gives the
same bits as the same step run in order on one stream, which the library does
while per-kernel timing is on."""

import numpy as np
import pytest
import torch

import scsc_inputs as si
from gpu_helpers import f32, packed, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
@pytest.mark.parametrize("hw", [[(48, 40), (33, 57), (20, 20)], [(64, 64), (64, 64)]])
def test_split_code_step_matches_one_stream(hw, precision):
    from paper_1909_00145_amd.ops import Context, Images

    say("split code step", hw, precision)
    torch.cuda.set_device(0)
    K, m = 24, 11
    split, single = Context(0), Context(0)
    single.lib.csc_profile_enable(single.h, 1)
    im = Images(hw)
    try:
        for call in range(5):
            xs = [f32(si.field(12, 10 * call + i, H, Wd)) for i, (H, Wd) in enumerate(hw)]
            d = f32(si.filters(12 + call, K, m))
            x = packed(im, xs)
            outs = []
            for ctx in (split, single):
                z = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")
                st = ctx.code_step(im, x, to_dev(d), z, 0.5, 0.3, 5, call + 1, 12, precision=precision, stats=True)
                outs.append((z.cpu().numpy(), st))
            np.testing.assert_array_equal(outs[0][0], outs[1][0])
            assert outs[0][1] == outs[1][1]
            assert outs[0][1].nnz > 0
    finally:
        split.close()
        single.close()
