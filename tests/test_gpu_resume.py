"""Checkpoint/resume of the online learner and the workspace limit, through the C ABI.

Resume: an online learner that runs 5 mini-batches straight ends where one that is
saved after 3 mini-batches (filters, C_bar, B_bar, t, sum of L_d written with
torch.save and read back with weights_only=True) and resumed in a fresh learner
ends after the same 2 further mini-batches.  The lag and corner sums of C_bar add
in a nondeterministic order (FP64 atomics), so the surrogates are compared to
1e-12 and the filters to 1e-6; the count t and the sampler draws continue exactly.

Workspace limit: a handle created with SCSC_WORKSPACE_LIMIT set reports
CSC_ENOMEM (with the limit in its message) when a call needs more device
workspace, and other handles are unaffected.
"""

import io
import os

import numpy as np
import pytest
import torch

import scsc_inputs as si
from tests.gpu_helpers import rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1909_00145_amd.ops import Context

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return Context(0)


def _stream(t, N, H, W):
    return torch.from_numpy(si.stream_batch(8, t, N, H, W).astype(np.float32).reshape(-1)).cuda()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_online_learner_resumes_from_a_checkpoint(ctx, precision):
    from paper_1909_00145_amd.drivers import OnlineLearner
    from paper_1909_00145_amd.ops import Images

    N, H, W, K, m = 4, 48, 40, 16, 11
    say("resume", precision)
    im = Images.uniform(N, H, W)
    d0 = torch.from_numpy(si.filters(8, K, m).astype(np.float32)).cuda()

    straight = OnlineLearner(ctx, im, d0.clone(), 0.5, 0.3, n_code_iter=10, precision=precision)
    for t in range(1, 6):
        straight.step(_stream(t, N, H, W))

    first = OnlineLearner(ctx, im, d0.clone(), 0.5, 0.3, n_code_iter=10, precision=precision)
    for t in range(1, 4):
        first.step(_stream(t, N, H, W))
    buf = io.BytesIO()
    torch.save(first.state_dict(), buf)
    buf.seek(0)
    saved = torch.load(buf, weights_only=True)
    resumed = OnlineLearner(ctx, im, torch.zeros_like(d0), 0.5, 0.3, n_code_iter=10, precision=precision)
    resumed.load_state_dict(saved)
    assert resumed.t == 3
    for t in range(4, 6):
        resumed.step(_stream(t, N, H, W))

    assert resumed.t == straight.t == 5
    assert abs(resumed.sur.Ld_sum - straight.sur.Ld_sum) <= 1e-12 * straight.sur.Ld_sum
    assert rel_err(resumed.sur.C.cpu().numpy(), straight.sur.C.cpu().numpy()) < 1e-12
    assert rel_err(resumed.sur.B.cpu().numpy(), straight.sur.B.cpu().numpy()) < 1e-12
    err = rel_err(resumed.d.cpu().numpy(), straight.d.cpu().numpy())
    say("  filters rel diff", err)
    assert err < 1e-6


def test_workspace_limit_reports_enomem(ctx):
    from paper_1909_00145_amd import _lib
    from paper_1909_00145_amd.ops import Context, Images

    hw = [(64, 64), (40, 30)]
    K, m = 16, 11
    im = Images(hw)
    x = torch.from_numpy(im.pack([si.field(9, i, H, W).astype(np.float32) for i, (H, W) in enumerate(hw)])).cuda()
    d = torch.from_numpy(si.filters(9, K, m).astype(np.float32)).cuda()
    os.environ["SCSC_WORKSPACE_LIMIT"] = "65536"
    try:
        small = Context(0)
    finally:
        del os.environ["SCSC_WORKSPACE_LIMIT"]
    say("workspace limit")
    z = torch.zeros(K * im.n_pix, device="cuda")
    with pytest.raises(_lib.CSCError) as e:
        small.code_step(im, x, d, z, 0.5, 0.3, 1, 1, 5)
    assert e.value.status == _lib.CSC_ENOMEM
    assert "limit" in str(e.value)
    small.close()
    # the unrestricted handle runs the same step
    z2 = torch.zeros(K * im.n_pix, device="cuda")
    st = ctx.code_step(im, x, d, z2, 0.5, 0.3, 1, 1, 5, stats=True)
    assert st.sampled > 0 and st.nnz > 0
