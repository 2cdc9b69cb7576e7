"""Graph replay of the code step's proximal-gradient iterations: every replay
gives the same bits as the eager launches, across new inputs, filters and step
sizes of the same shape, with eager work between the replays."""

import numpy as np
import pytest
import torch

import scsc_inputs as si
from gpu_helpers import f32, packed, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("hw,K,m,precision,with_W", [
    ([(64, 64)], 16, 11, "fp32", False),
    ([(37, 45), (16, 9), (50, 33)], 24, 7, "fp32", True),
    ([(40, 40), (23, 31)], 20, 11, "bf16", False),
])
def test_graph_replay_matches_eager(hw, K, m, precision, with_W):
    from paper_1909_00145_amd.ops import Context, Images

    say("graph replay", hw, K, m, precision, with_W)
    torch.cuda.set_device(0)
    eager, graph = Context(0), Context(0)
    graph.set_graph(True)
    im = Images(hw)
    W = packed(im, [si.observation_mask(8, i, H, Wd) for i, (H, Wd) in enumerate(hw)], torch.uint8) if with_W else None
    try:
        for call in range(5):
            xs = [f32(si.field(8, 10 * call + i, H, Wd)) for i, (H, Wd) in enumerate(hw)]
            d = f32(si.filters(8 + call, K, m))
            x = packed(im, xs)
            outs = []
            for ctx in (eager, graph):
                z = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")
                st = ctx.code_step(im, x, to_dev(d), z, 0.5, 0.3, 5, call + 1, 12, W=W, precision=precision,
                                   stats=True)
                outs.append((z.cpu().numpy(), st))
                # unrelated eager work on the same stream between replays
                ctx.synthesize(im, to_dev(d), z)
            np.testing.assert_array_equal(outs[1][0], outs[0][0])
            assert outs[1][1].nnz == outs[0][1].nnz and outs[1][1].nnz_iter_sum == outs[0][1].nnz_iter_sum
    finally:
        eager.close()
        graph.close()


def test_power_iteration_graph_matches_eager():
    """The lag-sum power iteration replayed from a graph gives the same L_d and filters as eager launches."""
    from paper_1909_00145_amd.ops import Context, Images

    say("power iteration graph replay")
    torch.cuda.set_device(0)
    hw = [(40, 36), (23, 50)]
    K, m = 12, 7
    eager, graph = Context(0), Context(0)
    graph.set_graph(True)
    im = Images(hw)
    try:
        for call in range(4):
            rng = np.random.default_rng(30 + call)
            xs = [f32(si.field(9, 10 * call + i, H, Wd)) for i, (H, Wd) in enumerate(hw)]
            zs = [f32(rng.standard_normal((K, H, Wd)) * (rng.random((K, H, Wd)) < 0.05)) for H, Wd in hw]
            d0 = f32(si.filters(9 + call, K, m))
            outs = []
            for ctx in (eager, graph):
                d = to_dev(d0)
                Ld = ctx.dict_step(im, packed(im, xs), packed(im, zs), d)
                outs.append((Ld, d.cpu().numpy()))
                # unrelated eager work on the same stream between replays
                ctx.synthesize(im, d, packed(im, zs))
            assert outs[1][0] == outs[0][0]
            np.testing.assert_array_equal(outs[1][1], outs[0][1])
    finally:
        eager.close()
        graph.close()
