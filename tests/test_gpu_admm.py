"""GPU parity of the ADMM code solver (csc_code_step_admm, Sec. 3.2) against the
FP64 oracle (code_step_admm).  FP32 vectors with FP64 CG dot products and
per-image CG scalars: 1e-5 normwise after the paper's 10 iterations (measured
below 1e-6), the selection count exactly, zero off S, and the argument checks."""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import f32, make_problem, packed, rel_err, say, to_dev

pytestmark = pytest.mark.gpu

TOLADMM = 1e-5


@pytest.fixture(scope="module")
def ctx():
    from paper_1909_00145_amd.ops import Context

    torch.cuda.set_device(0)
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("hw,K,m,lam,p,n_admm,n_cg,with_W,warm", [
    ([(40, 36)], 16, 11, 1.0, 0.1, 10, 5, False, False),
    ([(37, 53), (20, 17)], 10, 5, 0.3, 0.5, 10, 5, False, True),
    ([(45, 30)], 12, 7, 0.5, 0.3, 6, 3, True, False),
    ([(1, 40), (29, 1)], 4, 3, 0.2, 1.0, 4, 2, False, False),
])
def test_admm_matches_oracle(ctx, hw, K, m, lam, p, n_admm, n_cg, with_W, warm):
    from paper_1909_00145_amd.ops import Images

    say("admm", hw, K, m, p, n_admm, n_cg)
    xs, d, Ws = make_problem(9, hw, K, m, with_W)
    im = Images(hw, 2)
    rng = np.random.default_rng(3)
    z0 = [f32(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.2)) if warm else np.zeros((K, H, W))
          for H, W in hw]
    z = packed(im, z0)
    st = ctx.code_step_admm(im, packed(im, xs), to_dev(d), z, lam, p, 17, 3, n_admm, n_cg,
                            W=packed(im, Ws, torch.uint8) if Ws else None, stats=True)
    got = im.unpack(z.cpu().numpy(), K)
    refs, Ss = [], []
    for i, x in enumerate(xs):
        zr, S = oracle.code_step_admm(x, d, z0[i], lam, p, 17, 3, n_admm, n_cg, W=None if Ws is None else Ws[i],
                                      image_index=2 + i)
        refs.append(zr)
        Ss.append(S)
    err = rel_err(np.concatenate([g.ravel() for g in got]), np.concatenate([r.ravel() for r in refs]))
    say("  rel err", err, "nnz", st.nnz, "sampled", st.sampled)
    assert err < TOLADMM
    assert st.sampled == sum(int(S.sum()) for S in Ss)
    for g, S in zip(got, Ss):
        assert np.all(g[~S] == 0)
    assert st.nnz == sum(int(np.count_nonzero(g)) for g in got)


def test_admm_rejects_bad_arguments(ctx):
    from paper_1909_00145_amd import CSCError
    from paper_1909_00145_amd.ops import Images

    im = Images([(8, 8)])
    x = torch.zeros(64, device="cuda")
    d = torch.zeros(2 * 9, device="cuda").reshape(2, 3, 3)
    z = torch.zeros(2 * 64, device="cuda")
    with pytest.raises(CSCError):
        ctx.code_step_admm(im, x, d, z, 0.0, 0.5, 1, 1, 2, 2)  # lambda 0 and no rho
    with pytest.raises(CSCError):
        ctx.code_step_admm(im, x, d, z, 0.1, 0.5, 1, 1, 2, 2, alpha=2.0)
    with pytest.raises(CSCError):
        ctx.code_step_admm(im, x, d, z, 0.1, 0.5, 1, 1, -1, 2)
