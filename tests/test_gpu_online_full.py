"""The online filter step (eqs. (8)-(9)) at the full mini-batch size of the
online workload: 20 images 100x100, K = 100 filters 11x11, codes at the
density a code step leaves there (3.7 % non-zero), in the launch
configuration the bench times (filter-major lag pass over several filter
chunks and row ranges, expansion of every stored block, corner corrections).

The oracle's dense surrogate would hold (K m^2)^2 doubles, so C_bar is checked
on sampled entries, each the batch sum over pixels p of z_k[p - s] z_k2[p - s2]
(the product of columns (k, s) and (k2, s2) of Z in eq. (5), codes zero off the
image), located through csc_surrogate_index; B_bar is checked in full.  L_d and
the filter update are checked on a two-image slice of the batch in the same
launch shapes per image (the oracle's power iteration costs seconds per
image), with C_bar d formed matrix-free from oracle primitives.
"""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import f32, make_problem, packed, rel_err, say, to_dev

pytestmark = pytest.mark.gpu

N, H, W, K, m = 20, 100, 100, 100, 11
DENSITY = 0.037


@pytest.fixture(scope="module")
def ctx():
    from paper_1909_00145_amd.ops import Context

    torch.cuda.set_device(0)
    c = Context(0)
    yield c
    c.close()


def codes(n, seed):
    rng = np.random.default_rng(seed)
    return [f32(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < DENSITY)) for _ in range(n)]


def oracle_entry(zps, c, k, s, k2, s2):
    """sum over the batch of sum_p z_k[p - s] z_k2[p - s2], codes padded by c."""
    (sy, sx), (sy2, sx2) = s, s2
    tot = 0.0
    for zp in zps:
        a = zp[k, c - sy : c - sy + H, c - sx : c - sx + W]
        b = zp[k2, c - sy2 : c - sy2 + H, c - sx2 : c - sx2 + W]
        tot += float(np.sum(a * b))
    return tot


def test_online_step_full_batch_surrogates(ctx):
    from paper_1909_00145_amd import _lib
    from paper_1909_00145_amd.ops import Images, Surrogate

    say("online full batch: surrogates", N, H, W, K, m)
    hw = [(H, W)] * N
    im = Images(hw)
    xs, d, _ = make_problem(3, hw, K, m)
    d = f32(oracle.project_ball(d))
    zs = codes(N, 41)
    sur = Surrogate(K, m)
    dg = to_dev(d)
    ctx.dict_step(im, packed(im, xs), packed(im, zs), dg, surrogate=sur)
    assert sur.t == 1
    # B_bar in full
    Bsum = sum(oracle.filter_corr(z, x, m) for z, x in zip(zs, xs))
    say("  B rel err", rel_err(sur.B.cpu().numpy(), Bsum.ravel()))
    assert rel_err(sur.B.cpu().numpy(), Bsum.ravel()) < 1e-12
    # C_bar on sampled entries: random ones, and ones with both taps on the
    # window border (the entries the band and corner terms correct)
    c = m // 2
    zps = [oracle.pad_codes(z, c) for z in zs]
    rng = np.random.default_rng(7)
    lib = _lib.lib()
    picks = []
    for i in range(240):
        k, k2 = (int(v) for v in rng.integers(0, K, 2))
        if i % 2:
            s = tuple(int(v) for v in rng.integers(-c, c + 1, 2))
            s2 = tuple(int(v) for v in rng.integers(-c, c + 1, 2))
        else:
            edge = [-c, c]
            s = (edge[int(rng.integers(2))], int(rng.integers(-c, c + 1)))
            s2 = (int(rng.integers(-c, c + 1)), edge[int(rng.integers(2))])
        picks.append((k, s, k2, s2))
    idx = [lib.csc_surrogate_index(K, m, k, s[0], s[1], k2, s2[0], s2[1]) for k, s, k2, s2 in picks]
    assert min(idx) >= 0
    got = sur.C[torch.tensor(idx, dtype=torch.int64, device=sur.C.device)].cpu().numpy()
    ref = np.array([oracle_entry(zps, c, k, s, k2, s2) for k, s, k2, s2 in picks])
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    say("  C sampled max err / max |entry|", err, "max |entry|", scale)
    assert err < 1e-12


def test_online_step_full_size_filter_update(ctx):
    from paper_1909_00145_amd.ops import Images, Surrogate

    n = 2
    say("online full size: filter update on", n, "images", H, W, K, m)
    hw = [(H, W)] * n
    im = Images(hw)
    xs, d, _ = make_problem(3, hw, K, m)
    d = f32(oracle.project_ball(d))
    zs = codes(n, 43)
    sur = Surrogate(K, m)
    dg = to_dev(d)
    ctx.dict_step(im, packed(im, xs), packed(im, zs), dg, surrogate=sur)
    Ld = oracle.lipschitz_filter(zs, None, K, m)
    Bsum = sum(oracle.filter_corr(z, x, m) for z, x in zip(zs, xs))
    Cd = sum(oracle.filter_corr(z, oracle.synthesize(d, z), m) for z in zs)
    dr = oracle.project_ball(d - (Cd - Bsum) / Ld)
    say("  Ld", sur.Ld_sum, Ld, "d rel err", rel_err(dg.cpu().numpy(), dr))
    assert abs(sur.Ld_sum - Ld) <= 1e-5 * Ld
    assert rel_err(dg.cpu().numpy(), dr) < 1e-5
