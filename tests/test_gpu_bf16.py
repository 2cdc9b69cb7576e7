"""GPU parity of the BF16 path (matrix-core adjoint with BF16 operands, FP32
accumulation) against the FP64 oracle: exact operand rounding on one
iteration, and the 2e-2 normwise bar on full code steps."""

import numpy as np
import pytest
import torch

import oracle
import scsc_inputs as si
from gpu_helpers import f32, make_problem, packed, rel_err, say, to_dev

pytestmark = pytest.mark.gpu

TOLBF = 2e-2


@pytest.fixture(scope="module")
def ctx():
    from paper_1909_00145_amd.ops import Context

    torch.cuda.set_device(0)
    c = Context(0)
    yield c
    c.close()


def bf16_round(a):
    """Round FP32 values to BF16 (nearest, ties to even), returned as float64."""
    u = np.ascontiguousarray(np.asarray(a, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("hw,K,m", [([(40, 36)], 16, 11), ([(23, 50), (31, 17)], 33, 7), ([(19, 21)], 5, 3),
                                    ([(30, 30)], 20, 9), ([(18, 40)], 48, 5)])
def test_one_iteration_matches_bf16_rounded_operands(ctx, hw, K, m):
    """lambda = 0, one iteration from zero codes: z = eta D^T x on S with d and x rounded to BF16."""
    from paper_1909_00145_amd.ops import Images

    say("bf16 one iteration", hw, K, m)
    xs, d, _ = make_problem(6, hw, K, m)
    im = Images(hw)
    z = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")
    eta = 0.37
    ctx.code_step(im, packed(im, xs), to_dev(d), z, 0.0, 0.4, 3, 1, 1, step=eta, precision="bf16")
    got = z.cpu().numpy()
    db = bf16_round(d)
    refs = []
    for i, x in enumerate(xs):
        S = oracle.bernoulli_mask(K, x.shape[0], x.shape[1], 0.4, 3, 1, i)
        refs.append(np.where(S, eta * oracle.adjoint(db, bf16_round(x)), 0.0))
    err = rel_err(got, im.pack(refs))
    say("  rel err", err)
    assert err < 1e-5


def _code_step(ctx, hw, K, m, lam, p, n_iter, with_W=False, cfg=1):
    from paper_1909_00145_amd.ops import Images

    xs, d, Ws = make_problem(cfg, hw, K, m, with_W)
    im = Images(hw)
    out = {}
    for prec in ("fp32", "bf16"):
        z = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")
        out[prec] = ctx.code_step(im, packed(im, xs), to_dev(d), z, lam, p, 1, 1, n_iter,
                                  W=packed(im, Ws, torch.uint8) if Ws else None, precision=prec, stats=True), z
    Lz = oracle.lipschitz_code(d, im.max_side)
    refs = [oracle.code_step(x, d, np.zeros((K,) + x.shape), lam, p, 1, 1, n_iter, step=1.0 / Lz,
                             W=None if Ws is None else Ws[i], image_index=i)[0] for i, x in enumerate(xs)]
    return im, out, refs


@pytest.mark.parametrize("hw,K,m,lam,p,n_iter,with_W", [
    ([(64, 64)], 16, 11, 1.0, 0.1, 20, False),
    ([(37, 45), (16, 9), (50, 3)], 10, 5, 0.5, 0.3, 15, False),
    ([(40, 33), (27, 60)], 33, 11, 0.2, 0.5, 10, True),
])
def test_code_step_bf16_parity(ctx, hw, K, m, lam, p, n_iter, with_W):
    say("bf16 code step", hw, K, m)
    im, out, refs = _code_step(ctx, hw, K, m, lam, p, n_iter, with_W)
    (st32, z32), (stbf, zbf) = out["fp32"], out["bf16"]
    assert stbf.sampled == st32.sampled
    err = rel_err(zbf.cpu().numpy(), im.pack(refs))
    err32 = rel_err(zbf.cpu().numpy(), z32.cpu().numpy())
    say("  rel err vs oracle", err, "vs fp32", err32, "nnz", stbf.nnz, st32.nnz)
    assert err < TOLBF
    assert err32 < TOLBF


def test_code_step_bf16_full_size(ctx):
    """20 images 100 x 100, K = 100, p = 0.1, lambda = 1, 20 iterations; images 0 and 13 against the oracle."""
    from paper_1909_00145_amd.ops import Images

    say("bf16 full size")
    N, H, W, K, m = 20, 100, 100, 100, 11
    import scsc_inputs as si

    xs = [f32(a) for a in si.stream_batch(3, 1, N, H, W)]
    d = f32(si.filters(3, K, m))
    im = Images.uniform(N, H, W)
    z = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")
    ctx.code_step(im, packed(im, xs), to_dev(d), z, 1.0, 0.1, 3, 1, 20, precision="bf16")
    got = im.unpack(z.cpu().numpy(), K)
    Lz = oracle.lipschitz_code(d, 100)
    for i in (0, 13):
        ref, _ = oracle.code_step(xs[i], d, np.zeros((K, H, W)), 1.0, 0.1, 3, 1, 20, step=1.0 / Lz, image_index=i)
        err = rel_err(got[i], ref)
        say("  image", i, "rel err", err)
        assert err < TOLBF


@pytest.mark.parametrize("hw,K,m", [([(40, 36)], 16, 11), ([(23, 50), (31, 17)], 33, 7), ([(19, 21)], 5, 3),
                                    ([(30, 30), (7, 70)], 150, 5), ([(18, 40)], 20, 9)])
def test_filter_corr_bf16_rounded_operands(ctx, hw, K, m):
    """Z^T r on the matrix cores equals the FP64 correlation of BF16-rounded z and r."""
    from paper_1909_00145_amd.ops import Images

    say("bf16 filter corr", hw, K, m)
    rng = np.random.default_rng(K * m)
    im = Images(hw)
    zs = [f32(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.1)) for H, W in hw]
    rs = [f32(rng.standard_normal((H, W))) for H, W in hw]
    G = ctx.filter_corr(im, packed(im, zs), packed(im, rs), K, m, precision="bf16").cpu().numpy()
    ref = sum(oracle.filter_corr(bf16_round(z), bf16_round(r), m) for z, r in zip(zs, rs)).ravel()
    err = rel_err(G, ref)
    say("  rel err", err)
    assert err < 1e-5


@pytest.mark.parametrize("hw,K,m,with_W", [([(48, 40)], 16, 11, False), ([(24, 20), (16, 21)], 12, 7, True)])
def test_dict_step_batch_bf16(ctx, hw, K, m, with_W):
    from paper_1909_00145_amd.ops import Images

    say("bf16 batch dict step", hw, K, m, with_W)
    xs, d, Ws = make_problem(2, hw, K, m, with_W)
    rng = np.random.default_rng(5)
    zs = [f32(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.05)) for H, W in hw]
    im = Images(hw)
    dg = to_dev(d)
    Ld = ctx.dict_step(im, packed(im, xs), packed(im, zs), dg, W=packed(im, Ws, torch.uint8) if Ws else None,
                       precision="bf16")
    dr, Ldr = oracle.dict_step_batch(xs, Ws, zs, d)
    say("  L_d", Ld, Ldr, "d err", rel_err(dg.cpu().numpy(), dr))
    assert abs(Ld - Ldr) <= TOLBF * Ldr
    assert rel_err(dg.cpu().numpy(), dr) < TOLBF


# density 0.6 with K = 40 puts more code entries in a tile's region than the
# kernel stages in LDS, so those tiles read the lists from memory per chunk
@pytest.mark.parametrize("hw,K,m,density", [([(40, 36)], 16, 11, 0.1), ([(23, 50), (31, 17)], 33, 7, 0.1),
                                            ([(19, 21)], 5, 3, 0.1), ([(30, 30), (7, 70)], 70, 5, 0.1),
                                            ([(18, 40)], 20, 9, 0.1), ([(40, 36)], 40, 11, 0.6)])
def test_synthesis_bf16_rounded_operands(ctx, hw, K, m, density):
    """D z on the matrix cores equals the FP64 synthesis of BF16-rounded d and z."""
    from paper_1909_00145_amd.ops import Images

    say("bf16 synthesis", hw, K, m, density)
    rng = np.random.default_rng(K + 3 * m)
    im = Images(hw)
    d = f32(rng.standard_normal((K, m, m)))
    zs = [f32(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < density)) for H, W in hw]
    y = ctx.synthesize(im, to_dev(d), packed(im, zs), precision="bf16").cpu().numpy()
    ref = im.pack([oracle.synthesize(bf16_round(d), bf16_round(z)) for z in zs])
    err = rel_err(y, ref)
    say("  rel err", err)
    assert err < 1e-5


def test_synthesis_bf16_variants_bit_identical(ctx):
    """The three LDS chunk sizes of the BF16 synthesis give the same bits (synthesis and a code
    step); the code steps run both variants of the adjoint (the forced variant's low bit)."""
    from paper_1909_00145_amd.ops import Images

    say("bf16 synthesis variants")
    hw = [(70, 45), (33, 100)]
    K, m = 44, 11
    rng = np.random.default_rng(12)
    im = Images(hw)
    d = to_dev(f32(rng.standard_normal((K, m, m))))
    z = packed(im, [f32(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.05)) for H, W in hw])
    xs = [f32(si.field(4, i, H, W)) for i, (H, W) in enumerate(hw)]
    outs, codes = [], []
    try:
        for v in range(3):
            ctx.set_autotune(True, variant=v)
            outs.append(ctx.synthesize(im, d, z, precision="bf16").cpu().numpy())
            zz = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")
            ctx.code_step(im, packed(im, xs), d, zz, 0.5, 0.3, 7, 1, 10, precision="bf16")
            codes.append(zz.cpu().numpy())
    finally:
        ctx.set_autotune(True)
    for o, cd in zip(outs[1:], codes[1:]):
        np.testing.assert_array_equal(o, outs[0])
        np.testing.assert_array_equal(cd, codes[0])


@pytest.mark.parametrize("hw,K,m", [([(40, 36)], 16, 11), ([(23, 50), (31, 17)], 33, 7), ([(32, 32)] * 2, 256, 11),
                                    ([(19, 21)], 5, 3)])
def test_dense_adjoint_matches_bf16_rounded_operands(ctx, hw, K, m):
    """csc_adjoint with BF16 operands: every coordinate equals D^T r of the BF16-rounded d and r
    (FP32 accumulation of exact products)."""
    from paper_1909_00145_amd.ops import Images

    say("bf16 dense adjoint", hw, K, m)
    xs, d, _ = make_problem(8, hw, K, m)
    im = Images(hw)
    g = ctx.adjoint(im, to_dev(d), packed(im, xs), precision="bf16").cpu().numpy()
    ref = im.pack([oracle.adjoint(bf16_round(d), bf16_round(x)) for x in xs])
    err = rel_err(g, ref)
    say("  rel err", err)
    assert err < 1e-5
