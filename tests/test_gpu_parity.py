"""Parity of the HIP path against the FP64 oracle, through the C ABI.

Bars: selections bit-exact; FP64 reductions (objective, L_z, surrogates) to
1e-12 relative; FP32 operators and steps to 1e-5 relative in the normwise
metric ||gpu - oracle|| / ||oracle||.  Sizes span several 16 x 16 tiles with
ragged tails; edge cases cover n_iter = 0, p = 1, a zero solution, a single
image of one pixel row and K not a multiple of 4 or 32.
"""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import f32, make_problem, packed, rel_err, say, to_dev

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def ctx():
    from paper_1909_00145_amd.ops import Context

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return Context(0)


def Images(hw, base=0):
    from paper_1909_00145_amd.ops import Images as _I

    return _I(hw, base)


# ---------------------------------------------------------------------------
# selection (eq. 2): bit-exact
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("K,hw,p,seed,draw,base", [
    (16, [(64, 64)], 0.1, 1, 1, 0),
    (100, [(37, 53), (20, 17)], 0.5, 2**40 + 7, 9, 3),
    (33, [(1, 70), (19, 1)], 0.05, 5, 2, 0),
    (7, [(16, 16)], 1.0, 0, 0, 0),
])
def test_mask_bit_exact(ctx, K, hw, p, seed, draw, base):
    say("mask", K, hw, p)
    im = Images(hw, base)
    got = ctx.mask(im, K, p, seed, draw).cpu().numpy()
    ref = im.pack([oracle.bernoulli_mask(K, H, W, p, seed, draw, base + i) for i, (H, W) in enumerate(hw)])
    np.testing.assert_array_equal(got, ref.astype(np.uint8))


# ---------------------------------------------------------------------------
# step size and operators
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("K,m,side", [(16, 11, 64), (100, 11, 100), (5, 3, 37), (9, 7, 200)])
def test_lipschitz_code(ctx, K, m, side):
    d = f32(np.random.default_rng(K).standard_normal((K, m, m)))
    got = ctx.lipschitz_code(to_dev(d), side)
    ref = oracle.lipschitz_code(d, side)
    assert abs(got - ref) <= 1e-12 * ref


@pytest.mark.parametrize("K,m,hw", [(16, 11, [(64, 64)]), (5, 5, [(37, 45), (16, 9)]), (3, 3, [(1, 20)])])
def test_operators(ctx, K, m, hw):
    say("operators", K, m, hw)
    rng = np.random.default_rng(K + m)
    im = Images(hw)
    d = f32(rng.standard_normal((K, m, m)))
    zs = [f32(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.2)) for H, W in hw]
    rs = [f32(rng.standard_normal((H, W))) for H, W in hw]
    y = ctx.synthesize(im, to_dev(d), packed(im, zs)).cpu().numpy()
    assert rel_err(y, im.pack([oracle.synthesize(d, z) for z in zs])) < TOL32
    g = ctx.adjoint(im, to_dev(d), packed(im, rs)).cpu().numpy()
    assert rel_err(g, im.pack([oracle.adjoint(d, r) for r in rs])) < TOL32
    G = ctx.filter_corr(im, packed(im, zs), packed(im, rs), K, m).cpu().numpy()
    assert rel_err(G, sum(oracle.filter_corr(z, r, m) for z, r in zip(zs, rs)).ravel()) < TOL32


def test_launch_variants_bit_identical(ctx):
    """Every launch variant of the tuned kernels gives the same bits (synthesis and a code step)."""
    say("launch variants")
    hw = [(70, 45), (33, 100)]
    K, m = 24, 11
    rng = np.random.default_rng(11)
    im = Images(hw)
    d = to_dev(f32(rng.standard_normal((K, m, m))))
    z = packed(im, [f32(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.05)) for H, W in hw])
    xs, _, _ = make_problem(5, hw, K, m)
    outs, codes = [], []
    try:
        for v in range(4):
            ctx.set_autotune(True, variant=v)
            outs.append(ctx.synthesize(im, d, z).cpu().numpy())
            zz = torch.zeros(K * im.n_pix, dtype=torch.float32, device="cuda")
            ctx.code_step(im, packed(im, xs), d, zz, 0.5, 0.3, 7, 1, 10)
            codes.append(zz.cpu().numpy())
        ctx.set_autotune(True)
        outs.append(ctx.synthesize(im, d, z).cpu().numpy())
    finally:
        ctx.set_autotune(True)
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    for c in codes[1:]:
        np.testing.assert_array_equal(c, codes[0])


# ---------------------------------------------------------------------------
# objective (eq. 1), FP64 on both sides
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("with_W", [False, True])
def test_objective(ctx, with_W):
    hw = [(40, 33), (16, 50)]
    K, m, lam = 12, 11, 0.7
    xs, d, Ws = make_problem(1, hw, K, m, with_W)
    rng = np.random.default_rng(3)
    zs = [f32(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.05)) for H, W in hw]
    im = Images(hw)
    F, data, l1 = ctx.objective(im, packed(im, xs), to_dev(d), packed(im, zs), lam,
                                W=packed(im, Ws, torch.uint8) if Ws else None)
    Fr, datar, l1r = oracle.objective(xs, d, zs, lam, Ws)
    assert abs(data - datar) <= 1e-12 * datar
    assert abs(l1 - l1r) <= 1e-12 * l1r
    assert abs(F - Fr) <= 1e-12 * Fr


# ---------------------------------------------------------------------------
# code step (eqs. 2-4)
# ---------------------------------------------------------------------------
def run_code_step(ctx, hw, K, m, lam, p, seed, draw, n_iter, with_W=False, z0=None, base=0, cfg=1):
    xs, d, Ws = make_problem(cfg, hw, K, m, with_W)
    im = Images(hw, base)
    if z0 is None:
        z0 = [np.zeros((K, H, W)) for H, W in hw]
    z = packed(im, z0)
    stats = ctx.code_step(im, packed(im, xs), to_dev(d), z, lam, p, seed, draw, n_iter,
                          W=packed(im, Ws, torch.uint8) if Ws else None, stats=True)
    got = im.unpack(z.cpu().numpy(), K)
    refs = []
    Lz = oracle.lipschitz_code(d, im.max_side)
    for i, x in enumerate(xs):
        zr, S = oracle.code_step(x, d, z0[i], lam, p, seed, draw, n_iter, step=1.0 / Lz,
                                 W=None if Ws is None else Ws[i], image_index=base + i)
        refs.append(zr)
    return got, refs, stats, Lz


def test_code_step_small_config(ctx):
    """64 x 64 image, K = 16, p = 0.1, lambda = 1, 20 iterations from zero codes."""
    say("code_step C1")
    got, refs, st, Lz = run_code_step(ctx, [(64, 64)], 16, 11, 1.0, 0.1, 1, 1, 20)
    err = rel_err(np.concatenate([g.ravel() for g in got]), np.concatenate([r.ravel() for r in refs]))
    say("  rel err", err, "nnz", st.nnz, "sampled", st.sampled)
    assert err < TOL32
    assert abs(st.L_z - Lz) <= 1e-12 * Lz
    assert st.nnz == sum(int(np.count_nonzero(r)) for r in refs)


@pytest.mark.parametrize("hw,K,m,lam,p,n_iter,with_W", [
    ([(37, 53), (20, 17)], 10, 5, 0.3, 0.5, 15, False),
    ([(45, 30)], 33, 11, 0.5, 0.2, 10, True),
    ([(1, 40), (29, 1)], 4, 3, 0.2, 1.0, 8, False),
    ([(50, 50)], 8, 7, 0.4, 1.0, 12, False),
])
def test_code_step_ragged(ctx, hw, K, m, lam, p, n_iter, with_W):
    say("code_step", hw, K, m, p)
    got, refs, st, _ = run_code_step(ctx, hw, K, m, lam, p, 77, 3, n_iter, with_W=with_W, base=2)
    err = rel_err(np.concatenate([g.ravel() for g in got]), np.concatenate([r.ravel() for r in refs]))
    say("  rel err", err)
    assert err < TOL32


def test_code_step_warm_start_and_zero_iterations(ctx):
    hw = [(33, 40)]
    K, m = 6, 5
    rng = np.random.default_rng(11)
    z0 = [f32(rng.standard_normal((K, 33, 40)) * (rng.random((K, 33, 40)) < 0.3))]
    got, refs, _, _ = run_code_step(ctx, hw, K, m, 0.2, 0.4, 5, 2, 0, z0=z0)
    np.testing.assert_array_equal(got[0], refs[0])  # z restricted to S, exactly
    got, refs, _, _ = run_code_step(ctx, hw, K, m, 0.2, 0.4, 5, 2, 6, z0=z0)
    assert rel_err(got[0], refs[0]) < TOL32


def test_code_step_nnz_iter_sum(ctx):
    """nnz_iter_sum counts the non-zeros entering each iteration's synthesis."""
    hw = [(40, 37)]
    got1, refs1, st1, _ = run_code_step(ctx, hw, 9, 5, 0.3, 0.5, 4, 2, 1)
    _, _, st2, _ = run_code_step(ctx, hw, 9, 5, 0.3, 0.5, 4, 2, 2)
    assert st1.nnz_iter_sum == 0  # z^0 = 0
    assert st2.nnz_iter_sum == st1.nnz == int(np.count_nonzero(got1[0]))  # z^0 = 0, then z^1


def test_code_step_large_lambda_is_zero(ctx):
    got, refs, st, _ = run_code_step(ctx, [(30, 30)], 8, 5, 1e6, 0.5, 1, 1, 5)
    assert np.count_nonzero(got[0]) == 0 and st.nnz == 0


def test_code_step_rejects_bad_arguments(ctx):
    from paper_1909_00145_amd import CSCError

    im = Images([(8, 8)])
    x = torch.zeros(64, device="cuda")
    d = torch.zeros(2, 3, 3, device="cuda")
    z = torch.full((2 * 64,), 7.0, device="cuda")
    for kw in [dict(p=0.0), dict(p=1.5), dict(lam=-1.0), dict(n_iter=-1)]:
        args = dict(lam=1.0, p=0.5, n_iter=1)
        args.update(kw)
        with pytest.raises(CSCError) as e:
            ctx.code_step(im, x, d, z, args["lam"], args["p"], 1, 1, args["n_iter"], step=1.0)
        assert e.value.status == -1
        assert torch.all(z == 7.0)  # outputs untouched on invalid arguments
    with pytest.raises(CSCError) as e:
        ctx.code_step(im, x, torch.zeros(2, 4, 4, device="cuda"), z, 1.0, 0.5, 1, 1, 1, step=1.0)
    assert e.value.status == -1
    # an image array that is not 4-byte aligned (the buffer holds the whole image after the offset)
    import ctypes as C

    buf = torch.zeros(64 * 4 + 4, dtype=torch.uint8, device="cuda")
    rc = ctx.lib.csc_code_step(ctx.h, im.cref(), C.c_void_p(buf.data_ptr() + 2), None, C.c_void_p(d.data_ptr()),
                               2, 3, C.c_void_p(z.data_ptr()), 1.0, 0.5, 1, 1, 1, 1.0, 0, None)
    assert rc == -1 and b"aligned" in ctx.lib.csc_last_error(ctx.h)
    assert torch.all(z == 7.0)


def test_code_step_full_size_image(ctx):
    """10 images 100 x 100, K = 100, p = 0.1, 20 iterations; image 0 and 7 checked against the oracle."""
    hw = [(100, 100)] * 10
    K, m = 100, 11
    xs, d, _ = make_problem(2, hw, K, m)
    im = Images(hw)
    z = torch.zeros(K * im.n_pix, device="cuda")
    st = ctx.code_step(im, packed(im, xs), to_dev(d), z, 1.0, 0.1, 2, 1, 20, stats=True)
    got = im.unpack(z.cpu().numpy(), K)
    Lz = oracle.lipschitz_code(d, 100)
    for i in (0, 7):
        say("full-size image", i)
        zr, _ = oracle.code_step(xs[i], d, np.zeros((K, 100, 100)), 1.0, 0.1, 2, 1, 20, step=1.0 / Lz, image_index=i)
        err = rel_err(got[i], zr)
        say("  rel err", err)
        assert err < TOL32
    assert 0.09 * K * im.n_pix < st.sampled < 0.11 * K * im.n_pix


# ---------------------------------------------------------------------------
# filter steps (eq. 5; online: eqs. (8)-(9))
# ---------------------------------------------------------------------------
def sparse_codes(hw, K, density, seed):
    rng = np.random.default_rng(seed)
    return [f32(rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < density)) for H, W in hw]


# (20, 150): filter-major lists with several bitmap words per row; (3, 2000) with
# K = 200: bitmaps too large for LDS, so the lists take the scanning fallback
@pytest.mark.parametrize("hw,K,m,n_iter,with_W", [
    ([(64, 64)], 16, 11, 1, False),
    ([(37, 53), (20, 17)], 10, 5, 3, True),
    ([(40, 40)], 100, 11, 1, False),
    ([(20, 150), (9, 70)], 12, 5, 1, True),
    ([(3, 2000)], 200, 3, 1, False),
])
def test_dict_step_batch(ctx, hw, K, m, n_iter, with_W):
    say("dict batch", hw, K, m)
    xs, d, Ws = make_problem(3, hw, K, m, with_W)
    zs = sparse_codes(hw, K, 0.01, 5)
    im = Images(hw)
    dg = to_dev(d)
    Ld = ctx.dict_step(im, packed(im, xs), packed(im, zs), dg, n_iter=n_iter,
                       W=packed(im, Ws, torch.uint8) if Ws else None)
    dr, Ldr = oracle.dict_step_batch(xs, Ws, zs, d, n_iter=n_iter)
    say("  Ld", Ld, Ldr)
    assert abs(Ld - Ldr) <= 1e-5 * Ldr
    assert rel_err(dg.cpu().numpy(), dr) < TOL32


def test_dict_step_zero_codes(ctx):
    hw = [(20, 20)]
    xs, d, _ = make_problem(3, hw, 4, 5)
    im = Images(hw)
    dg = to_dev(d)
    Ld = ctx.dict_step(im, packed(im, xs), torch.zeros(4 * 400, device="cuda"), dg)
    assert Ld == 0.0
    np.testing.assert_array_equal(dg.cpu().numpy(), d.astype(np.float32))


# K = 30 with m = 11: the filter-major lag pass splits the filters into two chunks
@pytest.mark.parametrize("hw,K,m,with_W", [([(30, 26)], 4, 5, False), ([(24, 20), (16, 21)], 3, 11, True),
                                            ([(40, 45), (33, 17)], 5, 11, False), ([(7, 9), (12, 5)], 3, 11, False),
                                            ([(23, 31)], 6, 3, False), ([(20, 24), (13, 30)], 30, 11, False)])
def test_dict_step_online(ctx, hw, K, m, with_W):
    from paper_1909_00145_amd.ops import Surrogate

    say("dict online", hw, K, m)
    xs, d, Ws = make_problem(4, hw, K, m, with_W)
    im = Images(hw)
    sur = Surrogate(K, m)
    st = oracle.OnlineState(K, m)
    dg = to_dev(d)
    dr = d.copy()
    for t in range(3):
        zs = sparse_codes(hw, K, 0.05, 10 + t)
        ctx.dict_step(im, packed(im, xs), packed(im, zs), dg, surrogate=sur,
                      W=packed(im, Ws, torch.uint8) if Ws else None)
        dr = oracle.dict_step_online(xs, Ws, zs, dr, st)
        # the oracle runs its own FP64 filter chain; the GPU keeps FP32 filters
        assert sur.t == st.t
        assert abs(sur.Ld_sum - st.Ld_sum) <= 1e-5 * st.Ld_sum
        Cd = sur.dense_C()
        assert rel_err(Cd, st.C) < 1e-12
        assert rel_err(sur.B.cpu().numpy(), st.B) < 1e-12
        assert rel_err(dg.cpu().numpy(), dr) < TOL32
