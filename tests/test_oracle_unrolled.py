"""Pins for the oracle's unrolled subsampled ISTA and its reverse-mode gradient:
the layer equals one iteration of the oracle's code step, and the analytic
gradients match central finite differences of the FP64 loss."""

import numpy as np
import pytest

import oracle
from oracle import unrolled


def _problem(rng, H=12, W=14, K=3, m=5, p=0.5):
    x = rng.standard_normal((H, W))
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    S = rng.random((K, H, W)) < p
    z0 = np.where(S, 0.1 * rng.standard_normal((K, H, W)), 0.0)
    eta = 1.0 / oracle.lipschitz_code(d, max(H, W))
    return x, d, S, z0, eta


def test_layer_is_one_code_step_iteration(rng):
    x, d, S, z0, eta = _problem(rng)
    # the oracle's code step draws its own S; compare one iteration with that S
    z_cs, Scs = oracle.code_step(x, d, z0, 0.3, 0.5, 5, 1, 1, step=eta)
    z_l = unrolled.ista_layer(x, d, np.where(Scs, z0, 0.0), Scs, eta, 0.3)
    np.testing.assert_array_equal(z_l, z_cs)


@pytest.mark.parametrize("with_W", [False, True])
def test_gradients_match_finite_differences(rng, with_W):
    x, d, S, z0, eta = _problem(rng)
    W = (rng.random(x.shape) < 0.7).astype(np.uint8) if with_W else None
    lam, T = 0.05, 4
    loss, gz, gd, gx = unrolled.loss_and_grads(x, d, z0, S, eta, lam, T, W)

    def L(dd=d, xx=x, zz=z0):
        return unrolled.reconstruction_loss(xx, dd, unrolled.unrolled_forward(xx, dd, zz, S, eta, lam, T, W)[-1])

    assert abs(L() - loss) <= 1e-12 * loss
    h = 1e-6
    for trial in range(6):
        ed = rng.standard_normal(d.shape)
        ex = rng.standard_normal(x.shape)
        ez = np.where(S, rng.standard_normal(z0.shape), 0.0)
        fd_d = (L(dd=d + h * ed) - L(dd=d - h * ed)) / (2 * h)
        fd_x = (L(xx=x + h * ex) - L(xx=x - h * ex)) / (2 * h)
        fd_z = (L(zz=z0 + h * ez) - L(zz=z0 - h * ez)) / (2 * h)
        for fd, an in ((fd_d, np.sum(gd * ed)), (fd_x, np.sum(gx * ex)), (fd_z, np.sum(gz * ez))):
            assert abs(fd - an) <= 1e-6 * (abs(an) + 1e-3), (trial, fd, an)


def test_gradient_with_all_codes_inactive_is_loss_only(rng):
    """lambda so large that every layer outputs zero: only the loss's direct terms remain."""
    x, d, S, z0, eta = _problem(rng)
    loss, gz, gd, gx = unrolled.loss_and_grads(x, d, z0, S, eta, 1e6, 3)
    assert loss == pytest.approx(0.5 * float(np.sum(x * x)), rel=1e-15)
    np.testing.assert_array_equal(gz, 0.0)
    np.testing.assert_array_equal(gd, 0.0)
    np.testing.assert_array_equal(gx, x)


def test_gradients_finite_differences_differentiation_subset():
    """The differentiation workload's gradient subset: 4 images 32x32 (1/f^2 fields),
    K = 256 filters 11x11, p = 0.2 (the oracle's Bernoulli sample), lambda = 0.5,
    10 layers from zero codes.  Central differences with h = 1e-4 along 6 seeded
    unit directions in d and in x agree with the analytic gradient to 1e-4 of its
    norm (the soft-threshold's kinks bound how close a finite difference can get)."""
    import scsc_inputs as si

    K, m, H, W, N, p, lam, T = 256, 11, 32, 32, 4, 0.2, 0.5, 10
    xs = [si.field(5, n, H, W) for n in range(N)]
    d = si.filters(5, K, m)
    S = [oracle.bernoulli_mask(K, H, W, p, 5, 1, n) for n in range(N)]
    eta = 1.0 / oracle.lipschitz_code(d, H)
    z0 = np.zeros((K, H, W))

    def L(dd, xx):
        return sum(unrolled.reconstruction_loss(xx[n], dd, unrolled.unrolled_forward(xx[n], dd, z0, S[n], eta, lam,
                                                                                      T)[-1]) for n in range(N))

    res = [unrolled.loss_and_grads(xs[n], d, z0, S[n], eta, lam, T) for n in range(N)]
    gd = sum(r[2] for r in res)
    gx = [r[3] for r in res]
    assert abs(sum(r[0] for r in res) - L(d, xs)) <= 1e-12 * L(d, xs)
    ngd = np.linalg.norm(gd)
    ngx = np.sqrt(sum(float((g * g).sum()) for g in gx))
    rng = np.random.default_rng(0)
    h = 1e-4
    for _ in range(6):
        ed = rng.standard_normal(d.shape)
        ed /= np.linalg.norm(ed)
        ex = [rng.standard_normal((H, W)) for _ in range(N)]
        nx = np.sqrt(sum(float((e * e).sum()) for e in ex))
        ex = [e / nx for e in ex]
        fd_d = (L(d + h * ed, xs) - L(d - h * ed, xs)) / (2 * h)
        fd_x = (L(d, [a + h * e for a, e in zip(xs, ex)]) - L(d, [a - h * e for a, e in zip(xs, ex)])) / (2 * h)
        an_d = float(np.sum(gd * ed))
        an_x = sum(float(np.sum(g * e)) for g, e in zip(gx, ex))
        assert abs(fd_d - an_d) <= 1e-4 * ngd, (fd_d, an_d, ngd)
        assert abs(fd_x - an_x) <= 1e-4 * ngx, (fd_x, an_x, ngx)
