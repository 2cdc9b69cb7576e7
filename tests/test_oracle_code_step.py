"""Pins for the oracle's subsampled code update (eqs. 2-4) and its step size.

* delta filter: D = I, L_z = 1, one ISTA step from 0 gives S_lambda(x) on the
  sample and 0 elsewhere -- exactly;
* lambda >= max |D^T x| on the sample keeps z at 0;
* p = 1 is classical CSC: the objective never increases;
* after many iterations the result equals scikit-learn's coordinate-descent
  Lasso on the explicit subsampled operator D M^T (an independent solver);
* L_z bounds ||D||^2 computed by SVD of the explicit operator.

HOLD (the unselected variables keep their values, Sec. 3.1 randomization
paragraph):
* delta filter: S_lambda(x) on the sample, z_prev elsewhere -- exactly;
* the unselected coordinates are returned bit for bit, and z_prev = 0 or
  p = 1 reduce HOLD to the default;
* converged, the sample equals scikit-learn's Lasso on the sampled columns with
  the held part moved to the target (x - D_off z_prev); KKT holds there;
* the full objective never increases at step 1/L_z.
"""

import numpy as np
import pytest
from scipy import signal

import oracle
from oracle.csc import soft_threshold


def explicit_D(d, H, W):
    """Columns are scipy convolutions of unit impulses: D[:, k*H*W + q] = d_k * e_q."""
    K = d.shape[0]
    D = np.zeros((H * W, K * H * W))
    for k in range(K):
        for q in range(H * W):
            e = np.zeros(H * W)
            e[q] = 1.0
            D[:, k * H * W + q] = signal.convolve2d(e.reshape(H, W), d[k], mode="same").ravel()
    return D


def test_delta_filter_closed_form(rng):
    H, W, m = 9, 8, 3
    d = np.zeros((1, m, m))
    d[0, 1, 1] = 1.0
    assert oracle.lipschitz_code(d, max(H, W)) == pytest.approx(1.0, abs=1e-14)
    x = rng.standard_normal((H, W)) * 2
    lam, p = 0.6, 0.4
    z, S = oracle.code_step(x, d, np.zeros((1, H, W)), lam, p, seed=3, draw=1, n_iter=1, step=1.0)
    expect = np.where(S[0], soft_threshold(x, lam), 0.0)
    np.testing.assert_array_equal(z[0], expect)
    # a second iteration is a fixed point (D = I, step 1)
    z2, _ = oracle.code_step(x, d, z, lam, p, seed=3, draw=1, n_iter=3, step=1.0)
    np.testing.assert_allclose(z2, z, atol=1e-15)


def test_large_lambda_gives_zero(rng):
    K, m, H, W = 3, 5, 10, 9
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    x = rng.standard_normal((H, W))
    S = oracle.bernoulli_mask(K, H, W, 0.5, 11, 2, 0)
    lam_max = np.max(np.abs(oracle.adjoint(d, x))[S])
    z, _ = oracle.code_step(x, d, np.zeros((K, H, W)), lam_max * 1.0001, 0.5, 11, 2, n_iter=10)
    assert np.all(z == 0)
    z, _ = oracle.code_step(x, d, np.zeros((K, H, W)), lam_max * 0.9, 0.5, 11, 2, n_iter=1)
    assert np.count_nonzero(z) >= 1


def test_p1_objective_monotone(rng):
    K, m, H, W = 4, 5, 16, 14
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    x = rng.standard_normal((H, W))
    lam = 0.3
    z = np.zeros((K, H, W))
    L = oracle.lipschitz_code(d, max(H, W))
    prev = oracle.objective([x], d, [z], lam)[0]
    for it in range(30):
        z, S = oracle.code_step(x, d, z, lam, 1.0, 1, 1, n_iter=1, step=1.0 / L)
        assert S.all()
        f = oracle.objective([x], d, [z], lam)[0]
        assert f <= prev + 1e-12 * abs(prev)
        prev = f


def test_converged_matches_sklearn_lasso(rng):
    from sklearn.linear_model import Lasso

    K, m, H, W = 2, 3, 6, 5
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    x = rng.standard_normal((H, W))
    lam, p = 0.15, 0.6
    z, S = oracle.code_step(x, d, np.zeros((K, H, W)), lam, p, 21, 4, n_iter=20000)
    D = explicit_D(d, H, W)
    cols = S.reshape(-1)  # [K*H*W] in (k, y, x) order, same as D's columns
    A = D[:, cols]
    n = A.shape[0]
    las = Lasso(alpha=lam / n, fit_intercept=False, tol=1e-14, max_iter=1000000)
    las.fit(A, x.ravel())
    ref = np.zeros(K * H * W)
    ref[cols] = las.coef_
    np.testing.assert_allclose(z.ravel(), ref, atol=2e-7, rtol=0)
    # KKT of the subsampled LASSO: |g| <= lam on zeros, g = lam sign(z) on the support
    g = oracle.adjoint(d, x - oracle.synthesize(d, z))[S]
    zs = z[S]
    assert np.all(np.abs(g[zs == 0]) <= lam + 1e-7)
    np.testing.assert_allclose(g[zs != 0], lam * np.sign(zs[zs != 0]), atol=1e-7)


@pytest.mark.parametrize("K,m,H,W", [(3, 5, 12, 12), (2, 3, 7, 10), (1, 11, 12, 9)])
def test_lipschitz_code_bounds_operator_norm(rng, K, m, H, W):
    d = rng.standard_normal((K, m, m))
    D = explicit_D(d, H, W)
    smax = np.linalg.svd(D, compute_uv=False)[0]
    L = oracle.lipschitz_code(d, max(H, W))
    assert L >= smax ** 2 * (1 - 1e-12)
    # the bound is also not absurdly loose on these sizes
    assert L <= 3.0 * smax ** 2


def test_dft_size():
    assert oracle.dft_size(100, 11) == 128
    assert oracle.dft_size(118, 11) == 128
    assert oracle.dft_size(119, 11) == 256
    assert oracle.dft_size(64, 11) == 128


def test_hold_delta_filter_closed_form():
    rng = np.random.default_rng(11)
    H, W, m = 9, 8, 3
    d = np.zeros((1, m, m))
    d[0, 1, 1] = 1.0
    x = rng.standard_normal((H, W)) * 2
    z0 = rng.standard_normal((1, H, W))
    lam, p = 0.6, 0.4
    z, S = oracle.code_step(x, d, z0, lam, p, seed=3, draw=1, n_iter=1, step=1.0, hold=True)
    # on the sample u = z0 + (x - z0) = x up to one rounding of each operation
    np.testing.assert_allclose(z[0][S[0]], soft_threshold(x, lam)[S[0]], rtol=0, atol=1e-14)
    np.testing.assert_array_equal(z[0][~S[0]], z0[0][~S[0]])
    assert 0 < S.sum() < S.size


def test_hold_keeps_unselected_and_reduces_to_default():
    rng = np.random.default_rng(12)
    K, m, H, W = 3, 5, 11, 10
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    x = rng.standard_normal((H, W))
    z0 = rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.3)
    z, S = oracle.code_step(x, d, z0, 0.2, 0.5, 7, 3, n_iter=4, hold=True)
    np.testing.assert_array_equal(z[~S], z0[~S])
    # zero start: nothing to hold
    za, _ = oracle.code_step(x, d, np.zeros_like(z0), 0.2, 0.5, 7, 3, n_iter=4, hold=True)
    zb, _ = oracle.code_step(x, d, np.zeros_like(z0), 0.2, 0.5, 7, 3, n_iter=4)
    np.testing.assert_array_equal(za, zb)
    # p = 1: every coordinate is sampled
    za, S1 = oracle.code_step(x, d, z0, 0.2, 1.0, 7, 3, n_iter=4, hold=True)
    zb, _ = oracle.code_step(x, d, z0, 0.2, 1.0, 7, 3, n_iter=4)
    assert S1.all()
    np.testing.assert_array_equal(za, zb)


def test_hold_converged_matches_sklearn_lasso():
    rng = np.random.default_rng(13)
    from sklearn.linear_model import Lasso

    K, m, H, W = 2, 3, 6, 5
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    x = rng.standard_normal((H, W))
    z0 = rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.5)
    lam, p = 0.15, 0.6
    z, S = oracle.code_step(x, d, z0, lam, p, 21, 4, n_iter=20000, hold=True)
    D = explicit_D(d, H, W)
    cols = S.reshape(-1)
    A = D[:, cols]
    target = x.ravel() - D[:, ~cols] @ z0.reshape(-1)[~cols]
    n = A.shape[0]
    las = Lasso(alpha=lam / n, fit_intercept=False, tol=1e-14, max_iter=1000000)
    las.fit(A, target)
    ref = z0.reshape(-1).copy()
    ref[cols] = las.coef_
    np.testing.assert_allclose(z.ravel(), ref, atol=2e-7, rtol=0)
    g = oracle.adjoint(d, x - oracle.synthesize(d, z))[S]
    zs = z[S]
    assert np.all(np.abs(g[zs == 0]) <= lam + 1e-7)
    np.testing.assert_allclose(g[zs != 0], lam * np.sign(zs[zs != 0]), atol=1e-7)


def test_hold_objective_monotone():
    rng = np.random.default_rng(14)
    K, m, H, W = 4, 5, 16, 14
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    x = rng.standard_normal((H, W))
    lam = 0.3
    z = rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.2)
    L = oracle.lipschitz_code(d, max(H, W))
    prev = oracle.objective([x], d, [z], lam)[0]
    for it in range(12):
        z, S = oracle.code_step(x, d, z, lam, 0.3, 5, it, n_iter=2, step=1.0 / L, hold=True)
        f = oracle.objective([x], d, [z], lam)[0]
        assert f <= prev + 1e-12 * abs(prev)
        prev = f


# ADMM (the paper's code solver, Sec. 3.2)
def test_admm_delta_filter_converges_to_shrinkage():
    rng = np.random.default_rng(15)
    """D = I: the subsampled LASSO's solution is S_lambda(x) on the sample."""
    H, W, m = 9, 8, 3
    d = np.zeros((1, m, m))
    d[0, 1, 1] = 1.0
    x = rng.standard_normal((H, W)) * 2
    lam = 0.5
    z, S = oracle.code_step_admm(x, d, np.zeros((1, H, W)), lam, 0.4, 3, 1, n_admm=200, n_cg=2)
    np.testing.assert_allclose(z[0], np.where(S[0], soft_threshold(x, lam), 0.0), atol=1e-10)


def test_admm_converged_matches_sklearn_lasso():
    rng = np.random.default_rng(16)
    from sklearn.linear_model import Lasso

    K, m, H, W = 2, 3, 6, 5
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    x = rng.standard_normal((H, W))
    lam, p = 0.15, 0.6
    z, S = oracle.code_step_admm(x, d, np.zeros((K, H, W)), lam, p, 21, 4, n_admm=3000, n_cg=30)
    D = explicit_D(d, H, W)
    cols = S.reshape(-1)
    A = D[:, cols]
    las = Lasso(alpha=lam / A.shape[0], fit_intercept=False, tol=1e-14, max_iter=1000000)
    las.fit(A, x.ravel())
    ref = np.zeros(K * H * W)
    ref[cols] = las.coef_
    np.testing.assert_allclose(z.ravel(), ref, atol=1e-7, rtol=0)


def test_admm_cg_solves_the_quadratic_substep():
    rng = np.random.default_rng(17)
    """With enough CG iterations, the first ADMM step's zt solves (A^T A + rho I) zt = A^T x
    exactly (zero start): check the returned v against the shrinkage of the explicit solve."""
    K, m, H, W = 2, 3, 5, 6
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    x = rng.standard_normal((H, W))
    lam, p, alpha = 0.2, 0.7, 1.8
    rho = 10 * lam
    z, S = oracle.code_step_admm(x, d, np.zeros((K, H, W)), lam, p, 5, 2, n_admm=1, n_cg=200, alpha=alpha)
    D = explicit_D(d, H, W)
    cols = S.reshape(-1)
    A = D[:, cols]
    zt = np.linalg.solve(A.T @ A + rho * np.eye(A.shape[1]), A.T @ x.ravel())
    v = soft_threshold(alpha * zt, lam / rho)  # v0 = u0 = 0
    ref = np.zeros(K * H * W)
    ref[cols] = v
    np.testing.assert_allclose(z.ravel(), ref, atol=1e-10)


def test_admm_with_mask_reduces_masked_objective():
    rng = np.random.default_rng(18)
    K, m, H, W = 3, 5, 12, 11
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    x = rng.standard_normal((H, W))
    Wm = (rng.random((H, W)) < 0.6).astype(np.uint8)
    lam = 0.2
    z, S = oracle.code_step_admm(x, d, np.zeros((K, H, W)), lam, 0.5, 9, 1, W=Wm)
    f0 = oracle.objective([x], d, [np.zeros((K, H, W))], lam, [Wm])[0]
    f1 = oracle.objective([x], d, [z], lam, [Wm])[0]
    assert f1 < 0.9 * f0
    assert np.all(z[~S] == 0)
