"""Pins for the oracle's inpainting (reconstruction from observed pixels, Sec. 4)
and its PSNR.

* delta filter (D = I, L_z = 1, step 1): one iteration from zero gives
  S_lambda(x) on the observed pixels and 0 on the others -- exactly;
* the unobserved pixels of x are never read;
* PSNR of x + c against x is 10 log10(range^2 / c^2) exactly;
* with every pixel observed and a delta filter the reconstruction is S_lambda(x),
  and with an observation mask the data term of the result is the masked
  objective's (KKT of the masked LASSO at convergence).
"""

import math

import numpy as np
import pytest

import oracle
from oracle.csc import soft_threshold


def delta(m=3):
    d = np.zeros((1, m, m))
    d[0, m // 2, m // 2] = 1.0
    return d


def test_delta_filter_closed_form(rng):
    H, W = 9, 7
    x = rng.standard_normal((H, W)) * 2
    Wm = (rng.random((H, W)) < 0.5).astype(np.uint8)
    xh, z = oracle.inpaint(x, Wm, delta(), 0.4, 1, step=1.0)
    np.testing.assert_array_equal(xh, np.where(Wm != 0, soft_threshold(x, 0.4), 0.0))


def test_unobserved_pixels_are_not_read(rng):
    K, m, H, W = 3, 5, 12, 10
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    x = rng.standard_normal((H, W))
    Wm = (rng.random((H, W)) < 0.5).astype(np.uint8)
    x2 = np.where(Wm != 0, x, 1e6)
    a, _ = oracle.inpaint(x, Wm, d, 0.3, 5)
    b, _ = oracle.inpaint(x2, Wm, d, 0.3, 5)
    np.testing.assert_array_equal(a, b)


def test_psnr_constant_error(rng):
    x = rng.standard_normal((8, 9))
    c = 0.037
    rng_x = np.max(x) - np.min(x)
    assert oracle.psnr(x + c, x) == pytest.approx(10 * math.log10(rng_x**2 / c**2), rel=1e-12)
    assert oracle.psnr(x, x) == math.inf


def test_masked_kkt_at_convergence():
    rng = np.random.default_rng(2024)
    K, m, H, W = 2, 3, 7, 6
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    x = rng.standard_normal((H, W))
    Wm = (rng.random((H, W)) < 0.6).astype(np.uint8)
    lam = 0.1
    xh, z = oracle.inpaint(x, Wm, d, lam, 20000)
    # gradient of the masked data term, D^T W (x - D z): |g| <= lam on zeros, = lam sign(z) on the support
    g = oracle.adjoint(d, Wm * (x - oracle.synthesize(d, z)))
    assert np.all(np.abs(g[z == 0]) <= lam + 1e-7)
    np.testing.assert_allclose(g[z != 0], lam * np.sign(z[z != 0]), atol=1e-7)
    np.testing.assert_array_equal(xh, oracle.synthesize(d, z))
