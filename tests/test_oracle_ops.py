"""Pins for the oracle's convolution operators (Sec. 3.1 stacked operator D, eq. (5) operator Z).

Independent references: scipy.signal.convolve2d / correlate2d ("same" mode,
zero fill), pure-Python loops written from the definition on tiny inputs, and
the adjoint identities <D z, r> = <z, D^T r>, <Z d, r> = <d, Z^T r>.
"""

import numpy as np
import pytest
from scipy import signal

import oracle

SHAPES = [(1, 3, 7, 9), (3, 5, 12, 10), (2, 11, 13, 16), (4, 1, 5, 6)]


@pytest.mark.parametrize("K,m,H,W", SHAPES)
def test_synthesize_matches_scipy_convolve(rng, K, m, H, W):
    d = rng.standard_normal((K, m, m))
    z = rng.standard_normal((K, H, W))
    ref = sum(signal.convolve2d(z[k], d[k], mode="same", boundary="fill") for k in range(K))
    np.testing.assert_allclose(oracle.synthesize(d, z), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("K,m,H,W", SHAPES)
def test_adjoint_matches_scipy_correlate(rng, K, m, H, W):
    d = rng.standard_normal((K, m, m))
    r = rng.standard_normal((H, W))
    ref = np.stack([signal.correlate2d(r, d[k], mode="same", boundary="fill") for k in range(K)])
    np.testing.assert_allclose(oracle.adjoint(d, r), ref, rtol=1e-12, atol=1e-12)


def test_filter_corr_bruteforce(rng):
    K, m, H, W = 2, 3, 5, 4
    c = m // 2
    z = rng.standard_normal((K, H, W))
    r = rng.standard_normal((H, W))
    G = np.zeros((K, m, m))
    for k in range(K):
        for sy in range(-c, c + 1):
            for sx in range(-c, c + 1):
                acc = 0.0
                for qy in range(H):
                    for qx in range(W):
                        py, px = qy + sy, qx + sx
                        if 0 <= py < H and 0 <= px < W:
                            acc += z[k, qy, qx] * r[py, px]
                G[k, sy + c, sx + c] = acc
    np.testing.assert_allclose(oracle.filter_corr(z, r, m), G, rtol=1e-12, atol=1e-13)


def test_synthesize_bruteforce_tiny(rng):
    K, m, H, W = 2, 3, 4, 5
    c = m // 2
    d = rng.standard_normal((K, m, m))
    z = rng.standard_normal((K, H, W))
    y = np.zeros((H, W))
    for py in range(H):
        for px in range(W):
            for k in range(K):
                for sy in range(-c, c + 1):
                    for sx in range(-c, c + 1):
                        qy, qx = py - sy, px - sx
                        if 0 <= qy < H and 0 <= qx < W:
                            y[py, px] += d[k, sy + c, sx + c] * z[k, qy, qx]
    np.testing.assert_allclose(oracle.synthesize(d, z), y, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("K,m,H,W", SHAPES)
def test_adjoint_identities(rng, K, m, H, W):
    d = rng.standard_normal((K, m, m))
    z = rng.standard_normal((K, H, W))
    r = rng.standard_normal((H, W))
    lhs = np.sum(oracle.synthesize(d, z) * r)
    rhs = np.sum(z * oracle.adjoint(d, r))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    rhs2 = np.sum(d * oracle.filter_corr(z, r, m))
    assert abs(lhs - rhs2) <= 1e-12 * max(1.0, abs(lhs))


def test_code_matrix_is_operator(rng):
    K, m, H, W = 3, 5, 7, 6
    d = rng.standard_normal((K, m, m))
    z = rng.standard_normal((K, H, W))
    Z = oracle.code_matrix(z, m)
    np.testing.assert_allclose(Z @ d.ravel(), oracle.synthesize(d, z).ravel(), rtol=1e-12, atol=1e-12)
    r = rng.standard_normal((H, W))
    np.testing.assert_allclose(Z.T @ r.ravel(), oracle.filter_corr(z, r, m).ravel(), rtol=1e-12, atol=1e-12)


def test_objective_direct(rng):
    K, m, H, W = 2, 3, 6, 5
    d = rng.standard_normal((K, m, m))
    xs = [rng.standard_normal((H, W)), rng.standard_normal((H + 1, W + 2))]
    zs = [rng.standard_normal((K,) + x.shape) for x in xs]
    Ws = [None, (rng.random(xs[1].shape) < 0.5).astype(np.uint8)]
    lam = 0.7
    ref_data = 0.0
    for x, z, Wm in zip(xs, zs, Ws):
        y = sum(signal.convolve2d(z[k], d[k], mode="same") for k in range(K))
        e = x - y if Wm is None else Wm * (x - y)
        ref_data += 0.5 * np.sum(e * e)
    ref_l1 = sum(np.abs(z).sum() for z in zs)
    F, data, l1 = oracle.objective(xs, d, zs, lam, Ws)
    assert abs(data - ref_data) <= 1e-12 * ref_data
    assert abs(l1 - ref_l1) <= 1e-12 * ref_l1
    assert abs(F - (ref_data + lam * ref_l1)) <= 1e-12 * F


def test_project_ball(rng):
    v = rng.standard_normal((5, 3, 3))
    v[0] *= 0.01  # inside the ball: unchanged
    out = oracle.project_ball(v)
    n = np.sqrt((out ** 2).sum(axis=(1, 2)))
    assert np.all(n <= 1 + 1e-15)
    np.testing.assert_array_equal(out[0], v[0])
    for k in range(1, 5):
        assert abs(n[k] - 1.0) < 1e-14
        np.testing.assert_allclose(out[k] * np.linalg.norm(v[k]), v[k], rtol=1e-14)


def test_soft_threshold():
    u = np.array([-3.0, -1.0, -0.5, 0.0, 0.5, 1.0, 2.5])
    np.testing.assert_array_equal(oracle.soft_threshold(u, 1.0), [-2.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.5])
