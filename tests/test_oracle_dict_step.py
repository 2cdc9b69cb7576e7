"""Pins for the oracle's filter updates: batch eq. (5) and online eqs. (8)-(9).

* one delta code (K = 1, z = e_q inside the image): Z^T Z = I, L_d = 1 and one
  projected step from any d lands on P(patch_q(x)) -- exactly;
* L_d from power iteration against eigvalsh of the explicit normal matrix;
* surrogates: symmetric PSD, diag(C)_(k,s) = sum_p z_k[p - s]^2 (written from
  the definition with loops), C d - B = -Z^T W (x - Z d), and the running
  sums divided by t equal the eq. (8) recursion;
* the online step at t = 1 equals the batch projected-gradient step with the
  same step size;
* past t = 1: single delta codes give a closed form at every t, the t = 2 step
  equals the batch step on the union of both mini-batches with step
  1 / (L_1 + L_2), a repeated mini-batch gives the batch step at every t, and
  each step lowers the eq. (9) surrogate objective built from explicit code
  matrices.
"""

import numpy as np
import pytest

import oracle


def test_single_delta_code_closed_form(rng):
    H, W, m = 12, 13, 5
    c = m // 2
    x = rng.standard_normal((H, W))
    z = np.zeros((1, H, W))
    qy, qx = 6, 5
    z[0, qy, qx] = 1.0
    d0 = oracle.project_ball(rng.standard_normal((1, m, m)))
    d1, Ld = oracle.dict_step_batch([x], None, [z], d0)
    assert Ld == pytest.approx(1.0, rel=1e-12)
    patch = x[qy - c : qy + c + 1, qx - c : qx + c + 1][None]
    np.testing.assert_allclose(d1, oracle.project_ball(patch), rtol=1e-12, atol=1e-14)
    C, B = oracle.surrogate_increment([x], None, [z], 1, m)
    np.testing.assert_allclose(C, np.eye(m * m), atol=0)
    np.testing.assert_allclose(B, patch.ravel(), atol=0)


def test_lipschitz_filter_vs_eigvalsh(rng):
    K, m = 3, 3
    zs = [rng.standard_normal((K, 8, 9)) * (rng.random((K, 8, 9)) < 0.3), rng.standard_normal((K, 6, 7))]
    Ws = [None, (rng.random((6, 7)) < 0.7).astype(np.uint8)]
    A = sum(oracle.code_matrix(z, m).T @ ((1.0 if w is None else w.ravel()[:, None]) * oracle.code_matrix(z, m))
            for z, w in zip(zs, Ws))
    top = np.linalg.eigvalsh(A)[-1]
    est = oracle.lipschitz_filter(zs, Ws, K, m, n_power=200)
    assert 0.99 * top <= est <= top * (1 + 1e-12)


def test_padded_normal_matrix_is_lag_sums_and_dominates(rng):
    """Zero-padded normal matrix: entry (k, s; k2, s2) = sum_q z_k[q] z_k2[q + s - s2] (brute force),
    it dominates the exact sum Z^T Z, and the power estimate matches its top eigenvalue."""
    K, m, H, W = 2, 5, 7, 9
    c = m // 2
    M = m * m
    zs = [rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.5), rng.standard_normal((K, 4, 6))]
    A = sum(oracle.code_matrix(z, m).T @ oracle.code_matrix(z, m) for z in zs)
    P = sum(oracle.code_matrix(oracle.pad_codes(z, c), m).T @ oracle.code_matrix(oracle.pad_codes(z, c), m)
            for z in zs)
    for k in range(K):
        for k2 in range(K):
            for s in range(M):
                for s2 in range(M):
                    dy = s // m - s2 // m
                    dx = s % m - s2 % m
                    ref = 0.0
                    for z in zs:
                        Hh, Ww = z.shape[1:]
                        for y in range(Hh):
                            for x in range(Ww):
                                if 0 <= y + dy < Hh and 0 <= x + dx < Ww:
                                    ref += z[k, y, x] * z[k2, y + dy, x + dx]
                    assert abs(P[k * M + s, k2 * M + s2] - ref) <= 1e-12 * (1 + abs(ref))
    assert np.linalg.eigvalsh(P - A)[0] >= -1e-10  # P - A is PSD
    top = np.linalg.eigvalsh(P)[-1]
    est = oracle.lipschitz_filter(zs, None, K, m, n_power=300)
    assert 0.99 * top <= est <= top * (1 + 1e-12)
    assert est >= np.linalg.eigvalsh(A)[-1] * 0.99


def test_zero_codes_leave_filters(rng):
    d = oracle.project_ball(rng.standard_normal((2, 3, 3)))
    x = rng.standard_normal((6, 6))
    d1, Ld = oracle.dict_step_batch([x], None, [np.zeros((2, 6, 6))], d)
    assert Ld == 0.0
    # zero codes: the step is d <- P(d); P is idempotent up to the rounding of the norm
    np.testing.assert_array_equal(d1, oracle.project_ball(d))
    np.testing.assert_allclose(d1, d, rtol=0, atol=1e-15)


def test_surrogate_structure(rng):
    K, m, H, W = 2, 3, 7, 6
    c = m // 2
    z = rng.standard_normal((K, H, W)) * (rng.random((K, H, W)) < 0.4)
    x = rng.standard_normal((H, W))
    Wm = (rng.random((H, W)) < 0.6).astype(np.uint8)
    C, B = oracle.surrogate_increment([x], [Wm], [z], K, m)
    np.testing.assert_allclose(C, C.T, atol=0)
    assert np.linalg.eigvalsh(C)[0] >= -1e-10
    M = m * m
    for k in range(K):
        for sy in range(-c, c + 1):
            for sx in range(-c, c + 1):
                acc = 0.0
                for py in range(H):
                    for px in range(W):
                        qy, qx = py - sy, px - sx
                        if 0 <= qy < H and 0 <= qx < W and Wm[py, px]:
                            acc += z[k, qy, qx] ** 2
                i = k * M + (sy + c) * m + (sx + c)
                assert C[i, i] == pytest.approx(acc, rel=1e-12, abs=1e-14)
    # C d - B = -Z^T W (x - Z d)
    d = rng.standard_normal((K, m, m))
    r = Wm * (x - oracle.synthesize(d, z))
    np.testing.assert_allclose(C @ d.ravel() - B, -oracle.filter_corr(z, r, m).ravel(), rtol=1e-11, atol=1e-11)


def test_online_running_mean_equals_recursion(rng):
    K, m = 2, 3
    st = oracle.OnlineState(K, m)
    Crec = np.zeros((K * m * m,) * 2)
    Brec = np.zeros(K * m * m)
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    for t in range(1, 5):
        x = rng.standard_normal((6, 7))
        z = rng.standard_normal((K, 6, 7)) * (rng.random((K, 6, 7)) < 0.3)
        Ci, Bi = oracle.surrogate_increment([x], None, [z], K, m)
        Crec = (t - 1) / t * Crec + Ci / t
        Brec = (t - 1) / t * Brec + Bi / t
        d = oracle.dict_step_online([x], None, [z], d, st)
        assert st.t == t
        np.testing.assert_allclose(st.C / st.t, Crec, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(st.B / st.t, Brec, rtol=1e-13, atol=1e-14)


def test_online_first_step_equals_batch(rng):
    K, m = 3, 5
    xs = [rng.standard_normal((10, 9)), rng.standard_normal((8, 11))]
    zs = [rng.standard_normal((K,) + x.shape) * (rng.random((K,) + x.shape) < 0.2) for x in xs]
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    d_batch, Ld = oracle.dict_step_batch(xs, None, zs, d)
    st = oracle.OnlineState(K, m)
    d_online = oracle.dict_step_online(xs, None, zs, d, st)
    assert st.Ld_sum == pytest.approx(Ld, rel=1e-14)
    np.testing.assert_allclose(d_online, d_batch, rtol=1e-11, atol=1e-12)


def test_batch_dict_step_decreases_objective(rng):
    K, m, H, W = 4, 5, 16, 16
    x = rng.standard_normal((H, W))
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    z, _ = oracle.code_step(x, d, np.zeros((K, H, W)), 0.2, 1.0, 1, 1, n_iter=30)
    f0 = oracle.objective([x], d, [z], 0.2)[0]
    for _ in range(5):
        d, _ = oracle.dict_step_batch([x], None, [z], d)
        f1 = oracle.objective([x], d, [z], 0.2)[0]
        assert f1 <= f0 + 1e-12 * f0
        f0 = f1
    assert np.all(np.sqrt((d ** 2).sum(axis=(1, 2))) <= 1 + 1e-14)


# ---------------------------------------------------------------------------
# The online step past its first mini-batch (eq. (8) averaging, eq. (9) step).
# At t >= 2 the surrogates are C^t = (C_1 + ... + C_t) / t and
# B^t = (B_1 + ... + B_t) / t, and the step divides by L^t = (L_1 + ... + L_t) / t.
# Each pin below fails if one of the three averages is dropped or mis-scaled.
# ---------------------------------------------------------------------------


def test_online_delta_codes_closed_form_over_t(rng):
    """Mini-batch t holds one image x_t with a single code a_t at pixel q_t (K = 1).
    Then C_t = a_t^2 I, B_t = a_t patch_{q_t}(x_t), L_t = a_t^2, and for any
    previous filter the step lands on P(sum_i a_i patch_i / sum_i a_i^2)."""
    m, H, W = 5, 11, 12
    c = m // 2
    st = oracle.OnlineState(1, m)
    d = oracle.project_ball(rng.standard_normal((1, m, m)))
    num = np.zeros((1, m, m))
    den = 0.0
    for t in range(1, 5):
        x = rng.standard_normal((H, W))
        a = float(rng.uniform(0.5, 2.0)) * (1 if t % 2 else -1)
        qy, qx = int(rng.integers(c, H - c)), int(rng.integers(c, W - c))
        z = np.zeros((1, H, W))
        z[0, qy, qx] = a
        num += a * x[qy - c : qy + c + 1, qx - c : qx + c + 1][None]
        den += a * a
        d = oracle.dict_step_online([x], None, [z], d, st)
        assert st.Ld_sum == pytest.approx(den, rel=1e-12)
        np.testing.assert_allclose(d, oracle.project_ball(num / den), rtol=1e-12, atol=1e-14)


def test_online_second_step_is_batch_step_on_both_minibatches(rng):
    """(C^2 d - B^2) / L^2 = -sum_{both batches} Z^T (x - Z d) / (L_1 + L_2): the
    t = 2 step equals the batch step of eq. (5) over the union of the two
    mini-batches with step 1 / (L_1 + L_2)."""
    K, m = 3, 5
    mk = lambda: [rng.standard_normal((9, 10)), rng.standard_normal((8, 7))]
    xa, xb = mk(), mk()
    za = [rng.standard_normal((K,) + x.shape) * (rng.random((K,) + x.shape) < 0.25) for x in xa]
    zb = [rng.standard_normal((K,) + x.shape) * (rng.random((K,) + x.shape) < 0.25) for x in xb]
    d0 = oracle.project_ball(rng.standard_normal((K, m, m)))
    st = oracle.OnlineState(K, m)
    d1 = oracle.dict_step_online(xa, None, za, d0, st)
    d2 = oracle.dict_step_online(xb, None, zb, d1, st)
    La = oracle.lipschitz_filter(za, None, K, m)
    Lb = oracle.lipschitz_filter(zb, None, K, m)
    ref, _ = oracle.dict_step_batch(xa + xb, None, za + zb, d1, step=1.0 / (La + Lb))
    np.testing.assert_allclose(d2, ref, rtol=1e-11, atol=1e-12)
    assert not np.allclose(d2, d1)


def test_online_repeated_minibatch_is_batch_step(rng):
    """The same mini-batch fed t times: C^t = C_1, B^t = B_1, L^t = L_1, so every
    online step equals the batch step from the current filters."""
    K, m = 2, 3
    xs = [rng.standard_normal((7, 8))]
    zs = [rng.standard_normal((K, 7, 8)) * (rng.random((K, 7, 8)) < 0.3)]
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    st = oracle.OnlineState(K, m)
    for t in range(1, 5):
        ref, _ = oracle.dict_step_batch(xs, None, zs, d)
        d = oracle.dict_step_online(xs, None, zs, d, st)
        np.testing.assert_allclose(d, ref, rtol=1e-11, atol=1e-12)


def test_online_step_decreases_surrogate_objective(rng):
    """For t = 2..4 the projected step does not increase the eq. (9) surrogate
    objective f_t(d) = 1/2 d^T C^t d - d^T B^t (built here from explicit code
    matrices), since 1 / L^t is a descent step for C^t."""
    K, m = 3, 3
    st = oracle.OnlineState(K, m)
    Csum = np.zeros((K * m * m,) * 2)
    Bsum = np.zeros(K * m * m)
    d = oracle.project_ball(rng.standard_normal((K, m, m)))
    for t in range(1, 5):
        x = rng.standard_normal((8, 9))
        z = rng.standard_normal((K, 8, 9)) * (rng.random((K, 8, 9)) < 0.3)
        Z = oracle.code_matrix(z, m)
        Csum += Z.T @ Z
        Bsum += Z.T @ x.ravel()
        f = lambda v: 0.5 * v.ravel() @ (Csum / t) @ v.ravel() - v.ravel() @ (Bsum / t)
        d_new = oracle.dict_step_online([x], None, [z], d, st)
        if t >= 2:
            assert f(d_new) <= f(d) + 1e-12 * abs(f(d))
        d = d_new
