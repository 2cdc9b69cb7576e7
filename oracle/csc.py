"""Plain FP64 CPU oracle for stochastic convolutional sparse coding.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP path.

Paper: Xiong, Richtarik, Heidrich, "Stochastic Convolutional Sparse Coding"
(VMV 2019).  Conventions (readings of the paper where it is silent; each one
is listed with its reason in the design notes):

* Images x_n are H_n x W_n; codes z_{n,k} have the image's size (Sec. 2); the
  convolution of eq. (1) is linear, "same"-sized, zero outside the image, with
  the m x m filter anchored at its centre c = m // 2 (the spatial domain is
  used precisely to avoid circular boundaries, Sec. 1).
* Synthesis (the stacked operator D of Sec. 3.1):
      (D z)[p] = sum_k sum_{s in [-c,c]^2} d_k[s] z_k[p - s],
  with d_k[s] = d[k, s_y + c, s_x + c].
* Its adjoint: (D^T r)_k[q] = sum_s d_k[s] r[q + s].
* Code-side operator Z of eq. (5) (Z d == D z):  (Z^T r)_k[s] = sum_q z_k[q] r[q + s].
* Bernoulli(p) subsampling (eq. 2): i.i.d. per coordinate, from Philox4x32-10
  keyed by the seed, with counter (l >> 2, n, draw) and word l & 3 for the
  pixel-major coordinate index l = (y W + x) K + k of image n; sampled iff the
  word is < floor(p 2^32).
* Code solver: proximal gradient (ISTA) on the subsampled LASSO of eq. (3),
  step 1/L_z, unselected coordinates held at zero (the upsampling of eq. (4)).
  Optionally (``hold=True``) the unselected coordinates keep their previous
  values instead, as the randomization paragraph of Sec. 3.1 describes (only
  the pDK sampled variables change); their codes then stay in the residual.
* Filter solver: projected gradient on eq. (5) (batch) or on the surrogate
  problem eq. (9) with surrogates accumulated per eq. (8) (online).

Every array is float64 unless noted.  Batches are Python lists (images may have
different sizes).
"""

from __future__ import annotations

import math

import numpy as np

from .philox import philox4x32_10

# ---------------------------------------------------------------------------
# Convolution operators (Sec. 3.1: D z = sum_k d_k * z_k; eq. (5): Z d = D z)
# ---------------------------------------------------------------------------


def _taps(m: int):
    c = m // 2
    for sy in range(-c, c + 1):
        for sx in range(-c, c + 1):
            yield sy, sx


def _check_filters(d: np.ndarray) -> int:
    K, mh, mw = d.shape
    if mh != mw or mh % 2 != 1:
        raise ValueError("filters must be square with odd side")
    return K


def _padded(a: np.ndarray, c: int) -> np.ndarray:
    """a [..., H, W] embedded in c zero pixels on every side."""
    H, W = a.shape[-2:]
    ap = np.zeros(a.shape[:-2] + (H + 2 * c, W + 2 * c))
    ap[..., c : c + H, c : c + W] = a
    return ap


def _shifted_windows(r: np.ndarray, m: int) -> np.ndarray:
    """R[s, q] = r[q + s] (zero outside the image) for the m*m taps s in row-major
    order and the pixels q in row-major order: [m*m, H*W]."""
    c = m // 2
    H, W = r.shape
    rp = _padded(r, c)
    R = np.empty((m * m, H * W))
    for sy, sx in _taps(m):
        R[(sy + c) * m + (sx + c)] = rp[c + sy : c + sy + H, c + sx : c + sx + W].ravel()
    return R


def synthesize(d: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Reconstruction D z = sum_k d_k * z_k of eq. (1) for one image.

    d: [K, m, m]; z: [K, H, W]  ->  [H, W].  The sum over filters is one matrix
    product, Y[s] = sum_k d_k[s] z_k on the zero-padded grid; then
    y[p] = sum_s Y[s][p - s], tap by tap.
    """
    K = _check_filters(d)
    m = d.shape[1]
    c = m // 2
    _, H, W = z.shape
    zp = _padded(z, c)
    Hp, Wp = zp.shape[1:]
    Y = (d.reshape(K, m * m).T @ zp.reshape(K, Hp * Wp)).reshape(m * m, Hp, Wp)
    y = np.zeros((H, W))
    for sy, sx in _taps(m):
        # Y[s] at p - s for p in the image: padded rows (p_y - s_y + c)
        y += Y[(sy + c) * m + (sx + c), c - sy : c - sy + H, c - sx : c - sx + W]
    return y


def adjoint(d: np.ndarray, r: np.ndarray) -> np.ndarray:
    """D^T r: correlation of the residual with every filter, g_k[q] = sum_s d_k[s] r[q + s].
    [H, W] -> [K, H, W]; one matrix product of the filters with the shifted windows of r."""
    K = _check_filters(d)
    m = d.shape[1]
    H, W = r.shape
    return (d.reshape(K, m * m) @ _shifted_windows(r, m)).reshape(K, H, W)


def filter_corr(z: np.ndarray, r: np.ndarray, m: int) -> np.ndarray:
    """Z^T r for one image: G_k[s] = sum_q z_k[q] r[q + s].  [K,H,W],[H,W] -> [K,m,m];
    one matrix product of the codes with the shifted windows of r."""
    K, H, W = z.shape
    return (z.reshape(K, H * W) @ _shifted_windows(r, m).T).reshape(K, m, m)


def code_matrix(z: np.ndarray, m: int) -> np.ndarray:
    """Explicit Z of eq. (5) for one image: [H*W, K*m*m], column (k, s) holds z_k[p - s].

    Column index k*m*m + (s_y + c)*m + (s_x + c) matches a row-major flattening
    of d, so Z @ d.ravel() == synthesize(d, z).ravel().
    """
    K, H, W = z.shape
    c = m // 2
    M = m * m
    zp = np.zeros((K, H + 2 * c, W + 2 * c))
    zp[:, c : c + H, c : c + W] = z
    Z = np.zeros((H * W, K * M))
    for sy, sx in _taps(m):
        si = (sy + c) * m + (sx + c)
        shifted = zp[:, c - sy : c - sy + H, c - sx : c - sx + W]
        for k in range(K):
            Z[:, k * M + si] = shifted[k].ravel()
    return Z


# ---------------------------------------------------------------------------
# Bernoulli subsampling M^t (eq. 2)
# ---------------------------------------------------------------------------


def sample_threshold(p: float) -> int:
    """floor(p * 2^32), exact in binary64; p = 1 gives 2^32 (every word passes)."""
    if not (0.0 < p <= 1.0):
        raise ValueError("p must lie in (0, 1]")
    return int(math.floor(math.ldexp(p, 32)))


def bernoulli_mask(K: int, H: int, W: int, p: float, seed: int, draw: int, image_index: int) -> np.ndarray:
    """Selection of eq. (2) for one image as a bool array [K, H, W].

    Coordinate (k, y, x) has index l = (y*W + x)*K + k; its uniform word is
    word (l & 3) of Philox4x32-10 at counter (lo32(l>>2), hi32(l>>2),
    image_index, draw) under key (lo32(seed), hi32(seed)).
    """
    thr = sample_threshold(p)
    n = H * W * K
    # one Philox call per counter q = l >> 2 gives the words of l = 4q .. 4q + 3
    q = np.arange((n + 3) // 4, dtype=np.uint64)
    seed = int(seed) & ((1 << 64) - 1)
    w = philox4x32_10(
        q & np.uint64(0xFFFFFFFF),
        q >> np.uint64(32),
        np.uint64(image_index & 0xFFFFFFFF),
        np.uint64(draw & 0xFFFFFFFF),
        np.uint64(seed & 0xFFFFFFFF),
        np.uint64(seed >> 32),
    )
    words = np.stack(w, axis=1).reshape(-1)[:n]  # words[l] = word (l & 3) of counter l >> 2
    sampled = words < np.uint64(thr) if thr < (1 << 32) else np.ones(n, dtype=bool)
    sampled = sampled.reshape(H, W, K)  # l = (y W + x) K + k
    # [H, W, K] -> [K, H, W]
    return np.ascontiguousarray(np.transpose(sampled, (2, 0, 1)))


# ---------------------------------------------------------------------------
# Step sizes
# ---------------------------------------------------------------------------


def dft_size(max_side: int, m: int) -> int:
    """Smallest power of two >= max_side + m - 1 (no wrap-around of the full convolution)."""
    need = max_side + m - 1
    P = 1
    while P < need:
        P *= 2
    return P


def lipschitz_code(d: np.ndarray, max_side: int) -> float:
    """Upper bound on ||D||^2 (Lipschitz constant of the data-term gradient in z).

    "Same" convolution with zero boundary is a crop of a P x P circular
    convolution when P >= H + m - 1, so ||D||^2 <= max over the P x P DFT grid
    of sum_k |DFT_P(d_k)(w)|^2.
    """
    m = d.shape[1]
    P = dft_size(max_side, m)
    F = np.fft.fft2(d, s=(P, P), axes=(1, 2))
    return float(np.max(np.sum(np.abs(F) ** 2, axis=0)))


def soft_threshold(u: np.ndarray, t: float) -> np.ndarray:
    """Pointwise shrinkage sign(u) * max(|u| - t, 0) (the L1 proximal map)."""
    return np.sign(u) * np.maximum(np.abs(u) - t, 0.0)


# ---------------------------------------------------------------------------
# Code update: subsampled LASSO eq. (3) by ISTA, upsampled per eq. (4)
# ---------------------------------------------------------------------------


def code_step(
    x: np.ndarray,
    d: np.ndarray,
    z_prev: np.ndarray,
    lam: float,
    p: float,
    seed: int,
    draw: int,
    n_iter: int,
    step: float | None = None,
    W: np.ndarray | None = None,
    image_index: int = 0,
    max_side: int | None = None,
    hold: bool = False,
):
    """One code update for one image.  Returns (z_new [K,H,W], sampled mask [K,H,W]).

    The selected coordinates S (eq. 2) are drawn once and kept for all n_iter
    proximal-gradient iterations.  z starts from z_prev restricted to S; each
    iteration forms the masked residual r = W (x - D z), the gradient D^T r,
    and applies the soft-threshold on S; coordinates off S are zero (eq. 4).

    hold=True: coordinates off S keep their values z_prev throughout (Sec. 3.1,
    randomization paragraph: the variables that are not sampled remain
    unchanged), so z starts from z_prev itself and every residual includes
    them; only S is updated.
    """
    K = d.shape[0]
    H, Wd = x.shape
    S = bernoulli_mask(K, H, Wd, p, seed, draw, image_index)
    if step is None:
        step = 1.0 / lipschitz_code(d, max(H, Wd) if max_side is None else max_side)
    Wm = np.ones_like(x) if W is None else W.astype(np.float64)
    off = np.asarray(z_prev, dtype=np.float64) if hold else 0.0
    z = np.where(S, z_prev, off)
    for _ in range(n_iter):
        r = Wm * (x - synthesize(d, z))
        u = z + step * adjoint(d, r)
        z = np.where(S, soft_threshold(u, step * lam), off)
    return z, S


def code_step_admm(
    x: np.ndarray,
    d: np.ndarray,
    z_prev: np.ndarray,
    lam: float,
    p: float,
    seed: int,
    draw: int,
    n_admm: int = 10,
    n_cg: int = 5,
    rho: float | None = None,
    alpha: float = 1.8,
    W: np.ndarray | None = None,
    image_index: int = 0,
):
    """The paper's code solver for the subsampled LASSO of eq. (3) (Sec. 3.2, the
    paragraph after Alg. 1): ADMM splitting the data term from the L1 term, the
    quadratic substep solved by conjugate gradient, the L1 substep by shrinkage,
    with over-relaxation alpha and penalty rho = 10 lambda.  Returns (z_new, S).

    With A = W D M^T (the sampled columns of D, rows weighted by the observation
    mask), scaled dual u and split variable v, each of the n_admm iterations is
        zt = argmin 1/2 ||W x - A zt||^2 + rho/2 ||zt - v + u||^2
             (n_cg CG iterations on (A^T A + rho I) zt = A^T W x + rho (v - u),
              warm-started from the previous zt),
        zh = alpha zt + (1 - alpha) v,
        v  = S_{lambda/rho}(zh + u),
        u  = u + zh - v.
    zt and v start from z_prev restricted to S, u from 0; the result is v on S and
    zero elsewhere (eq. 4)."""
    K = d.shape[0]
    H, Wd = x.shape
    S = bernoulli_mask(K, H, Wd, p, seed, draw, image_index)
    rho = 10.0 * lam if rho is None else rho
    Wm = np.ones_like(x) if W is None else W.astype(np.float64)

    def A(v):  # S-restricted codes -> weighted image
        return Wm * synthesize(d, np.where(S, v, 0.0))

    def At(r):  # image -> codes on S
        return np.where(S, adjoint(d, Wm * r), 0.0)

    def op(v):
        return At(A(v)) + rho * v

    zt = np.where(S, z_prev, 0.0)
    v = zt.copy()
    u = np.zeros_like(zt)
    b0 = At(x)
    for _ in range(n_admm):
        # conjugate gradient, warm start at the previous zt
        b = b0 + rho * (v - u)
        r = b - op(zt)
        q = r.copy()
        rr = float(np.sum(r * r))
        for _ in range(n_cg):
            if rr == 0.0:
                break
            Aq = op(q)
            a = rr / float(np.sum(q * Aq))
            zt = zt + a * q
            r = r - a * Aq
            rr_new = float(np.sum(r * r))
            q = r + (rr_new / rr) * q
            rr = rr_new
        zh = alpha * zt + (1.0 - alpha) * v
        v = np.where(S, soft_threshold(zh + u, lam / rho), 0.0)
        u = u + zh - v
    return v, S


# ---------------------------------------------------------------------------
# Objective (eq. 1, summed over the images)
# ---------------------------------------------------------------------------


def objective(xs, d, zs, lam: float, Ws=None):
    """(F, data term, L1 term) with F = sum_n 1/2 ||W_n (x_n - D z_n)||^2 + lam sum |z|."""
    data = 0.0
    l1 = 0.0
    for i, (x, z) in enumerate(zip(xs, zs)):
        Wm = 1.0 if Ws is None or Ws[i] is None else Ws[i].astype(np.float64)
        e = Wm * (x - synthesize(d, z))
        data += 0.5 * float(np.sum(e * e))
        l1 += float(np.sum(np.abs(z)))
    return data + lam * l1, data, l1


# ---------------------------------------------------------------------------
# Inpainting (Sec. 4, over-complete dictionaries): reconstruction from a part
# of the pixels
# ---------------------------------------------------------------------------


def inpaint(x, W, d, lam: float, n_iter: int, step: float | None = None, max_side: int | None = None):
    """Reconstruction of a full image from its observed pixels (W = 1).

    The codes solve the masked problem of eq. (1), min_z 1/2 ||W (x - D z)||^2 +
    lam ||z||_1, over every coordinate (p = 1), by n_iter proximal-gradient
    iterations from zero (the paper runs ADMM here); the reconstruction is D z on
    all pixels.  Only x's observed pixels are read.  Returns (x_hat, z)."""
    K = d.shape[0]
    H, Wd = x.shape
    xo = np.where(W != 0, x, 0.0)
    z, _ = code_step(xo, d, np.zeros((K, H, Wd)), lam, 1.0, 0, 0, n_iter, step=step, W=W, max_side=max_side)
    return synthesize(d, z), z


def psnr(x_hat, x) -> float:
    """Peak signal-to-noise ratio of x_hat against x in dB over all pixels, with the
    peak taken as the dynamic range max(x) - min(x) of the original."""
    x = np.asarray(x, dtype=np.float64)
    err = np.asarray(x_hat, dtype=np.float64) - x
    mse = float(np.mean(err * err))
    peak = float(np.max(x) - np.min(x))
    return 10.0 * math.log10(peak * peak / mse) if mse > 0 else math.inf


# ---------------------------------------------------------------------------
# Filter update: eq. (5) (batch) and eqs. (8)-(9) (online)
# ---------------------------------------------------------------------------


def project_ball(v: np.ndarray) -> np.ndarray:
    """Euclidean projection of each filter onto ||d_k||_2 <= 1 (constraint of eq. 1)."""
    nrm = np.sqrt(np.sum(v * v, axis=(1, 2), keepdims=True))
    return v / np.maximum(1.0, nrm)


def _weight(Ws, i):
    return None if Ws is None or Ws[i] is None else Ws[i].astype(np.float64)


def pad_codes(z: np.ndarray, c: int) -> np.ndarray:
    """Codes [K, H, W] embedded with c zero pixels on every side: [K, H + 2c, W + 2c]."""
    K, H, W = z.shape
    zp = np.zeros((K, H + 2 * c, W + 2 * c))
    zp[:, c : c + H, c : c + W] = z
    return zp


def normal_matvec(zs, Ws, v: np.ndarray, padded: bool = False) -> np.ndarray:
    """sum_n Z_n^T W_n Z_n v (v filter-shaped [K, m, m]).

    padded: use the operator Z_n on codes embedded in c zero pixels, i.e. the
    synthesis over the image grown by c (every window that meets the image).
    Its normal matrix is block Toeplitz in the taps: entry (k, s; k2, s2) is the
    lag sum sum_q z_k[q] z_k2[q + s - s2] over the whole image, and it dominates
    the exact sum_n Z_n^T Z_n.  Only defined without an observation mask."""
    m = v.shape[1]
    out = np.zeros_like(v)
    for i, z in enumerate(zs):
        Wm = _weight(Ws, i)
        if padded:
            if Wm is not None:
                raise ValueError("the padded normal operator has no observation mask")
            z = pad_codes(z, m // 2)
        y = synthesize(v, z)
        if Wm is not None:
            y = Wm * y
        out += filter_corr(z, y, m)
    return out


def lipschitz_filter(zs, Ws, K: int, m: int, n_power: int = 20, padded: bool | None = None) -> float:
    """Power-iteration estimate of the filter-step Lipschitz constant L_d.

    The operator is sum_n Z_n^T W_n Z_n with an observation mask, and the
    zero-padded sum_n Z_n^T Z_n of ``normal_matvec(padded=True)`` without one
    (padded=None picks this way).  The padded matrix dominates the exact one,
    so 1 / L_d remains a safe step, and it is built from lag sums alone.
    Starts from the normalised all-ones vector; each iteration takes
    w = A v, the Rayleigh quotient v^T w, and v <- w / ||w||.  Returns the
    last Rayleigh quotient (0 when A v vanishes).
    """
    if padded is None:
        padded = Ws is None or all(w is None for w in Ws)
    v = np.ones((K, m, m)) / math.sqrt(K * m * m)
    lam = 0.0
    for _ in range(n_power):
        w = normal_matvec(zs, None if padded else Ws, v, padded=padded)
        lam = float(np.sum(v * w))
        nw = math.sqrt(float(np.sum(w * w)))
        if nw == 0.0:
            return 0.0
        v = w / nw
    return lam


def dict_step_batch(xs, Ws, zs, d: np.ndarray, n_iter: int = 1, step: float | None = None, n_power: int = 20):
    """Projected-gradient update of eq. (5): d <- P(d + step * sum_n Z_n^T W_n (x_n - Z_n d)).

    step defaults to 1 / L_d with L_d from ``lipschitz_filter``; when L_d is 0
    (all codes zero) the gradient vanishes and d is only projected.
    Returns (d_new, L_d).
    """
    K, m, _ = d.shape
    Ld = lipschitz_filter(zs, Ws, K, m, n_power)
    if step is None:
        step = 0.0 if Ld <= 0.0 else 1.0 / Ld
    for _ in range(n_iter):
        G = np.zeros_like(d)
        for i, (x, z) in enumerate(zip(xs, zs)):
            r = x - synthesize(d, z)
            Wm = _weight(Ws, i)
            if Wm is not None:
                r = Wm * r
            G += filter_corr(z, r, m)
        d = project_ball(d + step * G)
    return d, Ld


def surrogate_increment(xs, Ws, zs, K: int, m: int):
    """(sum_n Z_n^T W_n Z_n, sum_n Z_n^T W_n x_n): the batch terms of eq. (8).

    Returned dense: C_inc [K*m*m, K*m*m], B_inc [K*m*m] (row-major flattening of d).
    """
    KM = K * m * m
    C = np.zeros((KM, KM))
    B = np.zeros(KM)
    for i, (x, z) in enumerate(zip(xs, zs)):
        Z = code_matrix(z, m)
        Wm = _weight(Ws, i)
        w = np.ones(x.size) if Wm is None else Wm.ravel()
        C += Z.T @ (w[:, None] * Z)
        B += Z.T @ (w * x.ravel())
    return C, B


class OnlineState:
    """State of the online learner: unscaled sums C_bar, B_bar, the count t and the
    running sum of per-batch L_d estimates.  C^t = C_bar / t and B^t = B_bar / t
    equal the recursion of eq. (8) started from zero."""

    def __init__(self, K: int, m: int):
        KM = K * m * m
        self.C = np.zeros((KM, KM))
        self.B = np.zeros(KM)
        self.t = 0
        self.Ld_sum = 0.0


def dict_step_online(xs, Ws, zs, d: np.ndarray, state: OnlineState, n_iter: int = 1, n_power: int = 20):
    """Online filter update (surrogates of eq. 8, surrogate problem of eq. 9) for one mini-batch;
    mutates ``state``.

    C_bar += sum Z^T W Z, B_bar += sum Z^T W x, t += 1, Ld_sum += L_d(batch);
    then n_iter steps d <- P(d - (C^t d - B^t) / L^t) with L^t = Ld_sum / t, an
    upper bound on lambda_max(C^t) by subadditivity.  Returns d_new.
    """
    K, m, _ = d.shape
    Cinc, Binc = surrogate_increment(xs, Ws, zs, K, m)
    state.C += Cinc
    state.B += Binc
    state.t += 1
    state.Ld_sum += lipschitz_filter(zs, Ws, K, m, n_power)
    if state.Ld_sum <= 0.0:
        return project_ball(d)
    Ct = state.C / state.t
    Bt = state.B / state.t
    Lt = state.Ld_sum / state.t
    for _ in range(n_iter):
        g = Ct @ d.ravel() - Bt
        d = project_ball(d - (g / Lt).reshape(d.shape))
    return d
