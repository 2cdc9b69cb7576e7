"""Seeded synthetic inputs shared by the oracle, the GPU path, the tests and the bench.

This module only *generates data*: natural-image stand-ins, random unit-norm
filter banks, ragged image sizes and observation masks.  It contains none of
the sparse-coding arithmetic (no synthesis, no thresholding, no subsampling),
so the CPU oracle and the HIP path can both draw their inputs from it while
sharing no computation.

Image model (the paper trains on contrast-normalised natural images, Sec. 4.1;
those datasets are not available here, so a statistical stand-in is used):

1. white Gaussian noise w ~ N(0, 1) from ``SeedSequence([cfg, n])``;
2. spectral shaping by 1/|f| in amplitude, i.e. a 1/f^2 power spectrum, DC
   removed;
3. local contrast normalisation: subtract a Gaussian-weighted local mean
   (sigma = 2 px, truncated at 4 sigma, reflecting boundary) and divide by the
   local standard deviation, floored at its image mean;
4. a global z-score to zero mean and unit variance.

Filters are N(0, 1) draws normalised to unit L2 norm per filter, matching the
unit-ball constraint of the dictionary (eq. 1).
"""

from __future__ import annotations

import numpy as np
from scipy import ndimage

__all__ = [
    "field",
    "batch",
    "filters",
    "ragged_sizes",
    "observation_mask",
    "stream_batch",
]

LCN_SIGMA = 2.0
LCN_TRUNCATE = 4.0


def field(cfg: int, n: int, H: int, W: int, lcn_sigma: float | None = LCN_SIGMA) -> np.ndarray:
    """One synthetic image (float64, shape [H, W]) for config id ``cfg``, index ``n``.

    lcn_sigma: width (px) of the Gaussian windows of the local contrast
    normalisation; None skips that step (the 1/f^2 field is only z-scored)."""
    rng = np.random.default_rng(np.random.SeedSequence([int(cfg), int(n)]))
    w = rng.standard_normal((H, W))
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    f = np.sqrt(fy * fy + fx * fx)
    amp = np.zeros_like(f)
    amp[f > 0] = 1.0 / f[f > 0]
    g = np.real(np.fft.ifft2(np.fft.fft2(w) * amp))
    if lcn_sigma is None:
        y = g
    else:
        mu = ndimage.gaussian_filter(g, lcn_sigma, mode="reflect", truncate=LCN_TRUNCATE)
        c = g - mu
        v = ndimage.gaussian_filter(c * c, lcn_sigma, mode="reflect", truncate=LCN_TRUNCATE)
        y = c / np.sqrt(np.maximum(v, v.mean()))
    y = y - y.mean()
    s = y.std()
    return y / s if s > 0 else y


def batch(cfg: int, N: int, H: int, W: int, first: int = 0, lcn_sigma: float | None = LCN_SIGMA) -> np.ndarray:
    """N same-size images [N, H, W] (float64), image indices first..first+N-1."""
    return np.stack([field(cfg, first + i, H, W, lcn_sigma) for i in range(N)])


def stream_batch(cfg: int, t: int, batch_size: int, H: int, W: int,
                 lcn_sigma: float | None = LCN_SIGMA) -> np.ndarray:
    """Mini-batch t (1-based) of an image stream: indices (t-1)*b .. t*b-1."""
    return batch(cfg, batch_size, H, W, first=(t - 1) * batch_size, lcn_sigma=lcn_sigma)


def filters(cfg: int, K: int, m: int) -> np.ndarray:
    """K random filters [K, m, m] (float64), each with unit L2 norm."""
    rng = np.random.default_rng(np.random.SeedSequence([int(cfg), 10**6]))
    d = rng.standard_normal((K, m, m))
    nrm = np.sqrt((d * d).sum(axis=(1, 2), keepdims=True))
    return d / nrm


def ragged_sizes(cfg: int, N: int, lo: int = 64, hi: int = 512) -> np.ndarray:
    """N independent (H, W) pairs, integers uniform in [lo, hi] (int64 [N, 2])."""
    rng = np.random.default_rng(np.random.SeedSequence([int(cfg), 10**7]))
    return rng.integers(lo, hi + 1, size=(N, 2))


def observation_mask(cfg: int, n: int, H: int, W: int, frac: float = 0.5) -> np.ndarray:
    """0/1 observation mask (uint8 [H, W]) with each pixel observed w.p. ``frac``."""
    rng = np.random.default_rng(np.random.SeedSequence([int(cfg), int(n), 7]))
    return (rng.random((H, W)) < frac).astype(np.uint8)
