"""Outer loops of the method on top of the library: batch (Alg. 1) and online (Alg. 2).

Both alternate a subsampled code update (eqs. 2-4) with a filter update; the
batch learner solves eq. (5) over all images each outer iteration, the online
learner draws a mini-batch per iteration and updates the surrogates of eq. (8)
before solving eq. (9).  Mini-batching (the paper's extension of Alg. 2) is the
batch dimension of every call.
"""

from __future__ import annotations

import math

import torch

from .ops import Context, Images, Surrogate


class BatchLearner:
    """Stochastic batch CSC (Alg. 1): codes of every image are kept across outer
    iterations and warm-started on the new sample.  hold=True keeps the codes off
    the sample as they are (the HOLD reading of Sec. 3.1) instead of zeroing them."""

    def __init__(self, ctx: Context, im: Images, x, d, lam: float, p: float, n_code_iter: int = 20,
                 seed: int = 1, n_dict_iter: int = 1, n_power: int = 20, W=None, precision: str = "fp32",
                 hold: bool = False):
        self.ctx, self.im, self.x, self.d, self.W = ctx, im, x, d, W
        self.K, self.m = int(d.shape[0]), int(d.shape[-1])
        self.lam, self.p, self.T, self.seed = lam, p, n_code_iter, seed
        self.n_dict_iter, self.n_power, self.precision, self.hold = n_dict_iter, n_power, precision, hold
        self.z = torch.zeros(self.K * im.n_pix, dtype=torch.float32, device=x.device)
        self.t = 0

    def step(self):
        """One outer iteration: sample, code update for every image, filter update."""
        self.t += 1
        st = self.ctx.code_step(self.im, self.x, self.d, self.z, self.lam, self.p, self.seed, self.t, self.T,
                                W=self.W, precision=self.precision, stats=True, hold=self.hold)
        Ld = self.ctx.dict_step(self.im, self.x, self.z, self.d, n_iter=self.n_dict_iter, n_power=self.n_power,
                                W=self.W, precision=self.precision)
        return st, Ld

    def objective(self):
        return self.ctx.objective(self.im, self.x, self.d, self.z, self.lam, W=self.W)


class OnlineLearner:
    """Stochastic online CSC (Alg. 2) with mini-batches: every step codes a new
    mini-batch from zero, folds it into the surrogates and updates the filters."""

    def __init__(self, ctx: Context, im: Images, d, lam: float, p: float, n_code_iter: int = 20, seed: int = 1,
                 n_dict_iter: int = 1, n_power: int = 20, precision: str = "fp32", keep_codes: bool = False):
        """keep_codes: write every mini-batch's codes to ``self.z`` (else they stay on the
        device as lists only, and ``self.z`` is None)."""
        self.ctx, self.im, self.d = ctx, im, d
        self.K, self.m = int(d.shape[0]), int(d.shape[-1])
        self.lam, self.p, self.T, self.seed = lam, p, n_code_iter, seed
        self.n_dict_iter, self.n_power, self.precision = n_dict_iter, n_power, precision
        self.sur = Surrogate(self.K, self.m, device=d.device)
        self.z = torch.zeros(self.K * im.n_pix, dtype=torch.float32, device=d.device) if keep_codes else None

    @property
    def t(self):
        return self.sur.t

    def step(self, x, W=None):
        """Process one mini-batch x (packed like ``im``): one csc_online_step."""
        draw = self.sur.t + 1
        return self.ctx.online_step(self.im, x, self.d, self.sur, self.lam, self.p, self.seed, draw, self.T,
                                    z=self.z, W=W, precision=self.precision, n_dict_iter=self.n_dict_iter,
                                    n_power=self.n_power, stats=True)

    def evaluate(self, im: Images, x, n_iter: int = 50, lam: float | None = None, W=None, p: float = 1.0):
        """Objective of eq. (1) on held-out images with codes fitted from zero by n_iter
        FP32 proximal-gradient iterations on a Bernoulli(p) sample.  The sample is draw 0
        of the learner's seed, which no training step uses, so repeated evaluations of one
        dictionary see the same coordinates.  p = 1 codes every coordinate; p = the
        learner's own rate with n_iter = its iteration count evaluates the dictionary
        under the code update it is trained with."""
        lam = self.lam if lam is None else lam
        z = torch.zeros(self.K * im.n_pix, dtype=torch.float32, device=x.device)
        self.ctx.code_step(im, x, self.d, z, lam, p, self.seed, 0, n_iter, W=W, precision="fp32")
        return self.ctx.objective(im, x, self.d, z, lam, W=W)

    def state_dict(self):
        return {"d": self.d.detach().clone(), "sur": {k: (v.clone() if torch.is_tensor(v) else v)
                                                      for k, v in self.sur.state_dict().items()}}

    def load_state_dict(self, sd):
        self.d.copy_(sd["d"])
        self.sur.load_state_dict(sd["sur"])


def inpaint(ctx: Context, im: Images, x, W, d, lam: float = 0.4, n_iter: int = 50, precision: str = "fp32"):
    """Reconstruction of every image of the batch from its observed pixels (W = 1),
    as in the inpainting experiment of Sec. 4: codes of the masked problem of
    eq. (1) over every coordinate (p = 1) by n_iter proximal-gradient iterations
    from zero, then D z on all pixels.  The unobserved pixels of x are not used.
    Returns (x_hat, z), packed like x and z."""
    K = int(d.shape[0])
    z = torch.zeros(K * im.n_pix, dtype=torch.float32, device=x.device)
    ctx.code_step(im, x, d, z, lam, 1.0, 0, 0, n_iter, W=W, precision=precision)
    return ctx.synthesize(im, d, z, precision=precision), z


def psnr(im: Images, x_hat, x):
    """Per-image PSNR (dB) of x_hat against x over all pixels, with the peak taken as
    the dynamic range max(x) - min(x) of the original image (an evaluation in
    FP64 on the device)."""
    out = []
    for i, (H, W) in enumerate(im.hw):
        o = int(im.offsets[i])
        a = x[o:o + H * W].double()
        e = x_hat[o:o + H * W].double() - a
        mse = float((e * e).mean())
        peak = float(a.max() - a.min())
        out.append(10.0 * math.log10(peak * peak / mse) if mse > 0 else math.inf)
    return out
