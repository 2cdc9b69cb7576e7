"""Differentiable operators over the library's kernels.

* ``synthesis(ctx, im, z, d)``: y = D z (Sec. 3.1); backward
  dz = D^T g (adjoint kernel), dd = Z^T g (filter-correlation kernel).
* ``adjoint(ctx, im, r, d)``: g = D^T r; backward dr = D g_z (synthesis
  kernel), dd[k][s] = sum_q g_z,k[q] r[q + s] (filter correlation).
* ``unrolled_ista(...)``: T layers of the subsampled proximal-gradient code
  update of eqs. (3)-(4) with a fixed selection; each layer's forward and
  backward are single library calls (``csc_ista_forward`` /
  ``csc_ista_backward``), and a layer keeps only its input codes for the
  backward pass, which recomputes the residual and the shrink argument.
  ``checkpoint_every = c > 1`` keeps only every c-th layer input and
  recomputes the others during the backward pass.

The step eta is a plain float (held fixed under differentiation); the
selection mask is a uint8 tensor packed like the codes (``Context.mask``).
``precision="bf16"`` runs every product of the forward and backward passes
with BF16 operands on the matrix cores and FP32 accumulation (codes, filters,
residuals and gradients stay FP32).  All tensors live on the GPU; there is no
CPU path.
"""

from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

from .ops import Context, Images


class _Synthesis(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx: Context, im: Images, z, d, precision: str):
        fctx.ctx, fctx.im, fctx.prec = ctx, im, precision
        fctx.save_for_backward(z, d)
        return ctx.synthesize(im, d.contiguous(), z.contiguous(), precision=precision)

    @staticmethod
    def backward(fctx, g):
        z, d = fctx.saved_tensors
        ctx, im, prec = fctx.ctx, fctx.im, fctx.prec
        g = g.contiguous()
        K, m = int(d.shape[0]), int(d.shape[-1])
        gz = ctx.adjoint(im, d, g, precision=prec) if fctx.needs_input_grad[2] else None
        gd = ctx.filter_corr(im, z, g, K, m, precision=prec).view_as(d) if fctx.needs_input_grad[3] else None
        return None, None, gz, gd, None


class _Adjoint(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx: Context, im: Images, r, d, precision: str):
        fctx.ctx, fctx.im, fctx.prec = ctx, im, precision
        fctx.save_for_backward(r, d)
        return ctx.adjoint(im, d.contiguous(), r.contiguous(), precision=precision)

    @staticmethod
    def backward(fctx, gz):
        r, d = fctx.saved_tensors
        ctx, im, prec = fctx.ctx, fctx.im, fctx.prec
        gz = gz.contiguous()
        K, m = int(d.shape[0]), int(d.shape[-1])
        gr = ctx.synthesize(im, d, gz, precision=prec) if fctx.needs_input_grad[2] else None
        gd = ctx.filter_corr(im, gz, r, K, m, precision=prec).view_as(d) if fctx.needs_input_grad[3] else None
        return None, None, gr, gd, None


class _IstaLayer(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx: Context, im: Images, z, d, x, mask, W, eta: float, lam: float, precision: str):
        fctx.ctx, fctx.im, fctx.eta, fctx.lam, fctx.prec = ctx, im, eta, lam, precision
        fctx.save_for_backward(z, d, x, mask, W)
        return ctx.ista_forward(im, x.contiguous(), d.contiguous(), mask, z.contiguous(), eta, lam, W=W,
                                precision=precision)

    @staticmethod
    def backward(fctx, g_out):
        z, d, x, mask, W = fctx.saved_tensors
        gz, gd, gx = fctx.ctx.ista_backward(fctx.im, x, d, mask, z, g_out.contiguous(), fctx.eta, fctx.lam, W=W,
                                            want_x=fctx.needs_input_grad[4], precision=fctx.prec)
        return None, None, gz, gd, gx, None, None, None, None, None


def synthesis(ctx: Context, im: Images, z, d, precision: str = "fp32"):
    """D z with gradients for z and d."""
    return _Synthesis.apply(ctx, im, z, d, precision)


def adjoint(ctx: Context, im: Images, r, d, precision: str = "fp32"):
    """D^T r with gradients for r and d."""
    return _Adjoint.apply(ctx, im, r, d, precision)


def ista_layer(ctx: Context, im: Images, z, d, x, mask, eta: float, lam: float, W=None, precision: str = "fp32"):
    """mask * shrink(z + eta D^T W (x - D z), eta * lam) with gradients for z, d and x."""
    return _IstaLayer.apply(ctx, im, z, d, x, mask, W, float(eta), float(lam), precision)


def unrolled_ista(ctx: Context, im: Images, x, d, z0, mask, eta: float, lam: float, n_layers: int, W=None,
                  checkpoint_every: int = 1, precision: str = "fp32"):
    """z_T of n_layers stacked layers from z0 (differentiable in z0, d and x)."""
    z = z0
    if checkpoint_every <= 1:
        for _ in range(n_layers):
            z = ista_layer(ctx, im, z, d, x, mask, eta, lam, W, precision)
        return z

    def segment(zz, dd, xx, count):
        for _ in range(count):
            zz = ista_layer(ctx, im, zz, dd, xx, mask, eta, lam, W, precision)
        return zz

    done = 0
    while done < n_layers:
        count = min(checkpoint_every, n_layers - done)
        z = checkpoint(segment, z, d, x, count, use_reentrant=False)
        done += count
    return z
