"""FP64 oracle of unrolled subsampled ISTA and its reverse-mode gradient.

TEST INFRASTRUCTURE ONLY (same import rule as ``oracle.csc``).

A layer is one proximal-gradient iteration of the subsampled code problem
(eq. (3), upsampled per eq. (4)) with a fixed selection S, step eta and
threshold eta * lambda:

    r = W (x - D z),   u = z + eta D^T r,   z' = S * shrink(u, eta * lambda).

Stacking T layers from z0 gives z_T; the training loss of an unrolled network
is the squared reconstruction error 0.5 * ||x - D z_T||^2.  The backward pass
is written out from the chain rule, one layer at a time, recomputing r and u
from the layer input (what a checkpointed implementation stores):

    g_u  = g_out * S * [|u| > eta * lambda]        (derivative of the shrink)
    t    = W (D g_u)
    g_z  = g_u - eta D^T t
    g_x  = eta t
    g_d  = eta (Z(g_u)^T r - Z(z)^T t)

where Z(a)^T b is the filter correlation sum_q a_k[q] b[q + s].  Each function
handles one image; batches sum the filter gradients.
"""

from __future__ import annotations

import numpy as np

from .csc import adjoint, filter_corr, soft_threshold, synthesize


def _w(W, x):
    return np.ones_like(x) if W is None else W.astype(np.float64)


def ista_layer(x, d, z, S, eta: float, lam: float, W=None):
    """One layer: S * shrink(z + eta D^T W (x - D z), eta * lam)."""
    r = _w(W, x) * (x - synthesize(d, z))
    u = z + eta * adjoint(d, r)
    return np.where(S, soft_threshold(u, eta * lam), 0.0)


def unrolled_forward(x, d, z0, S, eta: float, lam: float, n_layers: int, W=None):
    """[z0, z1, ..., zT] of T stacked layers."""
    zs = [z0]
    for _ in range(n_layers):
        zs.append(ista_layer(x, d, zs[-1], S, eta, lam, W))
    return zs


def layer_backward(x, d, z, S, eta: float, lam: float, g_out, W=None):
    """Gradients of <g_out, layer(z)> with respect to (z, d, x), recomputing r and u from z."""
    m = d.shape[1]
    Wm = _w(W, x)
    r = Wm * (x - synthesize(d, z))
    u = z + eta * adjoint(d, r)
    g_u = np.where(S & (np.abs(u) > eta * lam), g_out, 0.0)
    t = Wm * synthesize(d, g_u)
    g_z = g_u - eta * adjoint(d, t)
    g_x = eta * t
    g_d = eta * (filter_corr(g_u, r, m) - filter_corr(z, t, m))
    return g_z, g_d, g_x


def reconstruction_loss(x, d, z):
    """0.5 * ||x - D z||^2."""
    e = x - synthesize(d, z)
    return 0.5 * float(np.sum(e * e))


def loss_and_grads(x, d, z0, S, eta: float, lam: float, n_layers: int, W=None):
    """Loss of the unrolled network and its gradients with respect to (z0, d, x)."""
    m = d.shape[1]
    zs = unrolled_forward(x, d, z0, S, eta, lam, n_layers, W)
    e = x - synthesize(d, zs[-1])
    loss = 0.5 * float(np.sum(e * e))
    # direct terms of the loss: d/dz_T = -D^T e, d/dd = -Z(z_T)^T e, d/dx = e
    g = -adjoint(d, e)
    g_d = -filter_corr(zs[-1], e, m)
    g_x = e.copy()
    for i in range(n_layers - 1, -1, -1):
        g, gd_i, gx_i = layer_backward(x, d, zs[i], S, eta, lam, g, W)
        g_d += gd_i
        g_x += gx_i
    return loss, g, g_d, g_x
