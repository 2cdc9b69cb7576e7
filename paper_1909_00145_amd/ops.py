"""Torch-facing binding of the C ABI: tensors in, library calls out.

PyTorch provides device memory and the stream; each method checks device,
dtype and contiguity, marshals pointers and sizes, and calls the library entry
point of the same name.  A non-zero status raises ``CSCError`` with the
library's message.  There is no CPU fallback: without a GPU and the built
library every call raises.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import CSC_BF16, CSC_FP32, CSCError

PRECISIONS = {"fp32": CSC_FP32, "bf16": CSC_BF16, CSC_FP32: CSC_FP32, CSC_BF16: CSC_BF16}


class Images:
    """A batch of image sizes (host) and the sampler's first image index."""

    def __init__(self, hw, index_base: int = 0):
        arr = np.ascontiguousarray(np.asarray(hw, dtype=np.int32).reshape(-1, 2))
        if arr.shape[0] < 1:
            raise ValueError("need at least one image")
        self.hw = arr
        self.index_base = int(index_base)
        self.sizes = arr[:, 0].astype(np.int64) * arr[:, 1].astype(np.int64)
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)])
        self.n_pix = int(self.offsets[-1])
        self._c = _lib.csc_images(arr.shape[0], arr.ctypes.data_as(C.POINTER(C.c_int32)), self.index_base)

    @classmethod
    def uniform(cls, n: int, H: int, W: int, index_base: int = 0) -> "Images":
        return cls([[H, W]] * n, index_base)

    def __len__(self):
        return int(self.hw.shape[0])

    @property
    def max_side(self) -> int:
        return int(self.hw.max())

    def cref(self):
        return C.byref(self._c)

    # packing helpers (host layout conversions, no arithmetic)
    def pack(self, arrays) -> np.ndarray:
        """Concatenate per-image arrays ([H, W] or [K, H, W]) in the packed layout."""
        return np.concatenate([np.ascontiguousarray(a).reshape(-1) for a in arrays])

    def unpack(self, flat, K: int | None = None):
        flat = flat.reshape(-1)
        out = []
        mult = 1 if K is None else K
        for i, (H, W) in enumerate(self.hw):
            a = flat[mult * int(self.offsets[i]) : mult * int(self.offsets[i + 1])]
            out.append(a.reshape((H, W) if K is None else (K, H, W)))
        return out


@dataclass
class CodeStats:
    sampled: int
    nnz: int
    L_z: float
    step: float
    nnz_iter_sum: int = 0


class Surrogate:
    """Online surrogates of eq. (8) as unscaled sums on the device (FP64).

    ``C`` holds the upper blocks (k <= k2) of the symmetric matrix in the
    library's lag layout (``csc_surrogate_index``); ``dense_C()`` expands it for
    inspection (small K only)."""

    def __init__(self, K: int, m: int, device=None):
        self.K, self.m = K, m
        n = int(_lib.lib().csc_surrogate_size(K, m))
        device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.C = torch.zeros(n, dtype=torch.float64, device=device)
        self.B = torch.zeros(K * m * m, dtype=torch.float64, device=device)
        self.t = 0
        self.Ld_sum = 0.0

    def state_dict(self):
        return {"C": self.C, "B": self.B, "t": self.t, "Ld_sum": self.Ld_sum, "K": self.K, "m": self.m}

    def load_state_dict(self, sd):
        self.C.copy_(sd["C"])
        self.B.copy_(sd["B"])
        self.t = int(sd["t"])
        self.Ld_sum = float(sd["Ld_sum"])

    def dense_C(self) -> np.ndarray:
        idx = lag_index_map(self.K, self.m)
        return self.C.cpu().numpy()[idx]


def lag_index_map(K: int, m: int) -> np.ndarray:
    """[KM, KM] int64 positions of the dense surrogate entries in the stored layout.

    Blocks (k, k2 >= k) are stored in row-major order of the upper triangle; an
    entry of a lower block (k > k2) is the transposed entry of block (k2, k)."""
    c = m // 2
    M = m * m
    s = np.arange(M)
    sy, sx = s // m - c, s % m - c
    dy = sy[:, None] - sy[None, :]
    dx = sx[:, None] - sx[None, :]
    wy, wx = m - np.abs(dy), m - np.abs(dx)

    def prefix(a):
        return np.where(a <= 0, (m + a - 1) * (m + a) // 2, m * (m - 1) // 2 + a * m - a * (a - 1) // 2)

    sylo = np.maximum(-c, dy - c)
    sxlo = np.maximum(-c, dx - c)
    within = prefix(dy) * M + wy * prefix(dx) + (sy[:, None] - sylo) * wx + (sx[:, None] - sxlo)
    k = np.arange(K)
    lo = np.minimum(k[:, None], k[None, :])
    hi = np.maximum(k[:, None], k[None, :])
    tri = (lo * (2 * K - lo + 1) // 2 + (hi - lo)) * M * M  # [K, K]
    upper = (k[:, None] <= k[None, :])[:, None, :, None]
    full = tri[:, None, :, None] + np.where(upper, within[None, :, None, :], within.T[None, :, None, :])
    return full.reshape(K * M, K * M).astype(np.int64)


def _ptr(t, dtype, name, numel=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))
    return C.c_void_p(t.data_ptr())


class Context:
    """A library handle bound to one device; calls run on torch's current stream."""

    def __init__(self, device: int | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available: the stochastic-CSC library has no CPU path")
        self.lib = _lib.lib()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = C.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        st = self.lib.csc_create(C.byref(h), self.device, C.c_void_p(stream))
        if st != 0:
            raise CSCError(st, "csc_create failed on device %d" % self.device)
        self.h = h
        self._stream = stream

    def close(self):
        if getattr(self, "h", None):
            self.lib.csc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, enable: bool):
        """Replay the code step's proximal-gradient iterations from a captured HIP graph."""
        self._check(self.lib.csc_set_graph(self.h, 1 if enable else 0))

    def set_autotune(self, enable, variant=None):
        """enable: tune launch variants on first use (default on); variant: force one variant."""
        mode = -(int(variant) + 1) if variant is not None else (1 if enable else 0)
        self._check(self.lib.csc_set_autotune(self.h, mode))

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            self._check(self.lib.csc_set_stream(self.h, C.c_void_p(s)))
            self._stream = s

    def _check(self, st):
        if st != 0:
            raise CSCError(st, self.lib.csc_last_error(self.h).decode())

    # ---- hot path -----------------------------------------------------------

    def code_step(self, im: Images, x, d, z, lam, p, seed, draw, n_iter, step=0.0, W=None, precision="fp32",
                  stats=False, hold=False):
        """hold=True: the unselected coordinates keep their values (csc_code_step_hold)."""
        K, m = int(d.shape[0]), int(d.shape[-1])
        self._sync_stream()
        st = _lib.csc_code_stats()
        fn = self.lib.csc_code_step_hold if hold else self.lib.csc_code_step
        rc = fn(
            self.h, im.cref(), _ptr(x, torch.float32, "x", im.n_pix), _ptr(W, torch.uint8, "W", im.n_pix),
            _ptr(d, torch.float32, "d", K * m * m), K, m, _ptr(z, torch.float32, "z", K * im.n_pix),
            float(lam), float(p), int(seed) & (2**64 - 1), int(draw) & (2**32 - 1), int(n_iter), float(step),
            PRECISIONS[precision], C.byref(st) if stats else None)
        self._check(rc)
        if stats:
            return CodeStats(st.sampled, st.nnz, st.L_z, st.step, st.nnz_iter_sum)
        return None

    def code_step_admm(self, im: Images, x, d, z, lam, p, seed, draw, n_admm=10, n_cg=5, rho=0.0, alpha=1.8, W=None,
                       stats=False):
        """Code update by ADMM (csc_code_step_admm); rho <= 0 selects 10 lambda."""
        K, m = int(d.shape[0]), int(d.shape[-1])
        self._sync_stream()
        st = _lib.csc_code_stats()
        rc = self.lib.csc_code_step_admm(
            self.h, im.cref(), _ptr(x, torch.float32, "x", im.n_pix), _ptr(W, torch.uint8, "W", im.n_pix),
            _ptr(d, torch.float32, "d", K * m * m), K, m, _ptr(z, torch.float32, "z", K * im.n_pix),
            float(lam), float(p), int(seed) & (2**64 - 1), int(draw) & (2**32 - 1), int(n_admm), int(n_cg),
            float(rho), float(alpha), C.byref(st) if stats else None)
        self._check(rc)
        if stats:
            return CodeStats(st.sampled, st.nnz, st.L_z, st.step, st.nnz_iter_sum)
        return None

    def dict_step(self, im: Images, x, z, d, n_iter=1, step=0.0, n_power=20, W=None, surrogate: Surrogate = None,
                  precision="fp32"):
        K, m = int(d.shape[0]), int(d.shape[-1])
        self._sync_stream()
        ld = C.c_double(0.0)
        sur = None
        if surrogate is not None:
            _ptr(surrogate.C, torch.float64, "surrogate.C")
            _ptr(surrogate.B, torch.float64, "surrogate.B", K * m * m)
            sur = _lib.csc_surrogate(surrogate.C.data_ptr(), surrogate.B.data_ptr(), surrogate.t,
                                     surrogate.Ld_sum)
        rc = self.lib.csc_dict_step(
            self.h, im.cref(), _ptr(x, torch.float32, "x", im.n_pix), _ptr(W, torch.uint8, "W", im.n_pix),
            _ptr(z, torch.float32, "z", K * im.n_pix), _ptr(d, torch.float32, "d", K * m * m), K, m,
            C.byref(sur) if sur is not None else None, int(n_iter), float(step), int(n_power),
            PRECISIONS[precision], C.byref(ld))
        self._check(rc)
        if surrogate is not None:
            surrogate.t = int(sur.t)
            surrogate.Ld_sum = float(sur.Ld_sum)
        return ld.value

    def online_step(self, im: Images, x, d, surrogate: Surrogate, lam, p, seed, draw, n_iter, z=None, step=0.0,
                    W=None, precision="fp32", n_dict_iter=1, n_power=20, stats=False):
        """One step of Alg. 2 (csc_online_step): codes of the mini-batch from zero, then the
        surrogate and filter update.  z (optional) receives the codes.  Returns
        (CodeStats or None, L_d of the mini-batch)."""
        K, m = int(d.shape[0]), int(d.shape[-1])
        self._sync_stream()
        _ptr(surrogate.C, torch.float64, "surrogate.C")
        _ptr(surrogate.B, torch.float64, "surrogate.B", K * m * m)
        sur = _lib.csc_surrogate(surrogate.C.data_ptr(), surrogate.B.data_ptr(), surrogate.t, surrogate.Ld_sum)
        st = _lib.csc_code_stats()
        ld = C.c_double(0.0)
        rc = self.lib.csc_online_step(
            self.h, im.cref(), _ptr(x, torch.float32, "x", im.n_pix), _ptr(W, torch.uint8, "W", im.n_pix),
            _ptr(d, torch.float32, "d", K * m * m), K, m, _ptr(z, torch.float32, "z", K * im.n_pix),
            float(lam), float(p), int(seed) & (2**64 - 1), int(draw) & (2**32 - 1), int(n_iter), float(step),
            PRECISIONS[precision], C.byref(sur), int(n_dict_iter), int(n_power), C.byref(st) if stats else None,
            C.byref(ld))
        self._check(rc)
        surrogate.t = int(sur.t)
        surrogate.Ld_sum = float(sur.Ld_sum)
        cs = CodeStats(st.sampled, st.nnz, st.L_z, st.step, st.nnz_iter_sum) if stats else None
        return cs, ld.value

    def objective(self, im: Images, x, d, z, lam, W=None, noalloc=False):
        """Objective of eq. (1); ``noalloc`` calls the entry point that allocates no
        device memory (its scratch is a fixed array in the library)."""
        K, m = int(d.shape[0]), int(d.shape[-1])
        self._sync_stream()
        f = C.c_double()
        terms = (C.c_double * 2)()
        fn = self.lib.csc_objective_noalloc if noalloc else self.lib.csc_objective
        rc = fn(
            self.h, im.cref(), _ptr(x, torch.float32, "x", im.n_pix), _ptr(W, torch.uint8, "W", im.n_pix),
            _ptr(d, torch.float32, "d", K * m * m), K, m, _ptr(z, torch.float32, "z", K * im.n_pix), float(lam),
            C.byref(f), terms)
        self._check(rc)
        return f.value, terms[0], terms[1]

    # ---- operators ------------------------------------------------------------

    def synthesize(self, im: Images, d, z, out=None, precision="fp32"):
        K, m = int(d.shape[0]), int(d.shape[-1])
        out = torch.empty(im.n_pix, dtype=torch.float32, device=z.device) if out is None else out
        self._sync_stream()
        self._check(self.lib.csc_synthesize(self.h, im.cref(), _ptr(d, torch.float32, "d", K * m * m), K, m,
                                            _ptr(z, torch.float32, "z", K * im.n_pix),
                                            _ptr(out, torch.float32, "y", im.n_pix), PRECISIONS[precision]))
        return out

    def adjoint(self, im: Images, d, r, out=None, precision="fp32"):
        K, m = int(d.shape[0]), int(d.shape[-1])
        out = torch.empty(K * im.n_pix, dtype=torch.float32, device=r.device) if out is None else out
        self._sync_stream()
        self._check(self.lib.csc_adjoint(self.h, im.cref(), _ptr(d, torch.float32, "d", K * m * m), K, m,
                                         _ptr(r, torch.float32, "r", im.n_pix),
                                         _ptr(out, torch.float32, "g", K * im.n_pix), PRECISIONS[precision]))
        return out

    def filter_corr(self, im: Images, z, r, K, m, out=None, precision="fp32"):
        out = torch.empty(K * m * m, dtype=torch.float32, device=r.device) if out is None else out
        self._sync_stream()
        self._check(self.lib.csc_filter_corr(self.h, im.cref(), _ptr(z, torch.float32, "z", K * im.n_pix), K, m,
                                             _ptr(r, torch.float32, "r", im.n_pix),
                                             _ptr(out, torch.float32, "G", K * m * m), PRECISIONS[precision]))
        return out

    def ista_forward(self, im: Images, x, d, mask, z_in, eta, lam, W=None, out=None, precision="fp32"):
        K, m = int(d.shape[0]), int(d.shape[-1])
        out = torch.empty_like(z_in) if out is None else out
        self._sync_stream()
        self._check(self.lib.csc_ista_forward(
            self.h, im.cref(), _ptr(x, torch.float32, "x", im.n_pix), _ptr(W, torch.uint8, "W", im.n_pix),
            _ptr(d, torch.float32, "d", K * m * m), K, m, _ptr(mask, torch.uint8, "mask", K * im.n_pix),
            _ptr(z_in, torch.float32, "z_in", K * im.n_pix), _ptr(out, torch.float32, "z_out", K * im.n_pix),
            float(eta), float(lam), PRECISIONS[precision]))
        return out

    def ista_backward(self, im: Images, x, d, mask, z_in, g_out, eta, lam, W=None, want_x=True, precision="fp32"):
        K, m = int(d.shape[0]), int(d.shape[-1])
        g_z = torch.empty_like(z_in)
        g_d = torch.empty_like(d)
        g_x = torch.empty_like(x) if want_x else None
        self._sync_stream()
        self._check(self.lib.csc_ista_backward(
            self.h, im.cref(), _ptr(x, torch.float32, "x", im.n_pix), _ptr(W, torch.uint8, "W", im.n_pix),
            _ptr(d, torch.float32, "d", K * m * m), K, m, _ptr(mask, torch.uint8, "mask", K * im.n_pix),
            _ptr(z_in, torch.float32, "z_in", K * im.n_pix), _ptr(g_out, torch.float32, "g_out", K * im.n_pix),
            float(eta), float(lam), _ptr(g_z, torch.float32, "g_z", K * im.n_pix),
            _ptr(g_d, torch.float32, "g_d", K * m * m), _ptr(g_x, torch.float32, "g_x", im.n_pix),
            PRECISIONS[precision]))
        return g_z, g_d, g_x

    def mask(self, im: Images, K, p, seed, draw, out=None):
        out = torch.empty(K * im.n_pix, dtype=torch.uint8, device=torch.device("cuda", self.device)) \
            if out is None else out
        self._sync_stream()
        self._check(self.lib.csc_mask(self.h, im.cref(), int(K), float(p), int(seed) & (2**64 - 1),
                                      int(draw) & (2**32 - 1), _ptr(out, torch.uint8, "mask", K * im.n_pix)))
        return out

    def lipschitz_code(self, d, max_side):
        K, m = int(d.shape[0]), int(d.shape[-1])
        L = C.c_double()
        self._sync_stream()
        self._check(self.lib.csc_lipschitz_code(self.h, _ptr(d, torch.float32, "d", K * m * m), K, m,
                                                int(max_side), C.byref(L)))
        return L.value
