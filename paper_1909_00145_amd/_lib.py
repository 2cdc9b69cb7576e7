"""ctypes binding of ``libscsc.so`` (the C ABI declared in ``include/scsc.h``).

Argument marshalling only: every computation happens inside the library.  The
library is loaded from the in-tree ``_lib/`` directory; importing this module
raises if it has not been built (``python -m paper_1909_00145_amd.build``).
"""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libscsc.so")

CSC_OK = 0
CSC_EINVAL = -1
CSC_ENOMEM = -2
CSC_EHIP = -3
CSC_EUNSUPPORTED = -4
CSC_FP32 = 0
CSC_BF16 = 1
CSC_NOALLOC_SCRATCH_BYTES = 8 << 20

STATUS_NAMES = {
    CSC_OK: "CSC_OK",
    CSC_EINVAL: "CSC_EINVAL",
    CSC_ENOMEM: "CSC_ENOMEM",
    CSC_EHIP: "CSC_EHIP",
    CSC_EUNSUPPORTED: "CSC_EUNSUPPORTED",
}


class csc_images(C.Structure):
    _fields_ = [("n", C.c_int32), ("hw", C.POINTER(C.c_int32)), ("index_base", C.c_int32)]


class csc_code_stats(C.Structure):
    _fields_ = [("sampled", C.c_int64), ("nnz", C.c_int64), ("L_z", C.c_double), ("step", C.c_double),
                ("nnz_iter_sum", C.c_int64)]


class csc_surrogate(C.Structure):
    _fields_ = [("C", C.c_void_p), ("B", C.c_void_p), ("t", C.c_int64), ("Ld_sum", C.c_double)]


_vp = C.c_void_p
_i = C.c_int
_d = C.c_double
_u64 = C.c_uint64
_u32 = C.c_uint32
_pimg = C.POINTER(csc_images)

# name -> (restype, argtypes); the same names as the C declarations.
SIGNATURES = {
    "csc_create": (_i, [C.POINTER(_vp), _i, _vp]),
    "csc_destroy": (_i, [_vp]),
    "csc_set_stream": (_i, [_vp, _vp]),
    "csc_last_error": (C.c_char_p, [_vp]),
    "csc_version": (_i, []),
    "csc_code_step": (_i, [_vp, _pimg, _vp, _vp, _vp, _i, _i, _vp, _d, _d, _u64, _u32, _i, _d, _i,
                           C.POINTER(csc_code_stats)]),
    "csc_code_step_hold": (_i, [_vp, _pimg, _vp, _vp, _vp, _i, _i, _vp, _d, _d, _u64, _u32, _i, _d, _i,
                                C.POINTER(csc_code_stats)]),
    "csc_code_step_admm": (_i, [_vp, _pimg, _vp, _vp, _vp, _i, _i, _vp, _d, _d, _u64, _u32, _i, _i, _d, _d,
                                C.POINTER(csc_code_stats)]),
    "csc_dict_step": (_i, [_vp, _pimg, _vp, _vp, _vp, _vp, _i, _i, C.POINTER(csc_surrogate), _i, _d, _i, _i,
                           C.POINTER(_d)]),
    "csc_online_step": (_i, [_vp, _pimg, _vp, _vp, _vp, _i, _i, _vp, _d, _d, _u64, _u32, _i, _d, _i,
                             C.POINTER(csc_surrogate), _i, _i, C.POINTER(csc_code_stats), C.POINTER(_d)]),
    "csc_objective": (_i, [_vp, _pimg, _vp, _vp, _vp, _i, _i, _vp, _d, C.POINTER(_d), C.POINTER(_d)]),
    "csc_objective_noalloc": (_i, [_vp, _pimg, _vp, _vp, _vp, _i, _i, _vp, _d, C.POINTER(_d), C.POINTER(_d)]),
    "csc_synthesize": (_i, [_vp, _pimg, _vp, _i, _i, _vp, _vp, _i]),
    "csc_adjoint": (_i, [_vp, _pimg, _vp, _i, _i, _vp, _vp, _i]),
    "csc_filter_corr": (_i, [_vp, _pimg, _vp, _i, _i, _vp, _vp, _i]),
    "csc_mask": (_i, [_vp, _pimg, _i, _d, _u64, _u32, _vp]),
    "csc_lipschitz_code": (_i, [_vp, _vp, _i, _i, _i, C.POINTER(_d)]),
    "csc_surrogate_size": (C.c_int64, [_i, _i]),
    "csc_surrogate_index": (C.c_int64, [_i, _i, _i, _i, _i, _i, _i, _i]),
    "csc_profile_enable": (_i, [_vp, _i]),
    "csc_profile_read": (_i, [_vp, _i, C.POINTER(C.c_int64), C.POINTER(_d)]),
    "csc_set_autotune": (_i, [_vp, _i]),
    "csc_set_graph": (_i, [_vp, _i]),
    "csc_ista_forward": (_i, [_vp, _pimg, _vp, _vp, _vp, _i, _i, _vp, _vp, _vp, _d, _d, _i]),
    "csc_ista_backward": (_i, [_vp, _pimg, _vp, _vp, _vp, _i, _i, _vp, _vp, _vp, _d, _d, _vp, _vp, _vp, _i]),
}

# csc_kernel_class
KERNEL_CLASSES = ["select", "gather", "synth", "adjoint", "scatter", "lists", "corr", "update", "sur_acc",
                  "sur_mv", "objective", "lipschitz", "dense", "sur_lag", "sur_expand", "sur_corner", "power", "ista_graph"]


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(
            "the HIP library %s is not built; run `python -m paper_1909_00145_amd.build` "
            "(there is no CPU fallback)" % path
        )
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


class CSCError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
