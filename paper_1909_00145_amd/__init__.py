"""MI355X (gfx950) implementation of the hot path of stochastic convolutional sparse coding.

The computation lives in the HIP library ``_lib/libscsc.so`` behind the C ABI of
``include/scsc.h``; ``ops`` marshals torch tensors into it, ``drivers`` runs the
batch (SBCSC) and online (SOCSC) outer loops on top of it.
"""

from ._lib import CSC_BF16, CSC_FP32, CSCError  # noqa: F401

__all__ = ["CSC_FP32", "CSC_BF16", "CSCError"]
