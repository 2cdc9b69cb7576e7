"""Philox4x32-10 counter-based generator, NumPy reference (test infrastructure).

Source: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11 -- the Philox-4x32 bijection with 10
rounds.  One round maps a counter (c0, c1, c2, c3) under key (k0, k1) to

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))

with M0 = 0xD2511F53, M1 = 0xCD9E8D57; between rounds the key is bumped by
the Weyl constants (0x9E3779B9, 0xBB67AE85) modulo 2^32.  Ten rounds use the
original key followed by nine bumped keys.

All arithmetic is done on uint64 arrays holding 32-bit values so that the
64-bit products are exact.
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)
SH32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Apply Philox4x32-10 elementwise; arguments broadcast; returns 4 uint64 arrays < 2^32."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & MASK32 for v in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0
        p1 = M1 * c2
        n0 = (p1 >> SH32) ^ c1 ^ k0
        n1 = p1 & MASK32
        n2 = (p0 >> SH32) ^ c3 ^ k1
        n3 = p0 & MASK32
        c0, c1, c2, c3 = n0, n1, n2, n3
    return c0, c1, c2, c3
