"""Philox4x32-10 counter-based generator, written from its published definition
(J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11, Sec. 3.3 and Table 2).

Part of the test oracle (see ``oracle/__init__``): not used by the product path.

Definition.  State: a 4-word counter (x0, x1, x2, x3) and a 2-word key
(k0, k1), all 32-bit.  One round maps

    (x0, x1, x2, x3) -> (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),
                         hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0))

with M0 = 0xD2511F53, M1 = 0xCD9E8D57 and hi/lo the halves of the 64-bit
product.  Ten rounds are applied; between consecutive rounds the key is
bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) modulo 2^32.

Arithmetic is done in NumPy uint64 so every 32x32 product is exact.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
SH = np.uint64(32)
ROUNDS = 10


def philox4x32(ctr, key, rounds: int = ROUNDS):
    """Vectorised Philox4x32-R.

    ctr: tuple of 4 integer arrays (broadcastable), key: tuple of 2.
    Returns a uint64 array of shape broadcast(...) + (4,) holding the four
    32-bit output words."""
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & MASK for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) & MASK for k in key)
    x0, x1, x2, x3, k0, k1 = np.broadcast_arrays(x0, x1, x2, x3, k0, k1)
    k0 = k0.copy()
    k1 = k1.copy()
    for r in range(rounds):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * x0          # < 2^64: exact in uint64
        p1 = M1 * x2
        x0, x1, x2, x3 = ((p1 >> SH) ^ x1 ^ k0, p1 & MASK,
                          (p0 >> SH) ^ x3 ^ k1, p0 & MASK)
    return np.stack([x0, x1, x2, x3], axis=-1)
