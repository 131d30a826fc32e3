"""Philox4x32-10 counter-based generator, written from its published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the constants
0xD2511F53 and 0xCD9E8D57, a Weyl key schedule with increments 0x9E3779B9 and
0xBB67AE85.  Test infrastructure only; vectorised over numpy arrays of
counters.
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: uint32 array [..., 4]; key: uint32 array [..., 2] (broadcast).
    Returns uint32 [..., 4]."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.broadcast_to(np.asarray(key, dtype=np.uint32), c.shape[:-1] + (2,))
    c0, c1, c2, c3 = (c[..., i].astype(np.uint64) for i in range(4))
    k0 = k[..., 0].astype(np.uint32)
    k1 = k[..., 1].astype(np.uint32)
    with np.errstate(over="ignore"):
        for _ in range(10):
            p0 = M0 * c0
            p1 = M1 * c2
            hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
            hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
            c0, c1, c2, c3 = (hi1 ^ c1 ^ k0.astype(np.uint64), lo1,
                              hi0 ^ c3 ^ k1.astype(np.uint64), lo0)
            k0 = (k0 + W0).astype(np.uint32)
            k1 = (k1 + W1).astype(np.uint32)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def u01(x):
    """uint32 -> double in (0, 1): (x + 0.5) / 2^32."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)
