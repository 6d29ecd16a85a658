"""Counter-based uniform noise of the training proxy y_hat = y + u.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw ("Parallel random
numbers: as easy as 1, 2, 3", SC 2011): ten rounds of two 32x32 -> 64-bit
multiplications on a 4-word counter, the 2-word key advanced by the Weyl
constants between rounds.  The noise of element 4g + e is
(word e >> 8) * 2^-24 - 1/2 for the counter (g mod 2^32, g >> 32, it,
stream_id) and the key (seed mod 2^32, seed >> 32).
"""
from __future__ import annotations

import numpy as np

MASK = 0xFFFFFFFF
M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(ctr, key):
    """One block: ctr = 4 words, key = 2 words (Python ints) -> 4 words."""
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for r in range(10):
        if r:
            k0, k1 = (k0 + W0) & MASK, (k1 + W1) & MASK
        p0, p1 = M0 * c0, M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & MASK, p1 & MASK, ((p0 >> 32) ^ c3 ^ k1) & MASK, p0 & MASK
    return c0, c1, c2, c3


def uniform_noise(n, seed, it=0, stream_id=0):
    """n float32 values in [-1/2, 1/2)."""
    key = (seed & MASK, (seed >> 32) & MASK)
    out = np.empty(n, np.float32)
    for g in range((n + 3) // 4):
        w = philox4x32_10((g & MASK, g >> 32, it & MASK, stream_id & MASK), key)
        for e in range(4):
            i = 4 * g + e
            if i < n:
                out[i] = np.float32((w[e] >> 8) * 2.0 ** -24 - 0.5)
    return out
