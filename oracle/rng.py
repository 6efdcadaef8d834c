"""Reference of the counter-based normal generator -- test infrastructure.

Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011): a 128-bit counter (c0, c1, c2, c3) and a 64-bit
key (k0, k1) of 32-bit words; each of ten rounds multiplies c0 and c2 by
fixed constants, keeps the high and low halves of the 64-bit products and
mixes them with the other two counter words and the key; the key is bumped
by two Weyl constants after every round.  The normals come from the
Box-Muller transform of pairs of words, with the same conventions as the
library's generator (see its header): u = ((x >> 8) + 1/2) 2^-24.

Plain Python integers and float64: slow, for a few thousand draws.
"""

from __future__ import annotations

import math

import numpy as np

MUL = (0xD2511F53, 0xCD9E8D57)
WEYL = (0x9E3779B9, 0xBB67AE85)
MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    """Four output words of one block (tuples of four and two 32-bit ints)."""
    c0, c1, c2, c3 = (int(v) & MASK for v in counter)
    k0, k1 = (int(v) & MASK for v in key)
    for _ in range(10):
        p0 = MUL[0] * c0
        p1 = MUL[1] * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & MASK, p1 & MASK, \
                         ((p0 >> 32) ^ c3 ^ k1) & MASK, p0 & MASK
        k0 = (k0 + WEYL[0]) & MASK
        k1 = (k1 + WEYL[1]) & MASK
    return c0, c1, c2, c3


def words(seed, stream_id, counter0, n):
    """The generator word behind each of n draws (uint32 array)."""
    out = np.empty(n, np.uint32)
    key = (seed & MASK, (seed >> 32) & MASK)
    for t in range((n + 3) // 4):
        b = counter0 + t
        w = philox4x32_10((b & MASK, (b >> 32) & MASK, stream_id & MASK,
                           (stream_id >> 32) & MASK), key)
        for e in range(4):
            if 4 * t + e < n:
                out[4 * t + e] = w[e]
    return out


def normals(seed, stream_id, counter0, n):
    """n standard normal draws (float64) by Box-Muller on word pairs."""
    w = words(seed, stream_id, counter0, ((n + 3) // 4) * 4).astype(np.float64)
    u = (np.floor(w / 256.0) + 0.5) * 2.0 ** -24
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty_like(w)
    z[0::2] = r * np.cos(2.0 * math.pi * u2)
    z[1::2] = r * np.sin(2.0 * math.pi * u2)
    return z[:n]
