"""Philox4x32-10 counter-based generator and Box-Muller normals, numpy.

Generator: Salmon, Moraes, Dror & Shaw (2011), "Parallel random numbers: as
easy as 1, 2, 3" -- 10 rounds of the Philox S-box on a 4x32-bit counter with
a 2x32-bit key bumped by the Weyl constants after every round.
Normal draw (a reading; the paper only says realisations use different
initial random modes): for particle id p the counter is (p lo, p hi, 0, 0) and
the key (seed lo, seed hi); with outputs x0, x1,
    u1 = (x0 + 1) 2^-32,  u2 = x1 2^-32,  z = sqrt(-2 ln u1) cos(2 pi u2).
"""
from __future__ import annotations

import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(counter: np.ndarray, key0: int, key1: int) -> np.ndarray:
    """counter: (4, n) uint32.  Returns (4, n) uint32."""
    c = [counter[i].astype(np.uint64) for i in range(4)]
    k0, k1 = key0 & 0xFFFFFFFF, key1 & 0xFFFFFFFF
    for _ in range(10):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return np.stack([x.astype(np.uint32) for x in c])


def normal_field(seed: int, np_side: int) -> np.ndarray:
    """float32 (np, np, np) N(0,1) field, particle id in C order."""
    n = np_side ** 3
    p = np.arange(n, dtype=np.uint64)
    ctr = np.zeros((4, n), np.uint32)
    ctr[0] = (p & _MASK).astype(np.uint32)
    ctr[1] = (p >> np.uint64(32)).astype(np.uint32)
    out = philox4x32_10(ctr, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    u1 = (out[0].astype(np.float64) + 1.0) * 2.0 ** -32
    u2 = out[1].astype(np.float64) * 2.0 ** -32
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return z.astype(np.float32).reshape((np_side,) * 3)
