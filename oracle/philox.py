"""Philox4x32-10 counter-based generator and Box-Muller normals (oracle).

Test infrastructure only.  Written from the published definition (Salmon,
Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11):
10 rounds of
    (hi0, lo0) = mulhilo(0xD2511F53, c0),  (hi1, lo1) = mulhilo(0xCD9E8D57, c2)
    c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),  k <- k + (0x9E3779B9, 0xBB67AE85)
Normal number t of stream s under 64-bit key `seed`: counter
(t mod 2^32, t >> 32, s mod 2^32, s >> 32); the first two output words u0, u1
give uniforms (u + 1) 2^-32 in (0, 1] and z = sqrt(-2 ln u0) cos(2 pi u1).
"""
from __future__ import annotations

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    c = [np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3)]
    ka, kb = k0 & 0xFFFFFFFF, k1 & 0xFFFFFFFF
    for _ in range(10):
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ np.uint64(ka), lo1, hi0 ^ c[3] ^ np.uint64(kb), lo0]
        ka = (ka + W0) & 0xFFFFFFFF
        kb = (kb + W1) & 0xFFFFFFFF
    return c


def normals(seed: int, stream: int, count: int) -> np.ndarray:
    t = np.arange(count, dtype=np.uint64)
    c = philox4x32_10(t & MASK, t >> np.uint64(32), np.full(count, stream & 0xFFFFFFFF),
                      np.full(count, (stream >> 32) & 0xFFFFFFFF), seed & 0xFFFFFFFF,
                      (seed >> 32) & 0xFFFFFFFF)
    u0 = (c[0].astype(np.float64) + 1.0) * 2.0 ** -32
    u1 = (c[1].astype(np.float64) + 1.0) * 2.0 ** -32
    return np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)
