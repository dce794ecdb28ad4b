"""Counter-based Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC 2011) and the seeded N(0,1) stream built on it.

Element e of a stream uses counter (e//4, 0, 0, 0) and key (seed & 0xffffffff,
seed >> 32); the four output words w_i become uniforms (w_i + 0.5) 2^-32 and the
pairs (0,1), (2,3) become normals by Box-Muller:
sqrt(-2 ln U0) (cos 2 pi U1, sin 2 pi U1).  Input generation only.
"""
from __future__ import annotations

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32 with 10 rounds; all arguments uint64 arrays holding
    32-bit values.  Returns the four output words."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return c0, c1, c2, c3


def normal_stream(n: int, seed: int) -> np.ndarray:
    """The first n values of the seeded N(0,1) stream."""
    nb = (n + 3) // 4
    q = np.arange(nb, dtype=np.uint64)
    w = philox4x32_10(q & MASK, q >> np.uint64(32), np.zeros_like(q), np.zeros_like(q),
                      np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF))
    u = [(wi.astype(np.float64) + 0.5) * 2.0 ** -32 for wi in w]
    a = np.sqrt(-2.0 * np.log(u[0]))
    c = np.sqrt(-2.0 * np.log(u[2]))
    out = np.empty((nb, 4))
    out[:, 0] = a * np.cos(2 * np.pi * u[1])
    out[:, 1] = a * np.sin(2 * np.pi * u[1])
    out[:, 2] = c * np.cos(2 * np.pi * u[3])
    out[:, 3] = c * np.sin(2 * np.pi * u[3])
    return out.reshape(-1)[:n]
