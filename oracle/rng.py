"""Philox4x32-10 counter-based generator and the sketch matrices drawn from it.

Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two
32x32->64-bit multiplies with constants 0xD2511F53 and 0xCD9E8D57, the key bumped
by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.

The randomized point selection of Sec. 4.3 needs two N x p random matrices G1,
G2 (per atom and once globally).  Their entries are drawn here as standard
normal deviates: element (mu, m) of sketch stream s uses counter
(idx & 0xffffffff, idx >> 32, s, 0) with idx = mu * p + m and key
(seed & 0xffffffff, seed >> 32); the first two output words x0, x1 give
u_k = (x_k + 0.5) / 2^32 and z = sqrt(-2 ln u0) cos(2 pi u1) (Box-Muller).
Streams: 0, 1 = global G1, G2; 2 + 2I, 3 + 2I = G1, G2 of atom I.
"""
from __future__ import annotations

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  Inputs are uint32-valued arrays (held as
    uint64); returns the four output words as uint64 arrays."""
    c = [np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def sketch_normal(nrow: int, ncol: int, seed: int, stream: int) -> np.ndarray:
    """(nrow, ncol) standard normal matrix for sketch stream ``stream``."""
    idx = np.arange(nrow * ncol, dtype=np.uint64)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    x = philox4x32_10(idx & MASK, idx >> np.uint64(32), np.full_like(idx, stream),
                      np.zeros_like(idx), seed & 0xFFFFFFFF, seed >> 32)
    u0 = (x[0].astype(np.float64) + 0.5) / 4294967296.0
    u1 = (x[1].astype(np.float64) + 0.5) / 4294967296.0
    z = np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)
    return z.reshape(nrow, ncol)
