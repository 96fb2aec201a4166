"""Counter-based random numbers: Philox4x32-10 and Box-Muller normals.

The random inputs of a time step (random forces and torques on the bodies,
the fluctuating-stress field W) are drawn from a counter-based generator so
that any element can be recomputed from its index.  Philox4x32-10 follows its
published definition (Salmon, Moraes, Dror & Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64-bit multiplies with
multipliers 0xD2511F53 and 0xCD9E8D57, the key bumped by the Weyl constants
0x9E3779B9 and 0xBB67AE85 between rounds.

Normal number n of (seed, stream, step):
  counter = (n >> 1, stream, step mod 2^32, step >> 32), key = (seed mod 2^32, seed >> 32)
  (x0, x1, x2, x3) = Philox4x32-10(counter, key)
  u1 = ((x1:x0 >> 12) + 1/2) * 2^-52,  u2 = ((x3:x2 >> 12) + 1/2) * 2^-52   (exact, in (0, 1))
  rho = sqrt(-2 log u1); normal = rho cos(2 pi u2) if n is even else rho sin(2 pi u2)
Streams: 0 = body random forces/torques (6 per body: W^f then W^tau),
         1 = fluid noise W (index space of the nine stress families).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)

STREAM_BODY = 0
STREAM_FLUID = 1


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10; all inputs uint32-valued arrays (held as uint64)."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK
    c1 = np.asarray(c1, dtype=np.uint64) & MASK
    c2 = np.asarray(c2, dtype=np.uint64) & MASK
    c3 = np.asarray(c3, dtype=np.uint64) & MASK
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> S32, p0 & MASK
        hi1, lo1 = p1 >> S32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return c0, c1, c2, c3


def normals(seed: int, stream: int, step: int, index: np.ndarray) -> np.ndarray:
    """Standard normals for the given element indices (uint64-valued)."""
    index = np.asarray(index, dtype=np.uint64)
    pair = index >> np.uint64(1)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    step = int(step) & 0xFFFFFFFFFFFFFFFF
    x0, x1, x2, x3 = philox4x32_10(pair & MASK, np.full(pair.shape, stream, dtype=np.uint64),
                                   np.full(pair.shape, step & 0xFFFFFFFF, dtype=np.uint64),
                                   np.full(pair.shape, step >> 32, dtype=np.uint64),
                                   np.uint64(seed & 0xFFFFFFFF), np.uint64(seed >> 32))
    a = ((x1 << S32) | x0) >> np.uint64(12)
    b = ((x3 << S32) | x2) >> np.uint64(12)
    u1 = (a.astype(np.float64) + 0.5) * 2.0 ** -52
    u2 = (b.astype(np.float64) + 0.5) * 2.0 ** -52
    rho = np.sqrt(-2.0 * np.log(u1))
    ang = (2.0 * np.pi) * u2
    return np.where((index & np.uint64(1)) == 0, rho * np.cos(ang), rho * np.sin(ang))


def body_normals(seed: int, step: int, nb: int):
    """(W^f, W^tau), each (nb, 3)."""
    z = normals(seed, STREAM_BODY, step, np.arange(6 * nb)).reshape(nb, 6)
    return z[:, :3].copy(), z[:, 3:].copy()


def fluid_normals(seed: int, step: int, nW: int) -> np.ndarray:
    return normals(seed, STREAM_FLUID, step, np.arange(nW))
