"""Philox4x32-10 counter-based generator and the maps the samplers use.

The paper draws its Monte Carlo randomness from JAX PRNG keys (Sec. 4.2
"Sampler"); it fixes no generator.  Reading: Philox4x32-10 as published by
Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
(SC'11): a 4 x 32-bit counter, a 2 x 32-bit key, ten rounds; each round
multiplies words 0 and 2 by the two round multipliers, takes high and low
halves, and mixes them with words 1 and 3 and the round key; the key is bumped
by the two Weyl increments between rounds.

Maps (part of the library's documented contract):
  integer in [0, n):   (x * n) >> 32            (multiply-high)
  uniform in [0, 1):   ((x1 << 21) | (x2 >> 11)) * 2^-53
"""
from __future__ import annotations

import numpy as np

MUL0 = np.uint64(0xD2511F53)
MUL1 = np.uint64(0xCD9E8D57)
WEYL0 = np.uint32(0x9E3779B9)
WEYL1 = np.uint32(0xBB67AE85)
_M32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(counter, key):
    """counter: (..., 4) uint32; key: (..., 2) uint32 -> (..., 4) uint32."""
    c = np.asarray(counter, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    shape = np.broadcast_shapes(c.shape[:-1], k.shape[:-1])
    c = np.broadcast_to(c, shape + (4,)).copy()
    k = np.broadcast_to(k, shape + (2,)).copy()
    for rnd in range(10):
        if rnd:
            k[..., 0] = k[..., 0] + WEYL0
            k[..., 1] = k[..., 1] + WEYL1
        p0 = MUL0 * c[..., 0].astype(np.uint64)
        p1 = MUL1 * c[..., 2].astype(np.uint64)
        hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
        lo0 = (p0 & _M32).astype(np.uint32)
        hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
        lo1 = (p1 & _M32).astype(np.uint32)
        c = np.stack([hi1 ^ c[..., 1] ^ k[..., 0], lo1, hi0 ^ c[..., 3] ^ k[..., 1], lo0], axis=-1)
    return c


def seed_key(seed: int) -> np.ndarray:
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32)


def to_index(x, n):
    """Multiply-high map of a uint32 to an integer in [0, n)."""
    return ((np.asarray(x, dtype=np.uint64) * np.uint64(n)) >> np.uint64(32)).astype(np.int64)


def to_uniform(x1, x2):
    """53-bit uniform in [0, 1) from two uint32 words."""
    hi = np.asarray(x1, dtype=np.uint64) << np.uint64(21)
    lo = np.asarray(x2, dtype=np.uint64) >> np.uint64(11)
    return (hi | lo).astype(np.float64) * 2.0 ** -53
