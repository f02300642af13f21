"""Philox4x32-10 counter-based generator and Box-Muller normals (oracle twin).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Philox4x32 as published by Salmon, Moraes, Dror & Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC 2011): a 4 x 32-bit counter, a 2 x 32-bit
key, ten rounds.  Each round multiplies counter words 0 and 2 by the two
round multipliers (full 64-bit products), and recombines hi/lo halves with
the other counter words and the key; the key is bumped by the two Weyl
constants between rounds.

The block noise of the block-Jacobi preconditioner draws one normal per
entry (block b, row r, column c of an nb x nb block):
    counter = (r*nb + c, b mod 2^32, b div 2^32, stream), key = (seed lo, seed hi)
    x = Philox4x32-10(counter, key)
    u1 = ((x1:x0) >> 11 + 1) 2^-53   in (0, 1]
    u2 = ((x3:x2) >> 11) 2^-53       in [0, 1)
    z  = sqrt(-2 ln u1) cos(2 pi u2)
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: (..., 4) uint32-valued, key: (..., 2).  Returns (..., 4) uint64
    holding 32-bit words."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) & MASK32 for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & MASK32
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = [(hi1 ^ c[1] ^ k0) & MASK32, lo1, (hi0 ^ c[3] ^ k1) & MASK32, lo0]
    return np.stack(c, axis=-1)


def normals_from_words(x):
    """Box-Muller on one Philox output (first variate only)."""
    a = (x[..., 0] | (x[..., 1] << np.uint64(32))) >> np.uint64(11)
    b = (x[..., 2] | (x[..., 3] << np.uint64(32))) >> np.uint64(11)
    u1 = (a.astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = b.astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def block_noise(seed, nb, blocks, stream=0):
    """Standard normals E[b, r, c] for the given block indices (array),
    nb x nb entries each."""
    blocks = np.asarray(blocks, dtype=np.uint64)
    rc = np.arange(nb * nb, dtype=np.uint64)
    B, RC = np.meshgrid(blocks, rc, indexing="ij")
    ctr = np.stack([RC, B & MASK32, B >> np.uint64(32),
                    np.full_like(RC, np.uint64(stream))], axis=-1)
    seed = int(seed)
    key = np.broadcast_to(np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF],
                                   dtype=np.uint64), ctr.shape[:-1] + (2,))
    z = normals_from_words(philox4x32_10(ctr, key))
    return z.reshape(len(blocks), nb, nb)
