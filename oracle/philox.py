"""Philox4x32-10 counter-based generator (test infrastructure only).

Written from its published definition: J. K. Salmon, M. A. Moraes, R. O. Dror,
D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11.  A 4x32-bit
counter and a 2x32-bit key go through 10 rounds; each round multiplies words 0
and 2 by the constants 0xD2511F53 and 0xCD9E8D57, takes high and low halves,
and mixes them with the other two words and the key; the key is bumped by the
Weyl constants 0x9E3779B9, 0xBB67AE85 between rounds.

Both the ABC oracle and the product library draw their random numbers from
this function of (seed, stream, particle, draw), so the two sides see the
same variates without sharing code.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32(ctr, key):
    """ctr: uint32 array (..., 4); key: uint32 array (..., 2). Returns uint32 (..., 4)."""
    c = np.array(ctr, dtype=np.uint32, copy=True)
    k = np.array(key, dtype=np.uint32, copy=True)
    c0, c1, c2, c3 = (c[..., i].astype(np.uint64) for i in range(4))
    k0, k1 = k[..., 0].astype(np.uint64), k[..., 1].astype(np.uint64)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & MASK
            k1 = (k1 + np.uint64(W1)) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def uniforms(seed, stream, index, draw):
    """Four U(0,1) doubles per (seed, stream, index, draw).

    counter = (index lo, index hi, draw, stream), key = (seed lo, seed hi).
    Each double uses 53 bits from two 32-bit words: u = (a * 2^21 + (b >> 11) + 0.5) / 2^53,
    so u lies strictly inside (0, 1); words (0,1) give u0, words (2,3) give u1.
    Returns array (..., 2).
    """
    index = np.asarray(index, dtype=np.uint64)
    draw = np.broadcast_to(np.asarray(draw, dtype=np.uint64), index.shape)
    ctr = np.stack([index & MASK, index >> np.uint64(32), draw & MASK,
                    np.full(index.shape, stream, dtype=np.uint64)], axis=-1).astype(np.uint32)
    s = np.uint64(seed)
    key = np.broadcast_to(np.array([s & MASK, s >> np.uint64(32)], dtype=np.uint32), index.shape + (2,))
    w = philox4x32(ctr, key).astype(np.uint64)
    a = (w[..., 0] << np.uint64(21)) + (w[..., 1] >> np.uint64(11))
    b = (w[..., 2] << np.uint64(21)) + (w[..., 3] >> np.uint64(11))
    scale = 1.0 / 9007199254740992.0
    return np.stack([(a.astype(np.float64) + 0.5) * scale, (b.astype(np.float64) + 0.5) * scale], axis=-1)
