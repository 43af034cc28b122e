"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11,
"Parallel random numbers: as easy as 1, 2, 3"), written from its definition.

State: a 128-bit counter (four 32-bit words) and a 64-bit key (two words).
One round multiplies words 0 and 2 by two fixed odd constants into 64-bit
products, and mixes high halves with the other words and the key; between
rounds the key is advanced by two Weyl constants.  Ten rounds are used.

Vectorised over numpy arrays of counters; all arithmetic in uint64 with
explicit 32-bit masking.  Pinned by the generator's published known-answer
vectors in ``tests/golden/philox4x32_10_kat.txt``.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Return the four 32-bit output words (uint64 arrays) for the given counters and key."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK
    c1 = np.asarray(c1, dtype=np.uint64) & MASK
    c2 = np.asarray(c2, dtype=np.uint64) & MASK
    c3 = np.asarray(c3, dtype=np.uint64) & MASK
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0            # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> S32, p0 & MASK
        hi1, lo1 = p1 >> S32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3
