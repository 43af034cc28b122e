"""Philox4x32 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11,
"Parallel random numbers: as easy as 1, 2, 3"), written from its definition.

State: a 128-bit counter (four 32-bit words) and a 64-bit key (two words).
One round multiplies words 0 and 2 by two fixed odd constants into 64-bit
products, and mixes high halves with the other words and the key; round r
uses the key advanced r times by two Weyl constants.

The authors' standard form takes ten rounds (Philox4x32-10); they report
seven as the fewest that pass their statistical test batteries.  The sketch
uses seven (``philox4x32_7``).  Pinned by the published known-answer vectors of
the ten-round form in ``tests/golden/philox4x32_10_kat.txt``: directly for ten
rounds, and for seven as the prefix that three further rounds (7, 8, 9) carry to
the same published outputs.

Vectorised over numpy arrays of counters; all arithmetic in uint64 with
explicit 32-bit masking.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)


def philox4x32_rounds(c0, c1, c2, c3, k0, k1, rounds, first=0):
    """Rounds first .. first+rounds-1 of Philox4x32 applied to the counter words (uint64 arrays).
    (k0, k1) is the key of round 0; round r uses it advanced r times."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK
    c1 = np.asarray(c1, dtype=np.uint64) & MASK
    c2 = np.asarray(c2, dtype=np.uint64) & MASK
    c3 = np.asarray(c3, dtype=np.uint64) & MASK
    k0 = (np.asarray(k0, dtype=np.uint64) + np.uint64(first) * W0) & MASK
    k1 = (np.asarray(k1, dtype=np.uint64) + np.uint64(first) * W1) & MASK
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0            # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> S32, p0 & MASK
        hi1, lo1 = p1 >> S32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """The standard ten-round form: four 32-bit output words (uint64 arrays)."""
    return philox4x32_rounds(c0, c1, c2, c3, k0, k1, 10)


def philox4x32_7(c0, c1, c2, c3, k0, k1):
    """The seven-round form the sketch uses: four 32-bit output words (uint64 arrays)."""
    return philox4x32_rounds(c0, c1, c2, c3, k0, k1, 7)
