"""Philox4x32-10 counter-based generator (test infrastructure only).

Written from the published definition in Salmon, Moraes, Dror & Shaw, "Parallel
Random Numbers: As Easy as 1, 2, 3" (SC'11), Section 4 (Philox): each of the ten
rounds multiplies counter words 0 and 2 by two fixed 32-bit multipliers, keeps the
high and low halves of the two 64-bit products, XORs the high halves with the other
two counter words and the two key words, and permutes the words; the key is bumped
by two Weyl constants between rounds.

Two independent implementations live here: ``philox4x32_10`` (vectorised NumPy on
uint64 carriers) and ``philox4x32_10_int`` (pure-Python integers, one block at a
time).  Tests require them to agree bit for bit, and both are checked against
rocRAND's host-side Philox4x32-10 as an external implementation.
"""
import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9  # golden ratio
PHILOX_W1 = 0xBB67AE85  # sqrt(3) - 1
ROUNDS = 10
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  All arguments are arrays (or scalars) of values in
    [0, 2^32); returns four uint32 arrays, the generator's output block."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for r in range(ROUNDS):
        p0 = m0 * c0  # < 2^64, exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r + 1 < ROUNDS:
            k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK
            k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def philox4x32_10_int(counter, key):
    """Pure-Python reference: ``counter`` is a 4-tuple and ``key`` a 2-tuple of ints."""
    x = [int(v) & 0xFFFFFFFF for v in counter]
    k = [int(v) & 0xFFFFFFFF for v in key]
    for r in range(ROUNDS):
        a = PHILOX_M0 * x[0]
        b = PHILOX_M1 * x[2]
        x = [((b >> 32) ^ x[1] ^ k[0]) & 0xFFFFFFFF, b & 0xFFFFFFFF,
             ((a >> 32) ^ x[3] ^ k[1]) & 0xFFFFFFFF, a & 0xFFFFFFFF]
        if r + 1 < ROUNDS:
            k = [(k[0] + PHILOX_W0) & 0xFFFFFFFF, (k[1] + PHILOX_W1) & 0xFFFFFFFF]
    return tuple(x)


def key_words(seed: int):
    """64-bit seed -> (low word, high word) Philox key."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32
