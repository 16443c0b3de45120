"""Philox4x32-10, the counter-based generator that drives PBAS's random choices.

Oracle (test infrastructure only).

Definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11, Sec. 3 "Philox"): a keyed bijection of a 128-bit counter
(four 32-bit words c0..c3) under a 64-bit key (k0, k1).  One round multiplies
c0 and c2 by the two round multipliers, producing 64-bit products split into
high and low halves, and permutes:

    (hi0, lo0) = M0 * c0        (hi1, lo1) = M1 * c2
    c' = (hi1 ^ c1 ^ k0,  lo1,  hi0 ^ c3 ^ k1,  lo0)

with M0 = 0xD2511F53, M1 = 0xCD9E8D57.  Between rounds the key is bumped by the
Weyl constants (0x9E3779B9, 0xBB67AE85) modulo 2^32.  Philox4x32-10 applies ten
rounds, the first with the unbumped key.

Two implementations are kept on purpose: ``philox4x32_10`` (numpy, vectorised
over uint64 lanes) and ``philox4x32_10_int`` (plain Python integers, one
counter at a time).  Parity pin: both agree with the Philox4x32-10 bijection of
the ROCm random-number library, compiled and run on the host by
``tests/test_oracle_philox.py``.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF
ROUNDS = 10


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Vectorised Philox4x32-10 (Salmon et al., SC'11).  Counter words are broadcastable
    uint32-valued arrays.

    Returns four uint32 arrays (the output words x0..x3).
    """
    c = [np.asarray(v, dtype=np.uint64) & np.uint64(MASK32) for v in (c0, c1, c2, c3)]
    c = list(np.broadcast_arrays(*c))
    c = [v.copy() for v in c]
    ka, kb = int(k0) & MASK32, int(k1) & MASK32
    m0, m1, mask = np.uint64(M0), np.uint64(M1), np.uint64(MASK32)
    for r in range(ROUNDS):
        p0 = c[0] * m0
        p1 = c[2] * m1
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [hi1 ^ c[1] ^ np.uint64(ka), lo1, hi0 ^ c[3] ^ np.uint64(kb), lo0]
        ka = (ka + W0) & MASK32
        kb = (kb + W1) & MASK32
    return tuple(v.astype(np.uint32) for v in c)


def philox4x32_10_int(ctr, key):
    """Philox4x32-10 for one counter, in Python integers: ctr = (c0,c1,c2,c3), key = (k0,k1)."""
    c0, c1, c2, c3 = (int(v) & MASK32 for v in ctr)
    k0, k1 = (int(v) & MASK32 for v in key)
    for r in range(ROUNDS):
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0, p1 & MASK32, (p0 >> 32) ^ c3 ^ k1, p0 & MASK32)
        k0 = (k0 + W0) & MASK32
        k1 = (k1 + W1) & MASK32
    return (c0, c1, c2, c3)


def seed_key(seed: int):
    """A 64-bit seed as the Philox key (k0 = low word, k1 = high word)."""
    s = int(seed) & 0xFFFFFFFFFFFFFFFF
    return s & MASK32, s >> 32
