"""Philox4x64-10 counter-based generator, written from its published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11, Sec. 3 (the Philox S-box: a 64x64->128 bit
multiply, the high half XORed with the other counter word and the round key; the
key is bumped by the Weyl constants after every round; 10 rounds).

Pinned against numpy.random.Philox (the library's own implementation of the same
generator) in tests/test_oracle_pins.py.

Vectorised over numpy uint64 arrays.  The 128-bit product is formed from 32-bit
halves so that every intermediate fits in uint64.
"""
import numpy as np

# Round multipliers and Weyl key increments of Philox4x64 (SC'11, Table 2).
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)
ROUNDS = 10

_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """Return (hi, lo) of the full 128-bit product a*b of uint64 arrays."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _MASK32, a >> _S32
    b_lo, b_hi = b & _MASK32, b >> _S32
    with np.errstate(over="ignore"):
        ll = a_lo * b_lo
        lh = a_lo * b_hi
        hl = a_hi * b_lo
        hh = a_hi * b_hi
        mid = (ll >> _S32) + (lh & _MASK32) + (hl & _MASK32)
        lo = (ll & _MASK32) | ((mid & _MASK32) << _S32)
        hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Apply Philox4x64-`rounds` to counters (c0..c3) under key (k0, k1).

    All arguments broadcast as uint64 arrays; returns four uint64 arrays.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64)
    k1 = np.asarray(k1, dtype=np.uint64)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
    for r in range(rounds):
        hi0, lo0 = mulhilo64(PHILOX_M0, c0)
        hi1, lo1 = mulhilo64(PHILOX_M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r + 1 < rounds:
            with np.errstate(over="ignore"):
                k0 = k0 + PHILOX_W0
                k1 = k1 + PHILOX_W1
    return c0, c1, c2, c3
