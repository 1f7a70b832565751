"""Philox4x64-10 counter-based generator, written from its published
definition (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11).  Test infrastructure only.

The paper draws "without replacement" from the residual squared-norm
distribution (Alg. 2, sampling step) but fixes no generator.  For bit-exact
skeleton parity the two implementations draw candidate number j of block t of
ID ``id`` from

    x_j = word 0 of Philox4x64-10(counter = (j, t, id, 0), key = (seed, 0)).

The generator maps a 256-bit counter and a 128-bit key to four 64-bit words
through ten rounds.  One round multiplies counter words 0 and 2 by two fixed
odd constants, keeps both halves of the 128-bit products, and mixes them with
counter words 1 and 3 and the key; between rounds the key is advanced by two
Weyl constants (the golden ratio and sqrt(3) - 1 scaled to 2^64).

Plain Python integers are used so the arithmetic is exact and readable.
"""

_MASK64 = (1 << 64) - 1

# Round multipliers and Weyl key increments of Philox4x64 (Salmon et al.).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B


def _mulhilo(a, b):
    p = a * b
    return (p >> 64) & _MASK64, p & _MASK64


def philox4x64_10(counter, key):
    """Return the four 64-bit output words for a 4-word counter, 2-word key."""
    c0, c1, c2, c3 = (int(v) & _MASK64 for v in counter)
    k0, k1 = (int(v) & _MASK64 for v in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & _MASK64
            k1 = (k1 + PHILOX_W1) & _MASK64
        hi0, lo0 = _mulhilo(PHILOX_M0, c0)
        hi1, lo1 = _mulhilo(PHILOX_M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox_word0(j, t, ident, seed):
    """Random word of candidate ``j`` in block ``t`` of ID ``ident``."""
    return philox4x64_10((j, t, ident, 0), (seed, 0))[0]
