"""Pure-Python Philox4x32-10 -- TEST INFRASTRUCTURE ONLY.

Written from the description in Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
as easy as 1, 2, 3" (SC'11): the 4x32 Philox bijection with multipliers 0xD2511F53 and
0xCD9E8D57, key schedule bumped by 0x9E3779B9 / 0xBB67AE85 between rounds, ten rounds.
It is a third implementation beside the C oracle and the HIP device code; the tests
check all three (and rocRAND's host-callable engine) against each other.
"""
from __future__ import annotations

MASK32 = 0xFFFFFFFF
M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85

TAG_ROOT, TAG_FIRST, TAG_EDGE, TAG_EDGE_LOW, TAG_LT = 0, 1, 2, 3, 4


def philox4x32_10(ctr, key):
    x0, x1, x2, x3 = (int(c) & MASK32 for c in ctr)
    k0, k1 = (int(k) & MASK32 for k in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ k0) & MASK32, p1 & MASK32, \
                         ((p0 >> 32) ^ x3 ^ k1) & MASK32, p0 & MASK32
    return (x0, x1, x2, x3)


def draw2(seed: int, sub: int, j: int, tag: int):
    """The two 64-bit words (X = y1:y0, Y = y3:y2) of the call keyed by the sample seed
    with counter (sub, j_lo, j_hi, tag)."""
    y = philox4x32_10((sub, j & MASK32, (j >> 32) & MASK32, tag), (seed & MASK32, (seed >> 32) & MASK32))
    return (y[1] << 32) | y[0], (y[3] << 32) | y[2]


def edge_coin_word(seed: int, j: int, e: int) -> int:
    """The 64-bit coin of edge e in sample j: high half = word e & 3 of the call with counter
    (e >> 2, j, TAG_EDGE), low half = word 0 of the call with counter (e, j, TAG_EDGE_LOW)."""
    key = (seed & MASK32, (seed >> 32) & MASK32)
    jl, jh = j & MASK32, (j >> 32) & MASK32
    hi = philox4x32_10((e >> 2, jl, jh, TAG_EDGE), key)[e & 3]
    lo = philox4x32_10((e & MASK32, jl, jh, TAG_EDGE_LOW), key)[0]
    return (hi << 32) | lo
