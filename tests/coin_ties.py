"""A graph whose edge weights force ties of the coin high halves (test infrastructure).

Edge e's coin is the 64-bit word high:low; its high half equals the high half of the
threshold floor(w * 2^64) with probability 2^-32, so a random workload almost never takes
the path that draws the low half.  Here node 0 has the in-edges e = 0..d-1 from nodes
1..d (no other node has in-edges, so every sample is rooted at 0), and each edge's weight
is chosen from the coin of one planted sample j_e: w_e = (hi + 1/2) * 2^-32, where hi is
the high half of (j_e, e)'s coin and hi < 2^23, so that w_e is a float32 and the
threshold is hi:2^31.  Sample j_e then ties on edge e and the edge is live iff the low
half is below 2^31.  The tie is reached iff e lies after the sample's first live in-edge
i*.
"""
import numpy as np

from oracle import philox as pyphilox


def coin_high_half(seed, j, e):
    key = (seed & 0xFFFFFFFF, seed >> 32)
    return pyphilox.philox4x32_10((e >> 2, j & 0xFFFFFFFF, j >> 32, pyphilox.TAG_EDGE), key)[e & 3]


def tie_star(seed, d=64, T=8192):
    """(row_ptr, col, w, planted) with planted = [(j_e, e)], one sample per edge."""
    w = np.empty(d, np.float32)
    planted = []
    for e in range(d):
        for j in range(T):
            hi = coin_high_half(seed, j, e)
            if hi < (1 << 23):
                w[e] = np.float32((hi + 0.5) * 2.0 ** -32)
                assert float(w[e]) == (hi + 0.5) * 2.0 ** -32
                planted.append((j, e))
                break
        else:
            w[e] = np.float32(1e-3)
    row_ptr = np.full(d + 2, d, np.int32)
    row_ptr[0] = 0
    col = np.arange(1, d + 1, dtype=np.int32)
    return row_ptr, col, w, planted


def first_live_edge(seed, j, P, q0):
    """i* of sample j rooted at node 0 (Eq. probn over the row's prefix products P)."""
    X, _ = pyphilox.draw2(seed, 0, j, pyphilox.TAG_FIRST)
    theta = float(X >> 11) * 2.0 ** -53 * (1.0 - q0)
    for e in range(len(P)):
        if 1.0 - P[e] > theta:
            return e
    return max(e for e in range(len(P)) if P[e] != (P[e - 1] if e else 1.0))
