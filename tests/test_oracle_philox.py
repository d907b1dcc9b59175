"""Pins of the canonical Philox4x32-10 stream (Salmon et al., SC'11): the pure-Python and
C oracle implementations agree with each other and with rocRAND's host-callable engine,
an implementation this project did not write."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from oracle import philox as pyphilox


def _vectors(count, seed, c1_max=(1 << 30) - 1):
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.integers(0, 1 << 32, size=(count, 6), dtype=np.uint64)
    v[:, 1] %= (c1_max + 1)
    # structured corners: zero counter/key, all-ones words, small counters
    extra = np.array([[0, 0, 0, 0, 0, 0],
                      [0xFFFFFFFF, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF],
                      [1, 0, 0, 2, 1, 0],
                      [7, 5, 0, 1, 1, 0]], np.uint64)
    return np.concatenate([extra, v])


def test_python_matches_c_oracle():
    for row in _vectors(3000, 11, c1_max=0xFFFFFFFF):
        ctr, key = [int(x) for x in row[:4]], [int(x) for x in row[4:]]
        assert tuple(int(x) for x in oracle.philox4x32_10(ctr, key)) == pyphilox.philox4x32_10(ctr, key)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_matches_rocrand_engine():
    vec = _vectors(2000, 12)
    src = os.path.join(os.path.dirname(__file__), "rocrand_philox_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "chk")
        subprocess.run(["hipcc", "-O1", "-o", exe, src], check=True, capture_output=True)
        inp = "\n".join(" ".join(str(int(x)) for x in r) for r in vec) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    got = [tuple(int(t) for t in line.split()) for line in out.strip().splitlines()]
    assert len(got) == len(vec)
    for row, g in zip(vec, got):
        ctr, key = [int(x) for x in row[:4]], [int(x) for x in row[4:]]
        assert pyphilox.philox4x32_10(ctr, key) == g
        assert tuple(int(x) for x in oracle.philox4x32_10(ctr, key)) == g


def test_output_words_look_uniform():
    # 2^14 calls -> 65536 words; byte histogram chi-square (255 dof) and bit balance.
    words = []
    for i in range(1 << 14):
        words.extend(oracle.philox4x32_10([i, 3, 0, 2], [1, 0]))
    w = np.array(words, np.uint32)
    b = np.frombuffer(w.tobytes(), np.uint8)
    h = np.bincount(b, minlength=256)
    e = len(b) / 256
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 255 + 6 * np.sqrt(2 * 255)
    bits = np.unpackbits(b).mean()
    assert abs(bits - 0.5) < 5 * 0.5 / np.sqrt(len(b) * 8)


def test_edge_coin_definition():
    # live iff w >= 1 or the 64-bit coin (high half: word e & 3 of the tag-2 call at e >> 2;
    # low half: word 0 of the tag-3 call at e) < floor(w * 2^64)
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(500):
        seed, j, e = int(rng.integers(0, 1 << 40)), int(rng.integers(0, 1 << 33)), int(rng.integers(0, 1 << 31))
        w = float(np.float32(rng.choice([0.0, 1.0, rng.random(), 1e-9, 0.5])))
        word = pyphilox.edge_coin_word(seed, j, e)
        want = w >= 1.0 or word < int(np.float64(w) * 2.0 ** 64)
        assert oracle.edge_coin(seed, j, e, w) == want
    # P(live) = w: frequency over many (j, e) for w = 0.3
    hits = sum(oracle.edge_coin(1, j, 0, 0.3) for j in range(40000))
    p = float(np.float32(0.3))
    assert abs(hits / 40000 - p) < 5 * np.sqrt(p * (1 - p) / 40000)


@pytest.mark.parametrize("w", [0.01, 0.1, 1.0 / 7.0, 1.0 / 3.0, 0.5, 0.9, 0.999])
def test_edge_coin_frequency_is_w(w):
    # P(live) = w for each of the four words of a Philox call (e mod 4) and for low and high
    # edge indices, over independent sample ids
    p = float(np.float32(w))
    N = 6000
    for e in (0, 1, 2, 3, 4097, (1 << 30) + 2):
        hits = sum(oracle.edge_coin(7, j, e, p) for j in range(N))
        assert abs(hits / N - p) < 5 * np.sqrt(p * (1 - p) / N), (w, e, hits)


def test_edge_coin_high_words_share_one_call():
    # four consecutive edges 4c..4c+3 take their high halves from the four words of one call
    seed, j = 0x1234_5678_9ABC, 77
    for c in (0, 1, 12345, (1 << 29) - 1):
        y = pyphilox.philox4x32_10((c, j, 0, pyphilox.TAG_EDGE), (seed & 0xFFFFFFFF, seed >> 32))
        for h in range(4):
            assert pyphilox.edge_coin_word(seed, j, 4 * c + h) >> 32 == y[h]


def _tie_cases(seed, e, count):
    # sample ids whose coin high half is below 2^23, so that a float32 w puts the threshold's
    # high half exactly on it with a non-zero low half
    out = []
    j = 0
    while len(out) < count:
        hi = pyphilox.edge_coin_word(seed, j, e) >> 32
        if hi < (1 << 23):
            out.append((j, hi))
        j += 1
    return out


def test_edge_coin_tie_of_high_halves_decided_by_low_half():
    # w = (hi + 1/2) * 2^-32 is a float32 for hi < 2^23 and floor(w * 2^64) = hi:2^31, so the
    # high halves tie and the edge is live iff the low half is below 2^31
    seed = 99
    live_seen = set()
    for e in (0, 3, 6, 1001):
        for j, hi in _tie_cases(seed, e, 4):
            w = np.float32((hi + 0.5) * 2.0 ** -32)
            assert float(w) == (hi + 0.5) * 2.0 ** -32
            thr = int(np.float64(w) * 2.0 ** 64)
            assert thr >> 32 == hi and thr & 0xFFFFFFFF == 1 << 31
            lo = pyphilox.edge_coin_word(seed, j, e) & 0xFFFFFFFF
            got = oracle.edge_coin(seed, j, e, float(w))
            assert got == (lo < (1 << 31))
            live_seen.add(got)
            # the threshold's low half at zero: a tie of the high halves is never live
            w0 = np.float32(hi * 2.0 ** -32)
            if int(np.float64(w0) * 2.0 ** 64) == hi << 32:
                assert not oracle.edge_coin(seed, j, e, float(w0))
            # one more than the tie in the high half: always live
            w1 = np.float32((hi + 1) * 2.0 ** -32)
            if int(np.float64(w1) * 2.0 ** 64) >> 32 == hi + 1:
                assert oracle.edge_coin(seed, j, e, float(w1))
    assert live_seen == {False, True}


def test_planted_coin_ties_reach_the_oracle_both_ways():
    # the tie graph used by the GPU parity test: the planted ties that lie after i* are
    # decided by the low half (live iff below 2^31), and both outcomes occur
    import coin_ties
    seed = 21
    row_ptr, col, w, planted = coin_ties.tie_star(seed)
    assert len(planted) == 64
    P, q = oracle.row_prefix(row_ptr, w)
    T = max(j for j, _ in planted) + 1
    sk = oracle.build_sketch(row_ptr, col, w, seed=seed, j0=0, j1=T)
    outcomes = []
    for j, e in planted:
        istar = coin_ties.first_live_edge(seed, j, P[:row_ptr[1]], q[0])
        members = set(sk.sample(j).tolist())
        if e > istar:
            lo = pyphilox.edge_coin_word(seed, j, e) & 0xFFFFFFFF
            assert ((e + 1) in members) == (lo < (1 << 31))
            outcomes.append(lo < (1 << 31))
    assert len(outcomes) >= 10 and 0 < sum(outcomes) < len(outcomes)
