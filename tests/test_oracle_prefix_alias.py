"""Pins of the oracle's preprocessing: prefix products and gamma_v (Eq. gamma_v,
Eq. probn), Gamma (Table 1), integer root weights and the alias table (Eq. probu)."""
import json
import math
import os
import zlib
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1709_03565_amd import inputs


def _wc_graph(degs):
    src, dst = [], []
    n = len(degs) + max(degs + [1])
    for v, d in enumerate(degs):
        for i in range(d):
            src.append(len(degs) + i)
            dst.append(v)
    row_ptr, col, _ = inputs.edges_to_in_csr(n, src, dst)
    return row_ptr, col, inputs.wc_weights(row_ptr)


def test_wc_rows_closed_form():
    # gamma_v of a WC row of in-degree d is 1 - (1 - 1/d)^d; the sequential fp64 product
    # of d exact factors has relative error at most about (d-1) * 2^-53.
    degs = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))["wc_row"]["degrees"]
    row_ptr, col, w = _wc_graph(degs)
    P, q = oracle.row_prefix(row_ptr, w)
    for v, d in enumerate(degs):
        f = 1 - Fraction(float(np.float32(1.0) / np.float32(d)))
        exact = f ** d
        rel = abs(Fraction(q[v]) - exact) / exact if exact else abs(Fraction(q[v]))
        assert rel <= (d + 1) * 2.0 ** -53, (d, float(rel))
        if d > 50:
            assert abs(q[v] - (1 - 1 / d) ** d) < 1e-6  # near e^-1 for large d
    # rows with no in-edges: q = 1, gamma = 0
    assert np.all(q[len(degs):] == 1.0)


def _rows_graph(rows):
    """A graph whose node v has the in-edge weights rows[v] (sources are fresh nodes)."""
    src, dst, ws = [], [], []
    n = len(rows) + max(len(r) for r in rows)
    for v, r in enumerate(rows):
        for i, x in enumerate(r):
            src.append(len(rows) + i)
            dst.append(v)
            ws.append(x)
    return inputs.edges_to_in_csr(n, src, dst, np.array(ws, np.float32))


def _running_product(ws):
    """P_e of a row by Python's own binary64 arithmetic: a plain loop over the factors."""
    out, run = [], 1.0
    for x in ws:
        run = run * (1.0 - float(x))
        out.append(run)
    return out


def test_prefix_rows_are_the_plain_running_product():
    # every row, short or long (up to a 1.2M-edge hub row, the size of the TRI workload's
    # largest), equals Python's left-to-right product bit for bit; compared with
    # itertools.accumulate as well on the short rows
    import itertools
    import operator
    rng = np.random.Generator(np.random.PCG64(12))
    vals = np.array([0.1, 0.01, 0.001, 0.5, 0.0, 0.999], np.float32)
    rows = [rng.choice(vals, size=d) for d in (1, 2, 17, 63, 64, 65, 257, 4097, 40000)]
    rows.append(rng.choice(np.array([0.1, 0.01, 0.001], np.float32), size=1_200_000))
    rows.append(np.full(50000, np.float32(1.0) / np.float32(50000), np.float32))
    row_ptr, col, ww = _rows_graph(rows)
    P, q = oracle.row_prefix(row_ptr, ww)
    for v in range(len(rows)):
        a, b = row_ptr[v], row_ptr[v + 1]
        want = _running_product(ww[a:b])
        assert P[a:b].tolist() == want, v
        if b - a <= 64:
            f = [1.0 - float(x) for x in ww[a:b]]
            assert want == list(itertools.accumulate(f, operator.mul))
        assert q[v] == P[b - 1]


def test_prefix_long_rows_within_rounding_bound_of_exact_products():
    # every P_e against the exact rational product of its factors: the i-th product of a
    # row (0-based) takes i roundings (the first, 1.0 times the first factor, is exact), so
    # |P_e - exact| <= i u / (1 - i u) * exact; a dropped, repeated or misplaced factor is
    # off by orders of magnitude more
    rng = np.random.Generator(np.random.PCG64(13))
    u = Fraction(1, 1 << 53)
    rows = [rng.choice(np.array([0.1, 0.01, 0.001], np.float32), size=d) for d in (65, 128, 129, 1000, 4097)]
    rows.append(np.full(300, np.float32(1.0) / np.float32(300), np.float32))
    row_ptr, col, ww = _rows_graph(rows)
    P, q = oracle.row_prefix(row_ptr, ww)
    for v in range(len(rows)):
        a, b = row_ptr[v], row_ptr[v + 1]
        exact = Fraction(1)
        for i, x in enumerate(ww[a:b]):
            exact *= 1 - Fraction(float(x))
            bound = i * u / (1 - i * u) * exact
            assert abs(Fraction(float(P[a + i])) - exact) <= bound, (v, i)
        assert q[v] == P[b - 1]


def test_prefix_special_values_and_monotone():
    rng = np.random.Generator(np.random.PCG64(3))
    n = 50
    src = rng.integers(0, n, 400)
    dst = rng.integers(0, n, 400)
    keep = src != dst
    w = rng.choice(np.array([0.0, 1.0, 0.25, 0.5, 0.001], np.float32), size=keep.sum())
    row_ptr, col, ww = inputs.edges_to_in_csr(n, src[keep], dst[keep], w)
    P, q = oracle.row_prefix(row_ptr, ww)
    for v in range(n):
        a, b = row_ptr[v], row_ptr[v + 1]
        if a == b:
            assert q[v] == 1.0
            continue
        assert q[v] == P[b - 1]
        assert np.all(np.diff(P[a:b]) <= 0)  # P nonincreasing within a row
        if np.any(ww[a:b] == 1.0):
            assert q[v] == 0.0  # any certain edge makes gamma_v = 1
        if np.all(ww[a:b] == 0.0):
            assert q[v] == 1.0


def test_gamma_total_is_exactly_rounded_sum():
    g = inputs.workload_graph("cl15k_wc")
    P, q = oracle.row_prefix(g.row_ptr, g.w)
    gam = 1.0 - q
    assert oracle.gamma_total(q) == math.fsum(gam.tolist())
    rng = np.random.Generator(np.random.PCG64(9))
    for _ in range(20):
        qq = rng.random(1000) ** rng.integers(1, 40)
        assert oracle.gamma_total(qq) == math.fsum((1.0 - qq).tolist())


def test_root_weights_definition():
    rng = np.random.Generator(np.random.PCG64(4))
    for n in [1, 2, 3, 17, 1000, 70000]:
        q = rng.random(n)
        q[rng.random(n) < 0.2] = 1.0  # some gamma = 0
        q[rng.random(n) < 0.1] = 0.0  # some gamma = 1
        W, C, s = oracle.root_weights(q)
        L = max(1, math.ceil(math.log2(max(n, 2))))
        assert s == 62 - L
        gam = 1.0 - q
        for v in range(0, n, max(1, n // 500)):
            want = math.ceil(Fraction(gam[v]) * 2 ** s)
            assert int(W[v]) == want
        assert np.all((W > 0) == (gam > 0))
        assert C == int(W.astype(object).sum())
        assert n * int(W.max()) < 2 ** 63  # alias masses n * W_v fit in 63 bits


def _alias_mass(thr, alias, C):
    n = len(thr)
    mass = [0] * n
    for b in range(n):
        mass[b] += int(thr[b])
        mass[int(alias[b])] += C - int(thr[b])
    return mass


@pytest.mark.parametrize("case", ["random", "equal", "one_heavy", "zeros", "tiny", "skewed"])
def test_alias_exact_mass(case):
    rng = np.random.Generator(np.random.PCG64(zlib.crc32(case.encode())))
    if case == "random":
        W = rng.integers(0, 1 << 40, 3000).astype(np.uint64)
    elif case == "equal":
        W = np.full(257, 12345, np.uint64)
    elif case == "one_heavy":
        W = np.ones(500, np.uint64); W[123] = 10 ** 12
    elif case == "zeros":
        W = rng.integers(0, 1 << 30, 800).astype(np.uint64); W[rng.random(800) < 0.5] = 0
    elif case == "tiny":
        W = np.array([5], np.uint64)
    else:
        W = (rng.pareto(1.1, 5000) * 1e6).astype(np.uint64) + 1
    C = int(W.astype(object).sum())
    thr, alias = oracle.alias_build(W, C)
    n = len(W)
    assert np.all(thr.astype(object) <= C)
    assert np.all((alias >= 0) & (alias < n))
    # every node owns exactly n * W_v of the n * C units
    assert _alias_mass(thr, alias, C) == [n * int(x) for x in W]


def test_alias_brute_force_small():
    # exhaustive: over all (bucket, r) with r in [0, C) the draw hits v exactly n*W_v times
    for W in ([1, 2, 3], [0, 4, 0, 4], [7], [1, 1, 1, 5], [3, 0, 0, 0, 9]):
        W = np.array(W, np.uint64)
        C = int(W.sum())
        thr, alias = oracle.alias_build(W, C)
        n = len(W)
        hits = [0] * n
        for b in range(n):
            for r in range(C):
                hits[b if r < thr[b] else int(alias[b])] += 1
        assert hits == [n * int(x) for x in W]
