"""Pins of the oracle's linear threshold sampler (Sec. 6): gamma_v is the sum of the in-weights,
the root is drawn with probability gamma_v / Gamma, it picks exactly one in-neighbour u with
probability w(u, root) / gamma_root, and the sample then follows the model's RIS walk (the last
node added picks at most one in-neighbour, u with probability w(u, x), until it picks none or a
node already in the sample).  Checked against exact enumeration of the model's live-edge graphs,
a simulation of the model's own threshold definition, closed forms on paths and cycles, and an
independent re-derivation of every step from the pure-Python Philox."""
from collections import Counter

import numpy as np
import pytest

import oracle
from oracle import philox as pyphilox
from oracle import tiny
from paper_1709_03565_amd import inputs

from test_oracle_sampling import _chi2_pvalue, _graph_edges, _sets


def _csr(n, src, dst, w):
    rp, col, ww = inputs.edges_to_in_csr(n, np.array(src), np.array(dst), np.array(w, np.float32))
    return rp, col, ww


def test_row_sums_closed_form_and_validation():
    # rows: 0 <- {1: 1/4, 2: 1/2}, 1 <- {} , 2 <- {0: 1/8, 1: 1/8, 3: 3/4}, 3 <- {0: 1/64}
    rp, col, w = _csr(4, [1, 2, 0, 1, 3, 0], [0, 0, 2, 2, 2, 3], [0.25, 0.5, 0.125, 0.125, 0.75, 1 / 64])
    S, q, st = oracle.row_sums_lt(rp, w)
    assert st == oracle.OK
    assert S.tolist() == [0.25, 0.75, 0.125, 0.25, 1.0, 1 / 64]
    assert q.tolist() == [0.25, 1.0, 0.0, 63 / 64]
    prep = oracle.Prepared(rp, col, w, model=1)
    assert prep.Gamma == 0.75 + 1.0 + 1 / 64
    assert np.array_equal(prep.q(), q)
    prep.close()
    # a row may exceed 1 by rounding only: 1 + 2^-22 is taken (q = 0), 1 + 2^-19 is not
    for extra, ok in ((2.0 ** -22, True), (2.0 ** -19, False)):
        rp, col, w = _csr(3, [1, 2], [0, 0], [0.5, 0.5 + extra])
        _, q, st = oracle.row_sums_lt(rp, w)
        if ok:
            assert st == oracle.OK and q[0] == 0.0
            oracle.Prepared(rp, col, w, model=1).close()
        else:
            assert st == oracle.EINVAL
            with pytest.raises(oracle.OracleError):
                oracle.Prepared(rp, col, w, model=1)
    # the RIS mode is defined for the independent cascade only
    rp, col, w = _csr(3, [1, 2], [0, 0], [0.5, 0.25])
    prep = oracle.Prepared(rp, col, w, model=1)
    with pytest.raises(oracle.OracleError):
        prep.sample(1, 0, 10, ris_mode=True)
    prep.close()


@pytest.mark.parametrize("gseed,full", [(1, False), (2, False), (3, True), (4, False)])
def test_exact_lt_iis_distribution_tiny(gseed, full):
    # P(A) = (1/Gamma) sum_v sum_{g: eta^-_g(v) = A, |A| >= 2} Pr[g] over the LT live-edge graphs
    rng = np.random.Generator(np.random.PCG64(300 + gseed))
    g = inputs.random_tiny_lt_graph(rng, n=5, m=9, full_rows=full)
    edges = _graph_edges(g)
    dist = tiny.exact_lt_iis_distribution(g.n, edges)
    T = 300_000
    sk = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=gseed, j0=0, j1=T, nthreads=8, model=1)
    _, Gamma = tiny.exact_lt_gamma(g.n, edges)
    assert sk.Gamma == float(Gamma)
    assert _chi2_pvalue(Counter(_sets(sk)), dist, T) > 1e-6


@pytest.mark.parametrize("gseed", [5, 6])
def test_threshold_definition_matches_live_edge_form(gseed):
    # the model's definition (uniform thresholds, activation once the active in-weight reaches
    # the threshold) simulated directly, against the exact live-edge enumeration used above
    rng = np.random.Generator(np.random.PCG64(400 + gseed))
    g = inputs.random_tiny_lt_graph(rng, n=5, m=8)
    edges = _graph_edges(g)
    for S in ([0], [1, 3], [4]):
        exact = float(tiny.exact_lt_influence(g.n, edges, S))
        mean, se = tiny.lt_threshold_influence_mc(g.n, edges, S, runs=20_000, seed=gseed)
        assert abs(mean - exact) <= 5 * se + 1e-9, (S, mean, exact, se)


@pytest.mark.parametrize("gseed", [7, 8])
def test_lt_estimates_are_unbiased_tiny(gseed):
    # Eq. (eq21) with the LT gamma and q: Gamma * Cov / T + sum_{v in S} q_v estimates I(S)
    rng = np.random.Generator(np.random.PCG64(500 + gseed))
    g = inputs.random_tiny_lt_graph(rng, n=6, m=10)
    edges = _graph_edges(g)
    T = 200_000
    prep = oracle.Prepared(g.row_ptr, g.col, g.w, model=1)
    sk = prep.sample(gseed, 0, T, nthreads=8)
    q = prep.q()
    sets = [[0], [2, 5], [1, 3, 4], list(range(6))]
    cov, est = oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=sets)
    for S, c, e in zip(sets, cov, est):
        exact = float(tiny.exact_lt_influence(g.n, edges, S))
        p = float(c) / T
        sd = sk.Gamma * np.sqrt(max(p * (1 - p), 1.0 / T) / T)
        assert abs(e - exact) <= 5 * sd + 1e-12, (S, e, exact)
    prep.close()


def test_path_closed_form():
    # path 0 -> 1 -> ... -> L-1 with weight p on every edge: gamma_0 = 0, gamma_v = p, so the
    # root r is uniform over 1..L-1; r picks r-1, and each later node v >= 1 goes on to v-1
    # with probability p: R = {r-1-K, ..., r} with P(K >= k) = p^k for k <= r-1
    L, p = 12, 0.75
    rp, col, w = _csr(L, list(range(L - 1)), list(range(1, L)), [p] * (L - 1))
    T = 200_000
    sk = oracle.build_sketch(rp, col, w, seed=3, j0=0, j1=T, nthreads=8, model=1)
    roots = sk.roots.astype(np.int64)
    counts = np.bincount(roots, minlength=L)
    assert counts[0] == 0
    e = T / (L - 1)
    assert np.all(np.abs(counts[1:] - e) < 5 * np.sqrt(e))
    sizes = np.diff(sk.sample_ptr)
    for i in range(T):
        R = sk.sample(i)
        r = int(roots[i])
        assert R[-1] == r and np.array_equal(R, np.arange(r - len(R) + 1, r + 1))
    # mean size given the root: 2 + sum_{k=1}^{r-1} p^k
    for r in (1, 2, 5, L - 1):
        sel = sizes[roots == r]
        want = 2 + sum(p ** k for k in range(1, r))
        assert abs(sel.mean() - want) < 5 * sel.std() / np.sqrt(len(sel)) + 1e-12
    # a full path (p = 1): every sample is {0, ..., r}
    rp, col, w = _csr(L, list(range(L - 1)), list(range(1, L)), [1.0] * (L - 1))
    sk = oracle.build_sketch(rp, col, w, seed=4, j0=0, j1=5000, model=1)
    assert np.array_equal(np.diff(sk.sample_ptr), sk.roots.astype(np.int64) + 1)


def test_cycle_closed_form():
    # directed cycle with weight 1: every walk goes round and stops at the root, R = V
    L = 37
    rp, col, w = _csr(L, list(range(L)), [(v + 1) % L for v in range(L)], [1.0] * L)
    sk = oracle.build_sketch(rp, col, w, seed=5, j0=0, j1=3000, model=1)
    assert np.all(np.diff(sk.sample_ptr) == L)
    assert np.all(sk.probed == L)
    # a weight-1 cycle 2 -> 3 -> 4 -> 2 with a weight-1 tail 4 -> 5 -> 6 leaving it, and 0 -> 1 of
    # weight 1/2: every root's walk is fixed -- it ends on the cycle, or at 0 (no in-edges)
    src = [2, 3, 4, 4, 5, 0]
    dst = [3, 4, 2, 5, 6, 1]
    rp, col, w = _csr(7, src, dst, [1.0, 1.0, 1.0, 1.0, 1.0, 0.5])
    want = {1: {0, 1}, 2: {2, 3, 4}, 3: {2, 3, 4}, 4: {2, 3, 4}, 5: {2, 3, 4, 5}, 6: {2, 3, 4, 5, 6}}
    T = 60000
    sk = oracle.build_sketch(rp, col, w, seed=6, j0=0, j1=T, model=1)
    assert sk.Gamma == 5.5
    for i in range(sk.T):
        assert set(sk.sample(i).tolist()) == want[int(sk.roots[i])]
    # roots: 1 with probability 0.5 / 5.5, each of 2..6 with 1 / 5.5
    counts = np.bincount(sk.roots.astype(np.int64), minlength=7)
    for v, p in [(0, 0.0), (1, 0.5 / 5.5)] + [(v, 1 / 5.5) for v in range(2, 7)]:
        assert abs(counts[v] - p * T) <= 5 * np.sqrt(p * T) + 1e-9


def test_star_first_pick_follows_weights():
    # one root with 40 in-neighbours: the forced pick is u with probability w(u, root) / gamma
    k = 40
    rng = np.random.Generator(np.random.PCG64(9))
    ws = rng.integers(1, 6, size=k).astype(np.float64)
    ws = (ws / 256.0).astype(np.float32)  # sum <= 200/256, exact
    rp, col, w = _csr(k + 1, list(range(1, k + 1)), [0] * k, ws)
    T = 200_000
    sk = oracle.build_sketch(rp, col, w, seed=7, j0=0, j1=T, nthreads=8, model=1)
    assert np.all(sk.roots == 0) and np.all(np.diff(sk.sample_ptr) == 2)
    picked = Counter(int(sk.sample(i)[1]) for i in range(T))
    expected = {u + 1: float(ws[u]) / float(ws.sum()) for u in range(k)}
    assert _chi2_pvalue(picked, expected, T) > 1e-6


def _py_row_sums(row_ptr, w):
    S = np.zeros(len(w))
    for v in range(len(row_ptr) - 1):
        run = 0.0
        for e in range(row_ptr[v], row_ptr[v + 1]):
            run = run + float(w[e])
            S[e] = run
    return S


def test_each_sample_rederived_from_python_philox():
    # every draw redone with the pure-Python Philox and a Python running sum
    g = inputs.chung_lu_graph(300, 1500, 2.2, 78, "lt", cache=False)
    S_or, q, st = oracle.row_sums_lt(g.row_ptr, g.w)
    assert st == oracle.OK
    S = _py_row_sums(g.row_ptr, g.w)
    assert np.array_equal(S, S_or)
    W, C, _ = oracle.root_weights(q)
    thr, alias = oracle.alias_build(W, C)
    seed = 0xABCDEF12345
    rp, col, w = g.row_ptr, g.col, g.w
    js = list(range(0, 200)) + [(1 << 32) + 17, 123456789]
    for j in js:
        sk = oracle.build_sketch(rp, col, w, seed=seed, j0=j, j1=j + 1, model=1)
        X, Y = pyphilox.draw2(seed, 0, j, pyphilox.TAG_ROOT)
        b = (X * g.n) >> 64
        r = (Y * C) >> 64
        root = b if r < int(thr[b]) else int(alias[b])
        assert root == int(sk.roots[0])
        X, _ = pyphilox.draw2(seed, 0, j, pyphilox.TAG_FIRST)
        theta = float(X >> 11) * 2.0 ** -53 * (1.0 - q[root])
        a, e_end = rp[root], rp[root + 1]
        cand = [e for e in range(a, e_end) if S[e] > theta]
        e = cand[0] if cand else max(e for e in range(a, e_end) if w[e] > 0)
        R = [root]
        x = int(col[e])
        while x not in R:
            R.append(x)
            X, _ = pyphilox.draw2(seed, x, j, pyphilox.TAG_LT)
            V = float(X >> 11) * 2.0 ** -53
            cand = [f for f in range(rp[x], rp[x + 1]) if S[f] > V]
            if not cand:
                break
            x = int(col[cand[0]])
        assert sk.sample(0).tolist() == sorted(R)
        assert int(sk.probed[0]) == int(sum(rp[y + 1] - rp[y] for y in R))


def test_lt_invariants_and_thread_independence():
    g = inputs.workload_graph("cl15k_lt")
    T = 30000
    a = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=1, j0=0, j1=T, nthreads=1, model=1)
    b = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=1, j0=0, j1=T, nthreads=6, model=1)
    for x, y in [(a.sample_ptr, b.sample_ptr), (a.nodes, b.nodes), (a.roots, b.roots), (a.probed, b.probed)]:
        assert np.array_equal(x, y)
    c = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=1, j0=7000, j1=9000, nthreads=3, model=1)
    assert np.array_equal(c.nodes, a.nodes[a.sample_ptr[7000]:a.sample_ptr[9000]])
    deg = np.diff(g.row_ptr)
    for i in range(T):
        R = a.sample(i)
        assert len(R) >= 2 and np.all(np.diff(R) > 0) and a.roots[i] in R
        assert int(a.probed[i]) == int(deg[R].sum())
    # the walk's length: each added node continues with probability gamma_x, here about 1/2
    assert 2.0 < np.diff(a.sample_ptr).mean() < 6.0
    # the IC sampler on the same graph is another distribution
    ic = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=1, j0=0, j1=T, nthreads=6)
    assert ic.Gamma != a.Gamma or not np.array_equal(ic.nodes, a.nodes)
