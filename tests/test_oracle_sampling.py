"""Pins of the oracle's IIS sampler (Alg. 1, Lemma 2) against the mathematics: exact
enumeration of live-edge graphs, closed forms, textbook reverse BFS and an independent
re-derivation of each sample from its materialised live-edge graph."""
import json
import os
from collections import Counter

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order
from scipy.stats import chi2

import oracle
from oracle import philox as pyphilox
from oracle import tiny
from paper_1709_03565_amd import inputs

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _chi2_pvalue(observed: Counter, expected: dict, total: int) -> float:
    """Pearson chi-square of counts against exact probabilities, pooling cells whose
    expected count is below 5 into one."""
    stat, dof, pool_o, pool_e = 0.0, -1, 0, 0.0
    for key, p in expected.items():
        e = float(p) * total
        o = observed.get(key, 0)
        if e < 5:
            pool_o += o
            pool_e += e
            continue
        stat += (o - e) ** 2 / e
        dof += 1
    unexpected = sum(c for k, c in observed.items() if k not in expected)
    assert unexpected == 0, "sampled a set of probability zero"
    if pool_e > 0:
        stat += (pool_o - pool_e) ** 2 / max(pool_e, 1e-9)
        dof += 1
    return float(chi2.sf(stat, max(dof, 1)))


def _sets(sk):
    return [frozenset(int(x) for x in sk.sample(i)) for i in range(sk.T)]


def _graph_edges(g):
    return [(int(g.col[e]), v, float(g.w[e])) for v in range(g.n) for e in range(g.row_ptr[v], g.row_ptr[v + 1])]


def test_star_bucket_and_later_coins():
    # Root 0 with in-neighbours 1..4 (no other edges).  Eq. probn: the first live
    # neighbour is u_i with probability prod_{t<i}(1-w_t) w_i / gamma; in-neighbours after
    # it are live independently, those before it are dead.
    w = [0.3, 0.5, 0.2, 0.7]
    row_ptr = np.array([0, 4, 4, 4, 4, 4], np.int32)
    col = np.array([1, 2, 3, 4], np.int32)
    ww = np.array(w, np.float32)
    T = 400_000
    sk = oracle.build_sketch(row_ptr, col, ww, seed=7, j0=0, j1=T, nthreads=8)
    assert np.all(sk.roots == 0)
    wf = [float(np.float32(x)) for x in w]
    gamma = 1 - np.prod([1 - x for x in wf])
    expected = {}
    for mask in range(1, 16):
        A = [i for i in range(4) if mask >> i & 1]
        i0 = A[0]
        p = np.prod([1 - wf[t] for t in range(i0)]) * wf[i0] / gamma
        for t in range(i0 + 1, 4):
            p *= wf[t] if t in A else 1 - wf[t]
        expected[frozenset([0] + [a + 1 for a in A])] = p
    assert abs(sum(expected.values()) - 1) < 1e-12
    obs = Counter(_sets(sk))
    assert _chi2_pvalue(obs, expected, T) > 1e-6


def test_two_edge_star_reading_of_other_in_edges():
    # u1 -> v, u2 -> v, w = 0.5.  Buckets then independent coins for t > i give
    # P(u1 in R) = 2/3 and E[I_hat({u1})] = 0.75 * 2/3 + 1 = 1.5; coins for every t != i
    # would give 5/6 and 1.625.
    row_ptr = np.array([0, 2, 2, 2], np.int32)
    col = np.array([1, 2], np.int32)
    ww = np.array([0.5, 0.5], np.float32)
    T = 1_000_000
    sk = oracle.build_sketch(row_ptr, col, ww, seed=1, j0=0, j1=T, nthreads=8)
    has_u1 = np.array([1 in set(sk.sample(i).tolist()) for i in range(0, T, 10)])
    p = has_u1.mean()
    se = np.sqrt(2 / 9 / len(has_u1))
    gold = GOLDEN["two_edge_star"]
    assert abs(p - gold["p_u1_in_R"]) < 5 * se
    assert abs(p - gold["literal_reading_p_u1_in_R"]) > 50 * se
    _, q = oracle.row_prefix(row_ptr, ww)
    cov, est = oracle.estimate(3, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=[[1]])
    assert abs(est[0] - gold["estimate_u1"]) < 5 * 0.75 * np.sqrt(2 / 9 / T)


def test_single_edge_deterministic_estimates():
    # u -> v with weight w: every sample is {v, u}; I_hat({u}) = 1 + w, I_hat({v}) = 1.
    for w in GOLDEN["single_edge"]["weights"]:
        row_ptr = np.array([0, 0, 1], np.int32)  # node 1 = v has in-edge from node 0 = u
        col = np.array([0], np.int32)
        ww = np.array([w], np.float32)
        for T in [1, 3, 1000, 4096]:
            sk = oracle.build_sketch(row_ptr, col, ww, seed=3, j0=0, j1=T)
            assert np.all(np.diff(sk.sample_ptr) == 2)
            _, q = oracle.row_prefix(row_ptr, ww)
            cov, est = oracle.estimate(2, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=[[0], [1], [0, 1]])
            wf = float(np.float32(w))
            assert list(cov) == [T, T, T]
            assert abs(est[0] - (1 + wf)) <= 2 ** -51
            assert abs(est[1] - 1.0) <= 2 ** -51
            assert abs(est[2] - 2.0) <= 2 ** -51


def test_deterministic_weights_match_textbook_reverse_bfs():
    # w in {0, 1}: each sample is exactly the set of nodes that reach the root over
    # certain edges (the reverse BFS of Alg. 1 with every coin decided).
    rng = np.random.Generator(np.random.PCG64(21))
    n, m = 300, 900
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    keep = src != dst
    w = (rng.random(keep.sum()) < 0.4).astype(np.float32)
    row_ptr, col, ww = inputs.edges_to_in_csr(n, src[keep], dst[keep], w)
    T = 3000
    sk = oracle.build_sketch(row_ptr, col, ww, seed=5, j0=0, j1=T, nthreads=4)
    live = ww == 1.0
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    # adjacency v -> u for each certain edge u -> v (walk against edge direction)
    A = sp.csr_matrix((np.ones(live.sum()), (rows[live], col[live])), shape=(n, n))
    eligible = set(rows[live].tolist())
    for i in range(T):
        root = int(sk.roots[i])
        assert root in eligible
        want = set(breadth_first_order(A, root, directed=True, return_predecessors=False).tolist())
        assert set(sk.sample(i).tolist()) == want
    # roots uniform over nodes with a certain in-edge (all have gamma = 1)
    cnt = Counter(sk.roots.tolist())
    exp = {v: 1 / len(eligible) for v in eligible}
    assert _chi2_pvalue(cnt, exp, T) > 1e-6


def _py_prefix(row_ptr, w):
    P = np.zeros(len(w))
    for v in range(len(row_ptr) - 1):
        prod = 1.0
        for e in range(row_ptr[v], row_ptr[v + 1]):
            prod = prod * (1.0 - float(w[e]))
            P[e] = prod
    return P


def test_each_sample_is_reverse_reachability_in_its_live_edge_graph():
    # Independent re-derivation: draw the root and the first live edge from the pure
    # Python Philox, decide every edge coin, materialise the live-edge graph g_j and
    # take the reverse reachability of the root with scipy.
    g = inputs.chung_lu_graph(200, 900, 2.2, 77, "wc", cache=False)
    rng = np.random.Generator(np.random.PCG64(8))
    w = np.where(rng.random(g.m) < 0.5, g.w * 3, g.w).clip(0, 1).astype(np.float32)
    P, q = oracle.row_prefix(g.row_ptr, w)
    Pp = _py_prefix(g.row_ptr, w)
    assert np.array_equal(P, Pp)
    W, C, s = oracle.root_weights(q)
    thr, alias = oracle.alias_build(W, C)
    seed = 0x1234_5678_9ABC
    js = [0, 1, 2, 3, 999, 123456, (1 << 32) + 5] + list(range(40, 90))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    for j in js:
        sk = oracle.build_sketch(g.row_ptr, g.col, w, seed=seed, j0=j, j1=j + 1)
        X, Y = pyphilox.draw2(seed, 0, j, pyphilox.TAG_ROOT)
        b = (X * g.n) >> 64
        r = (Y * C) >> 64
        root = b if r < int(thr[b]) else int(alias[b])
        assert root == int(sk.roots[0])
        X, _ = pyphilox.draw2(seed, 0, j, pyphilox.TAG_FIRST)
        theta = float(X >> 11) * 2.0 ** -53 * (1.0 - q[root])
        a, bnd = g.row_ptr[root], g.row_ptr[root + 1]
        cand = [e for e in range(a, bnd) if 1.0 - Pp[e] > theta]
        istar = cand[0] if cand else max(e for e in range(a, bnd) if w[e] > 0)
        live = np.zeros(g.m, bool)
        for e in range(g.m):
            word = pyphilox.edge_coin_word(seed, j, e)
            live[e] = w[e] >= 1.0 or word < int(np.float64(w[e]) * 2.0 ** 64)
        live[a:istar] = False
        live[istar] = True
        A = sp.csr_matrix((np.ones(live.sum()), (rows[live], g.col[live])), shape=(g.n, g.n))
        want = set(breadth_first_order(A, root, directed=True, return_predecessors=False).tolist())
        assert set(sk.sample(0).tolist()) == want
        assert int(sk.probed[0]) == int(sum(g.row_ptr[x + 1] - g.row_ptr[x] for x in want))


@pytest.mark.parametrize("gseed", [1, 2, 3, 4])
def test_exact_iis_distribution_tiny(gseed):
    # Lemma 2: the IIS sample has P(A) = (1/Gamma) sum_v sum_{g: eta^-_g(v) = A, |A|>=2} Pr[g].
    rng = np.random.Generator(np.random.PCG64(100 + gseed))
    g = inputs.random_tiny_graph(rng, n=5, m=8)
    edges = _graph_edges(g)
    dist = tiny.exact_iis_distribution(g.n, edges)
    T = 300_000
    sk = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=gseed, j0=0, j1=T, nthreads=8)
    assert _chi2_pvalue(Counter(_sets(sk)), dist, T) > 1e-6


def test_exact_ris_distribution_tiny():
    # RIS mode (Sec. 2.3.1): uniform root, no conditioning; Eq. ris_prob.
    rng = np.random.Generator(np.random.PCG64(55))
    g = inputs.random_tiny_graph(rng, n=5, m=7)
    dist = tiny.exact_ris_distribution(g.n, _graph_edges(g))
    T = 300_000
    sk = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=9, j0=0, j1=T, nthreads=8, ris_mode=True)
    assert _chi2_pvalue(Counter(_sets(sk)), dist, T) > 1e-6


def test_ris_singular_fraction_is_one_minus_gamma_over_n():
    # Sec. 3.1: a RIS sample rooted at v is singular with probability prod(1 - w) = q_v,
    # so the singular fraction over uniform roots is 1 - Gamma/n.
    g = inputs.workload_graph("cl15k_wc")
    T = 1_000_000
    sk = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=2, j0=0, j1=T, nthreads=8, ris_mode=True)
    single = np.diff(sk.sample_ptr) == 1
    p = 1 - sk.Gamma / g.n
    assert abs(single.mean() - p) < 5 * np.sqrt(p * (1 - p) / T)
    # per-root: among samples rooted at high-degree nodes, singular frequency -> q_v
    _, q = oracle.row_prefix(g.row_ptr, g.w)
    expected_single = q[sk.roots].sum()
    var = (q[sk.roots] * (1 - q[sk.roots])).sum()
    assert abs(single.sum() - expected_single) < 5 * np.sqrt(var)


def test_invariants_and_thread_independence():
    g = inputs.workload_graph("cl15k_wc")
    T = 20000
    a = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=1, j0=0, j1=T, nthreads=1)
    b = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=1, j0=0, j1=T, nthreads=7)
    for x, y in [(a.sample_ptr, b.sample_ptr), (a.nodes, b.nodes), (a.roots, b.roots), (a.probed, b.probed)]:
        assert np.array_equal(x, y)
    # a window is the same samples
    c = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=1, j0=5000, j1=6000, nthreads=3)
    assert np.array_equal(c.nodes, a.nodes[a.sample_ptr[5000]:a.sample_ptr[6000]])
    assert np.array_equal(c.roots, a.roots[5000:6000])
    deg = np.diff(g.row_ptr)
    for i in range(T):
        R = a.sample(i)
        assert len(R) >= 2  # non-singular (Sec. 1, Alg. 1)
        assert np.all(np.diff(R) > 0)  # sorted, distinct
        assert a.roots[i] in R
        assert int(a.probed[i]) == int(deg[R].sum())
    # different seeds give different sketches
    d = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=2, j0=0, j1=1000)
    assert not np.array_equal(d.roots, a.roots[:1000])


def test_root_frequencies_follow_gamma():
    # Eq. probu: P(root = v) = gamma_v / Gamma (integer weights W_v / C).
    g = inputs.workload_graph("cl15k_wc")
    T = 1_000_000
    sk = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=4, j0=0, j1=T, nthreads=8)
    _, q = oracle.row_prefix(g.row_ptr, g.w)
    W, C, s = oracle.root_weights(q)
    # pool nodes into 50 groups of about equal mass, chi-square
    order = np.argsort(-W.astype(np.float64))
    grp = np.zeros(g.n, np.int64)
    cum = np.cumsum(W[order].astype(np.float64)) / float(C)
    grp[order] = np.minimum((cum * 50).astype(np.int64), 49)
    obs = Counter(grp[sk.roots].tolist())
    exp = Counter()
    for v in range(g.n):
        exp[int(grp[v])] += float(W[v]) / float(C)
    assert _chi2_pvalue(obs, dict(exp), T) > 1e-6
    assert np.all(W[sk.roots] > 0)


def test_validation_errors():
    ok = (np.array([0, 1, 1], np.int32), np.array([1], np.int32), np.array([0.5], np.float32))
    assert oracle.validate(*ok) == oracle.OK
    bad = [
        (np.array([0, 1, 1], np.int32), np.array([0], np.int32), np.array([0.5], np.float32)),   # self-loop
        (np.array([0, 1, 1], np.int32), np.array([2], np.int32), np.array([0.5], np.float32)),   # col out of range
        (np.array([0, 1, 1], np.int32), np.array([1], np.int32), np.array([np.nan], np.float32)),
        (np.array([0, 1, 1], np.int32), np.array([1], np.int32), np.array([1.5], np.float32)),
        (np.array([0, 1, 1], np.int32), np.array([1], np.int32), np.array([-0.1], np.float32)),
        (np.array([1, 1, 1], np.int32), np.array([1], np.int32), np.array([0.5], np.float32)),   # row_ptr[0] != 0
        (np.array([0, 2, 1], np.int32), np.array([1], np.int32), np.array([0.5], np.float32)),   # not monotone
    ]
    for b in bad:
        assert oracle.validate(*b) == oracle.EINVAL
    with pytest.raises(oracle.OracleError):
        oracle.build_sketch(*bad[0], seed=1, j0=0, j1=10)


def test_degenerate_gamma_zero():
    # No edge can be live: Gamma = 0, no non-singular sample exists; I_hat(S) = |S|.
    row_ptr = np.array([0, 1, 2, 2], np.int32)
    col = np.array([1, 2], np.int32)
    w = np.zeros(2, np.float32)
    sk = oracle.build_sketch(row_ptr, col, w, seed=1, j0=0, j1=100)
    assert sk.status == oracle.WDEGENERATE and sk.T == 0 and sk.Gamma == 0.0
    _, q = oracle.row_prefix(row_ptr, w)
    cov, est = oracle.estimate(3, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=[[0, 1], [2]])
    assert list(cov) == [0, 0] and list(est) == [2.0, 1.0]


def test_device_chung_lu_recipe_on_cpu():
    # the GPU generator of the 1.4B-edge workload, run on the CPU at a small size: exactly m
    # distinct non-loop edges, rows by (target, source), WC weights 1/d_in in fp32
    import torch
    rp, col, w = inputs.chung_lu_graph_device(3000, 30000, 2.2, 9, "wc", device="cpu")
    rp, col, w = rp.numpy(), col.numpy(), w.numpy()
    assert rp[0] == 0 and rp[-1] == 30000 and len(col) == 30000
    dst = np.repeat(np.arange(3000), np.diff(rp))
    keys = dst.astype(np.int64) * 3000 + col
    assert np.all(np.diff(keys) > 0)
    assert np.all(col != dst) and np.all((col >= 0) & (col < 3000))
    deg = np.diff(rp)
    assert np.array_equal(w, (1.0 / np.repeat(np.maximum(deg, 1), deg).astype(np.float64)).astype(np.float32))
    # heavy-tailed in-degrees, as the recipe's power-law weights give
    assert deg.max() > 20 * deg.mean()
    _, _, w2 = inputs.chung_lu_graph_device(3000, 30000, 2.2, 9, "tri", device="cpu")
    assert set(np.unique(w2.numpy()).tolist()) <= set(inputs.TRI_VALUES.tolist())
