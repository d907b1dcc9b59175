"""Pins of the oracle's queries: the estimator of Eq. (eq21) against exact influence
(Lemma 3) and its variance (Lemma 4), coverage against brute force, submodularity
(Lemma 8) and the greedy (Alg. 3) against a naive recompute and the (1-(1-1/k)^k)
bound of Lemma 9."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order

import oracle
from oracle import tiny
from paper_1709_03565_amd import inputs


def _edges(g):
    return [(int(g.col[e]), v, float(g.w[e])) for v in range(g.n) for e in range(g.row_ptr[v], g.row_ptr[v + 1])]


@pytest.mark.parametrize("gseed", [11, 12, 13])
def test_lemma3_identity_exact(gseed):
    # I(S) = Pr[R ∩ S != {}] * Gamma + sum_{v in S} (1 - gamma_v), exactly, for every S.
    rng = np.random.Generator(np.random.PCG64(gseed))
    g = inputs.random_tiny_graph(rng, n=5, m=7)
    edges = _edges(g)
    dist = tiny.exact_iis_distribution(g.n, edges)
    gam, Gamma = tiny.exact_gamma(g.n, edges)
    for r in range(1, g.n + 1):
        for S in itertools.combinations(range(g.n), r):
            lhs = tiny.exact_influence(g.n, edges, S)
            rhs = tiny.exact_hit_probability(dist, S) * Gamma + sum((1 - gam[v] for v in S), Fraction(0))
            assert lhs == rhs


@pytest.mark.parametrize("gseed", [21, 22])
def test_estimator_unbiased_against_exact_influence(gseed):
    # E[I_hat(S)] = I(S) (Eq. zvar); the z-test width uses Lemma 4:
    # Var[I_hat] = Gamma^2 p (1 - p) / T, p = (I(S) - sum q) / Gamma.
    rng = np.random.Generator(np.random.PCG64(gseed))
    g = inputs.random_tiny_graph(rng, n=6, m=9)
    edges = _edges(g)
    gam, Gamma = tiny.exact_gamma(g.n, edges)
    T = 200_000
    sk = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=gseed, j0=0, j1=T, nthreads=8)
    _, q = oracle.row_prefix(g.row_ptr, g.w)
    sets = [[0], [1, 2], [3, 4, 5], [0, 5], list(range(6))]
    cov, est = oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=sets)
    for S, e in zip(sets, est):
        I = float(tiny.exact_influence(g.n, edges, S))
        p = (I - float(sum(1 - gam[v] for v in S))) / float(Gamma)
        sd = float(Gamma) * math.sqrt(max(p * (1 - p), 1e-300) / T)
        assert abs(e - I) <= 5 * sd + 1e-9, (S, e, I, sd)


def _forward_influence(g, S, runs, seed):
    """Monte-Carlo forward IC simulation (Sec. 2.1, independent numpy coins)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    tot = 0
    for _ in range(runs):
        live = rng.random(g.m) < g.w
        A = sp.csr_matrix((np.ones(live.sum()), (g.col[live], rows[live])), shape=(g.n + 1, g.n + 1))
        # virtual super-source n -> S
        B = sp.csr_matrix((np.ones(len(S)), (np.full(len(S), g.n), np.array(S))), shape=(g.n + 1, g.n + 1))
        reach = breadth_first_order(A + B, g.n, directed=True, return_predecessors=False)
        tot += len(reach) - 1
    return tot / runs


def test_estimate_matches_forward_simulation_midsize():
    g = inputs.chung_lu_graph(150, 600, 2.2, 31, "wc", cache=False)
    w = np.minimum(g.w * 2, 1).astype(np.float32)
    T = 300_000
    sk = oracle.build_sketch(g.row_ptr, g.col, w, seed=3, j0=0, j1=T, nthreads=8)
    _, q = oracle.row_prefix(g.row_ptr, w)
    gg = inputs.Graph(g.n, g.m, g.row_ptr, g.col, w)
    for S in ([0, 1, 2], [int(np.argmax(np.bincount(g.col, minlength=g.n)))], list(range(0, 150, 10))):
        runs = 4000
        I_mc = _forward_influence(gg, S, runs, seed=sum(S) + 1)
        cov, est = oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=[S])
        # forward-simulation sd bounded by n/sqrt(runs)/2; SKIS sd by Gamma/sqrt(T)/2
        tol = 5 * (g.n / 2 / math.sqrt(runs) + sk.Gamma / 2 / math.sqrt(T))
        assert abs(est[0] - I_mc) < tol, (S, est[0], I_mc)


def _sketch15k(T=40000, seed=1):
    g = inputs.workload_graph("cl15k_wc")
    sk = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=seed, j0=0, j1=T, nthreads=8)
    _, q = oracle.row_prefix(g.row_ptr, g.w)
    return g, sk, q


def test_coverage_and_estimate_brute_force():
    g, sk, q = _sketch15k(T=20000)
    sets = inputs.random_sets(g.n, 40, 50, seed=7)
    sets.append(np.array([5, 5, 5, 9], np.int32))      # duplicates collapse
    sets.append(np.array(sorted(set(sk.sample(0).tolist())), np.int32))
    cov, est = oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=sets)
    samples = [set(sk.sample(i).tolist()) for i in range(sk.T)]
    for S, c, e in zip(sets, cov, est):
        Sset = set(int(x) for x in S)
        want = sum(1 for R in samples if R & Sset)
        assert int(c) == want
        exact = math.fsum([want * sk.Gamma / sk.T] + [q[v] for v in Sset])
        assert abs(e - exact) <= 4 * 2 ** -52 * abs(exact)
    # empty set
    cov, est = oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma,
                               set_ptr=np.array([0, 0], np.int64), set_nodes=np.zeros(0, np.int32))
    assert cov[0] == 0 and est[0] == 0.0
    with pytest.raises(oracle.OracleError):
        oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=[[g.n]])


def test_estimator_invariants_and_submodularity():
    g, sk, q = _sketch15k(T=20000)
    rng = np.random.Generator(np.random.PCG64(17))
    # I_hat(V) = Gamma + sum q = n up to rounding
    cov, est = oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=[np.arange(g.n)])
    assert cov[0] == sk.T and abs(est[0] - g.n) < 1e-9 * g.n
    for _ in range(30):
        B = rng.choice(g.n, size=60, replace=False)
        A = B[:30]
        x = int(rng.integers(g.n))
        sets = [A, B, np.append(A, x), np.append(B, x)]
        c, e = oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=sets)
        assert e[0] <= e[1] + 1e-9 and c[0] <= c[1]                        # monotone
        assert (c[2] - c[0]) >= (c[3] - c[1])                               # submodular coverage
        assert (e[2] - e[0]) >= (e[3] - e[1]) - 1e-9                        # submodular I_hat (Lemma 8)
        lo = math.fsum(q[np.unique(B)])
        assert lo - 1e-9 <= e[1] <= sk.Gamma + lo + 1e-9


def test_inverse_index_is_transpose():
    g, sk, q = _sketch15k(T=5000)
    node_ptr, ns = oracle.inverse(g.n, sk.sample_ptr, sk.nodes)
    assert node_ptr[-1] == len(sk.nodes)
    for v in range(0, g.n, 7):
        lst = ns[node_ptr[v]:node_ptr[v + 1]]
        assert np.all(np.diff(lst) > 0)
        for j in lst[:20]:
            assert v in set(sk.sample(int(j)).tolist())
    cnt = np.bincount(sk.nodes, minlength=g.n)
    assert np.array_equal(np.diff(node_ptr), cnt)
    # every entry: the (node, sample) pairs of the sketch, ordered by node then sample with a
    # numpy sort, are the inverse lists in order
    sizes = np.diff(np.asarray(sk.sample_ptr, np.int64))
    owner = np.repeat(np.arange(len(sizes), dtype=np.int64), sizes)
    order = np.lexsort((owner, np.asarray(sk.nodes, np.int64)))
    assert np.array_equal(np.asarray(ns, np.int64), owner[order])


def _naive_greedy(n, samples, q, Gamma, T, k):
    S = []
    covered = set()
    for _ in range(k):
        best, bg = -1, None
        for v in range(n):
            if v in S:
                continue
            d = sum(1 for j, R in enumerate(samples) if j not in covered and v in R)
            gain = (d * Gamma) / T + q[v]
            if best < 0 or gain > bg:
                best, bg = v, gain
        S.append(best)
        covered |= {j for j, R in enumerate(samples) if best in R}
    return S, len(covered)


def test_greedy_matches_naive_recompute_and_bound():
    rng = np.random.Generator(np.random.PCG64(41))
    g = inputs.random_tiny_graph(rng, n=10, m=16)
    T = 400
    sk = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=2, j0=0, j1=T)
    _, q = oracle.row_prefix(g.row_ptr, g.w)
    samples = [set(sk.sample(i).tolist()) for i in range(T)]
    for k in [1, 2, 3, 4]:
        seeds, marg, cov, est = oracle.greedy(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, k)
        nseeds, ncov = _naive_greedy(g.n, samples, q, sk.Gamma, T, k)
        assert list(seeds) == nseeds and cov == ncov
        assert int(np.sum(marg)) == cov
        c2, e2 = oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=[seeds])
        assert c2[0] == cov and e2[0] == est
        # Lemma 9: I_hat(greedy) >= (1 - (1-1/k)^k) * max over k-sets
        best = 0.0
        allsets = [list(c) for c in itertools.combinations(range(g.n), k)]
        c3, e3 = oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=allsets)
        best = float(np.max(e3))
        assert est >= (1 - (1 - 1 / k) ** k) * best - 1e-9
        assert est <= best + 1e-9


def test_greedy_midsize_properties():
    g, sk, q = _sketch15k(T=20000)
    k = 25
    seeds, marg, cov, est = oracle.greedy(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, k)
    assert len(set(seeds.tolist())) == k
    # greedy gains on a submodular function are nonincreasing in pick order
    gains = marg.astype(np.float64) * sk.Gamma / sk.T + q[seeds]
    assert np.all(np.diff(gains) <= 1e-12)
    c2, e2 = oracle.estimate(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, sets=[seeds])
    assert c2[0] == cov and abs(e2[0] - est) <= 1e-12 * est
    with pytest.raises(oracle.OracleError):
        oracle.greedy(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, 0)
    with pytest.raises(oracle.OracleError):
        oracle.greedy(g.n, sk.sample_ptr, sk.nodes, q, sk.Gamma, g.n + 1)
