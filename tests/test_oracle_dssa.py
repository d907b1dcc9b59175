"""The oracle's D-SSA on IIS sketches (Sec. 5 and the appendix on D-SSA with SKIS): on a tiny
graph whose influences are known exactly the returned seeds reach (1 - 1/e - eps) OPT (the
algorithm's guarantee, which holds with probability at least 1 - delta), and on a larger graph
the run is consistent with its own definition: the seeds are the greedy on the first T samples,
the check estimate is eq21 on the next T, and a stopped run meets its coverage and error
conditions while an unstopped one reached N_max."""
import itertools
import math

import numpy as np

import oracle
from oracle import tiny
from paper_1709_03565_amd import inputs


def test_dssa_reaches_the_approximation_bound_on_exact_influences():
    src = [0, 1, 2, 0, 3, 4, 1, 5, 6, 2, 6]
    dst = [1, 2, 3, 4, 4, 5, 5, 0, 3, 6, 0]
    w = np.array([0.5, 0.3, 0.8, 0.2, 0.6, 0.4, 0.7, 0.25, 0.35, 0.45, 0.15], np.float32)
    n = 7
    row_ptr, col, ww = inputs.edges_to_in_csr(n, src, dst, w)
    edges = [(int(col[e]), v, float(ww[e])) for v in range(n) for e in range(row_ptr[v], row_ptr[v + 1])]
    eps, delta = 0.3, 0.05
    for k in (1, 2, 3):
        infl = {S: float(tiny.exact_influence(n, edges, S)) for S in itertools.combinations(range(n), k)}
        opt = max(infl.values())
        misses = 0
        for seed in range(12):
            seeds, info = oracle.dssa(row_ptr, col, ww, k, eps, delta, seed)
            assert len(set(seeds.tolist())) == k
            got = infl[tuple(sorted(int(s) for s in seeds))]
            misses += got < (1 - 1 / math.e - eps) * opt
        assert misses <= 1, (k, misses)


def test_dssa_run_matches_its_definition():
    g = inputs.workload_graph("cl15k_wc")
    prep = oracle.Prepared(g.row_ptr, g.col, g.w)
    q = prep.q()
    for k, eps, delta in [(1, 0.3, 0.01), (10, 0.3, 0.01), (25, 0.15, 0.001)]:
        seeds, info = oracle.dssa(g.row_ptr, g.col, g.w, k, eps, delta, 3, nthreads=4)
        T = info["T"]
        assert T == math.ceil(info["Lambda"]) * 2 ** (info["iterations"] - 1)
        R = prep.sample(3, 0, T, nthreads=3)
        s2, _, c2, e2 = oracle.greedy(g.n, R.sample_ptr, R.nodes, q, R.Gamma, k)
        assert np.array_equal(seeds, s2) and info["cov_select"] == c2 and info["est_select"] == e2
        if info["stopped"]:
            assert info["cov_select"] >= info["Lambda"] and info["eps_t"] <= eps
            Rc = prep.sample(3, T, 2 * T, nthreads=2)
            sp, sn = inputs.sets_to_csr([seeds])
            cc, ec = oracle.estimate(g.n, Rc.sample_ptr, Rc.nodes, q, Rc.Gamma, set_ptr=sp, set_nodes=sn)
            assert int(cc[0]) == info["cov_check"] and float(ec[0]) == info["est_check"]
            e1 = 1 - 1 / math.e
            assert abs(info["eps1"] - (info["est_select"] / info["est_check"] - 1)) < 1e-12
            assert info["eps_t"] == (info["eps1"] + info["eps2"] + info["eps1"] * info["eps2"]) * (e1 - eps) \
                + e1 * info["eps3"] or abs(info["eps_t"] - ((info["eps1"] + info["eps2"] + info["eps1"] * info["eps2"])
                                                             * (e1 - eps) + e1 * info["eps3"])) < 1e-12
        else:
            assert T >= info["N_max"]
