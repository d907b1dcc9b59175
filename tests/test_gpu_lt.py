"""The linear threshold model (Sec. 6) on the GPU through the C ABI, against the oracle's LT
sampler: the running sums S, q, root weights and alias table bit for bit; every sketch (sample
sizes, nodes, roots, edges probed) bit for bit on the LT-weight workloads, on WC weights (every
row sums to 1: long walks that end on cycles, through the long-walk kernel), on paths and
cycles whose walks exceed the LDS path, and on tiny graphs; estimates, greedy, budgeted sketches
and D-SSA on LT sketches against the oracle's."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1709_03565_amd import inputs

pytestmark = pytest.mark.gpu

REL = 1e-12


def _say(*a):
    print("[gpu-lt]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def skis():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_03565_amd import skis as s
    s.lib()
    return s


def _np(t):
    return t.cpu().numpy()


def _csr(n, src, dst, w):
    return inputs.edges_to_in_csr(n, np.array(src), np.array(dst), np.array(w, np.float32))


def _equal(sk, ora):
    sp, nodes, roots, probed = (_np(x) for x in sk.export())
    assert np.array_equal(sp, ora.sample_ptr)
    assert np.array_equal(nodes, ora.nodes)
    assert np.array_equal(roots, ora.roots)
    assert np.array_equal(probed.astype(np.uint64), ora.probed)


def _long_rows_lt():
    # rows on both sides of the one-thread limit (256) and of the long-row kernel's chunk (4096)
    lens = [3, 256, 257, 4095, 4096, 4097, 20000]
    src, dst, ws = [], [], []
    n = len(lens) + max(lens)
    rng = np.random.Generator(np.random.PCG64(21))
    for v, d in enumerate(lens):
        u = rng.random()
        x = (np.full(d, u / d)).astype(np.float32)
        x[rng.integers(0, d)] = 0.0
        src.append(np.arange(len(lens), len(lens) + d))
        dst.append(np.full(d, v))
        ws.append(x)
    return inputs.edges_to_in_csr(n, np.concatenate(src), np.concatenate(dst), np.concatenate(ws))


@pytest.mark.parametrize("which", ["cl15k_lt", "cl15k_wc", "long_rows", "cl1m_lt"])
def test_lt_preprocess_bit_exact(skis, which):
    _say("preprocess", which)
    if which == "long_rows":
        row_ptr, col, w = _long_rows_lt()
    else:
        g = inputs.workload_graph(which)
        row_ptr, col, w = g.row_ptr, g.col, g.w
    out = skis.preprocess(row_ptr, col, w, model=1)
    S, q, st = oracle.row_sums_lt(row_ptr, w)
    assert st == oracle.OK
    assert np.array_equal(_np(out["P"]), S)
    assert np.array_equal(_np(out["q"]), q)
    W, C, _ = oracle.root_weights(q)
    assert np.array_equal(_np(out["W"]).astype(np.uint64), W)
    assert out["C"] == C and out["Gamma"] == oracle.gamma_total(q)
    thr, alias = oracle.alias_build(W, C)
    assert np.array_equal(_np(out["thr"]).astype(np.uint64), thr)
    assert np.array_equal(_np(out["alias"]), alias)


def test_lt_preprocess_rejects_rows_above_one(skis):
    rp, col, w = _csr(3, [1, 2], [0, 0], [0.5, 0.5 + 2.0 ** -19])
    with pytest.raises(skis.SkisError):
        skis.preprocess(rp, col, w, model=1)
    with pytest.raises(skis.SkisError):
        skis.build_sketch(rp, col, w, 10, 1, model=1)
    rp, col, w = _csr(3, [1, 2], [0, 0], [0.5, 0.5 + 2.0 ** -22])
    out = skis.preprocess(rp, col, w, model=1)
    assert float(_np(out["q"])[0]) == 0.0
    # the LT sampler has one form and no RIS mode
    g = inputs.workload_graph("cl15k_lt")
    for kw in (dict(form=1), dict(form=2), dict(ris_mode=1), dict(model=2)):
        with pytest.raises(skis.SkisError):
            skis.build_sketch(g.row_ptr, g.col, g.w, 100, 1, model=kw.pop("model", 1), **kw)


@pytest.mark.parametrize("name,T", [("cl15k_lt", 200_000), ("cl15k_wc", 50_000), ("cl1m_lt", 1 << 22)])
def test_lt_sketch_bit_exact(skis, name, T):
    g = inputs.workload_graph(name)
    _say("oracle", name, T)
    prep = oracle.Prepared(g.row_ptr, g.col, g.w, model=1)
    ora = prep.sample(1, 0, T, nthreads=8)
    _say("gpu", name, T)
    sk = skis.build_sketch(g.row_ptr, g.col, g.w, T, 1, model=1)
    inf = sk.info()
    _say(inf)
    assert inf.T == T and inf.entries == len(ora.nodes) and inf.Gamma == ora.Gamma and inf.C == ora.C
    assert inf.tier_samples[0] + inf.tier_samples[1] == T
    _equal(sk, ora)
    if name == "cl15k_wc":
        assert inf.tier_samples[1] > 0  # rows summing to 1: walks past the LDS path
    # estimates and greedy (Eq. eq21 with the LT gamma and q, Alg. 3)
    q = prep.q()
    sets = inputs.random_sets(g.n, 80, 50, seed=5) + [np.array([], np.int32)]
    set_ptr, set_nodes = inputs.sets_to_csr(sets)
    cov, est = sk.estimate(set_ptr, set_nodes)
    ocov, oest = oracle.estimate(g.n, ora.sample_ptr, ora.nodes, q, ora.Gamma, set_ptr=set_ptr,
                                 set_nodes=set_nodes)
    assert np.array_equal(_np(cov).astype(np.uint64), ocov)
    assert np.all(np.abs(_np(est) - oest) <= REL * np.maximum(np.abs(oest), 1e-300))
    k = 25
    seeds, marg, c, e = sk.greedy(k)
    oseeds, omarg, oc, oe = oracle.greedy(g.n, ora.sample_ptr, ora.nodes, q, ora.Gamma, k)
    assert np.array_equal(_np(seeds), oseeds) and np.array_equal(_np(marg).astype(np.uint64), omarg)
    assert c == oc and abs(e - oe) <= REL * abs(oe)
    prep.close()


def test_lt_walks_beyond_the_lds_path(skis):
    # a weight-1 path of 300 nodes (sample = {0..root}), weight-1 cycles of 33 and 5000 nodes
    # (sample = the cycle), and a cycle with a tail: walk lengths on both sides of 32
    cases = []
    L = 300
    cases.append(("path300", _csr(L, list(range(L - 1)), list(range(1, L)), [1.0] * (L - 1))))
    for L in (31, 32, 33, 5000):
        cases.append(("cycle%d" % L, _csr(L, list(range(L)), [(v + 1) % L for v in range(L)], [1.0] * L)))
    # a 40-cycle with a 100-node tail hanging off it (weights 1) and a half-weight branch
    src = [v for v in range(40)] + [39] + list(range(40, 139)) + [5]
    dst = [(v + 1) % 40 for v in range(40)] + [40] + list(range(41, 140)) + [140]
    w = [1.0] * 40 + [1.0] + [1.0] * 99 + [0.5]
    cases.append(("tail", _csr(141, src, dst, w)))
    for name, (rp, col, w) in cases:
        for T in (1, 64, 5000):
            _say(name, T)
            ora = oracle.build_sketch(rp, col, w, seed=3, j0=0, j1=T, nthreads=4, model=1)
            sk = skis.build_sketch(rp, col, w, T, 3, model=1)
            _equal(sk, ora)


def test_lt_tiny_graphs(skis):
    rng = np.random.Generator(np.random.PCG64(31))
    for t in range(12):
        n = int(rng.integers(2, 9))
        g = inputs.random_tiny_lt_graph(rng, n=n, m=min(int(rng.integers(1, 14)), n * (n - 1)),
                                        full_rows=bool(t % 3 == 0))
        for T in (1, 7, 3000):
            _say("tiny", t, g.n, g.m, T)
            prep = oracle.Prepared(g.row_ptr, g.col, g.w, model=1)
            if prep.C == 0:
                sk = skis.build_sketch(g.row_ptr, g.col, g.w, T, 2, model=1)
                assert sk.status == skis.SKIS_WDEGENERATE
                prep.close()
                continue
            ora = prep.sample(2, 0, T, nthreads=2)
            prep.close()
            _equal(skis.build_sketch(g.row_ptr, g.col, g.w, T, 2, model=1), ora)


def test_lt_staging_overflow_retry(skis):
    g = inputs.workload_graph("cl15k_lt")
    T = 100_000
    ora = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=4, j0=0, j1=T, nthreads=8, model=1)
    _equal(skis.build_sketch(g.row_ptr, g.col, g.w, T, 4, model=1, staging_entries=1000), ora)


def test_lt_retry_lists_large_samples_once(skis):
    # every sample of a weight-1 cycle of 1500 nodes is the cycle, above the 1024 nodes that
    # the compaction sorts in registers, so each is listed for the larger sorts; a first
    # staging of 1000 entries overflows, and the retry must list each sample once
    L = 1500
    rp, col, w = _csr(L, list(range(L)), [(v + 1) % L for v in range(L)], [1.0] * L)
    for T in (700, 3000):
        _say("retry", L, T)
        ora = oracle.build_sketch(rp, col, w, seed=5, j0=0, j1=T, nthreads=4, model=1)
        sk = skis.build_sketch(rp, col, w, T, 5, model=1, staging_entries=1000)
        _equal(sk, ora)


def test_lt_budgeted_sketch(skis):
    g = inputs.workload_graph("cl15k_lt")
    budget = int(math.ceil(2 * g.n * math.log(g.n)))
    cap = 1 << 21
    prep = oracle.Prepared(g.row_ptr, g.col, g.w, model=1)
    T = oracle.first_T_reaching(prep, 1, budget, cap, chunk=1 << 16, nthreads=8)
    _say("budget", budget, "T", T)
    ora = prep.sample(1, 0, T, nthreads=8)
    prep.close()
    sk = skis.build_sketch(g.row_ptr, g.col, g.w, cap, 1, model=1, entry_budget=budget)
    assert sk.info().T == T
    _equal(sk, ora)


@pytest.mark.parametrize("k,eps,delta", [(5, 0.3, 0.01), (40, 0.2, 1e-4)])
def test_lt_dssa_matches_oracle(skis, k, eps, delta):
    g = inputs.workload_graph("cl15k_lt")
    seeds, info, st = skis.im_dssa(g.row_ptr, g.col, g.w, k, eps, delta, 7, model=1)
    oseeds, oinfo = oracle.dssa(g.row_ptr, g.col, g.w, k, eps, delta, 7, nthreads=8, model=1)
    _say("gpu", info)
    _say("oracle", oinfo)
    assert st == skis.SKIS_OK
    for key in ("T", "iterations", "stopped", "cov_select", "cov_check", "Lambda", "N_max", "t_max", "Gamma"):
        assert info[key] == oinfo[key], key
    assert np.array_equal(seeds, oseeds)
    for key in ("est_select", "est_check"):
        assert abs(info[key] - oinfo[key]) <= REL * abs(oinfo[key]), key
