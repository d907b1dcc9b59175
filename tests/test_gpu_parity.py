"""Parity of the HIP path (through the C ABI) with the CPU oracle on the same seeded
inputs: bit-exact for every integer array (prefix products and gamma included, since both
sides compute them in the same order), FP64 estimates within 1e-12 relative."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1709_03565_amd import inputs

pytestmark = pytest.mark.gpu

REL = 1e-12


def _say(*a):
    print("[gpu-parity]", *a, flush=True)
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


def _assert_tiers_add_up(inf):
    assert sum(inf.tier_samples) == inf.T
    assert sum(inf.tier_entries) == inf.entries
    assert sum(inf.tier_probed) == inf.probed_total


def _assert_sketch_equal(sk_gpu, ora, j0=0):
    sp, nodes, roots, probed = (_np(x) for x in sk_gpu.export())
    T = ora.T
    assert np.array_equal(sp[j0:j0 + T + 1] - sp[j0], ora.sample_ptr)
    assert np.array_equal(nodes[sp[j0]:sp[j0 + T]], ora.nodes)
    assert np.array_equal(roots[j0:j0 + T], ora.roots)
    assert np.array_equal(probed[j0:j0 + T].astype(np.uint64), ora.probed)


# ---------------------------------------------------------------------------------------
# a1-a3: preprocessing
# ---------------------------------------------------------------------------------------
def _special_graph(seed=3, n=400, m=3000):
    rng = np.random.Generator(np.random.PCG64(seed))
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    keep = src != dst
    vals = np.array([0.0, 1.0, 0.5, 0.25, 0.1, 0.01, 0.001, 1e-7, 0.999], np.float32)
    w = vals[rng.integers(0, len(vals), keep.sum())]
    w = np.where(rng.random(keep.sum()) < 0.5, rng.random(keep.sum()).astype(np.float32), w)
    return inputs.edges_to_in_csr(n, src[keep], dst[keep], w)


def _long_rows_graph():
    # rows on both sides of the one-thread limit (256 in-edges), of the long-row kernel's
    # chunk (4096 in-edges) and of its 16-factor chain batches, up to a 1.2M-edge row (the
    # TRI workload's largest); one row holds w = 0 and w = 1 edges
    rng = np.random.Generator(np.random.PCG64(17))
    lens = [63, 64, 65, 256, 257, 1000, 4095, 4096, 4097, 8193, 40000, 1_200_000]
    vals = np.array([1e-3, 1e-4, 1e-5, 3e-4], np.float32)  # the products stay well above 0
    src, dst, ws = [], [], []
    n = len(lens) + max(lens)
    for v, d in enumerate(lens):
        x = vals[rng.integers(0, len(vals), d)]
        if d == 1000:
            x[500] = 0.0
            x[700] = 1.0
        src.append(np.arange(len(lens), len(lens) + d))
        dst.append(np.full(d, v))
        ws.append(x)
    return inputs.edges_to_in_csr(n, np.concatenate(src), np.concatenate(dst), np.concatenate(ws))


@pytest.mark.parametrize("which", ["cl15k_wc", "special", "tri_small", "long_rows", "cl1m_wc", "cl4m_tri"])
def test_preprocess_bit_exact(skis, which):
    _say("preprocess", which)
    if which in ("cl15k_wc", "cl1m_wc", "cl4m_tri"):
        g = inputs.workload_graph(which)
        row_ptr, col, w = g.row_ptr, g.col, g.w
    elif which == "special":
        row_ptr, col, w = _special_graph()
    elif which == "long_rows":
        row_ptr, col, w = _long_rows_graph()
    else:
        g = inputs.chung_lu_graph(20000, 200000, 2.0, 9, "tri", cache=False)
        row_ptr, col, w = g.row_ptr, g.col, g.w
    out = skis.preprocess(row_ptr, col, w)
    P, q = oracle.row_prefix(row_ptr, w)
    assert np.array_equal(_np(out["P"]), P)
    assert np.array_equal(_np(out["q"]), q)
    W, C, _ = oracle.root_weights(q)
    assert np.array_equal(_np(out["W"]).astype(np.uint64), W)
    assert out["C"] == C
    assert out["Gamma"] == oracle.gamma_total(q)
    thr, alias = oracle.alias_build(W, C)
    assert np.array_equal(_np(out["thr"]).astype(np.uint64), thr)
    assert np.array_equal(_np(out["alias"]), alias)


# ---------------------------------------------------------------------------------------
# a4-a7: the sketch
# ---------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def cl15k(skis):
    g = inputs.workload_graph("cl15k_wc")
    T = inputs.WORKLOADS["cl15k_wc"]["T"]
    _say("oracle cl15k T=%d" % T)
    ora = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=1, j0=0, j1=T, nthreads=8)
    _say("gpu cl15k T=%d" % T)
    sk = skis.build_sketch(g.row_ptr, g.col, g.w, T, 1)
    return g, ora, sk


def test_sketch_bit_exact_cl15k(cl15k):
    g, ora, sk = cl15k
    inf = sk.info()
    _say("cl15k info", inf)
    assert inf.T == ora.T and inf.entries == len(ora.nodes)
    assert inf.probed_total == int(ora.probed.sum())
    assert inf.Gamma == ora.Gamma and inf.C == ora.C
    _assert_tiers_add_up(inf)
    _assert_sketch_equal(sk, ora)
    assert np.array_equal(_np(sk.q()), oracle.row_prefix(g.row_ptr, g.w)[1])


@pytest.mark.parametrize("threads,slots,visited,qpl,big_row", [
    (64, 4, 192, 2, 16384), (64, 4, 192, 1, 16384), (64, 4, 256, 2, 16384), (64, 4, 256, 1, 16384),
    (64, 2, 256, 1, 16384), (64, 3, 256, 1, 16384), (64, 2, 384, 1, 16384),
    (64, 6, 256, 2, 16384), (64, 8, 128, 2, 16384), (64, 8, 192, 2, 16384), (64, 8, 192, 1, 16384),
    (64, 8, 256, 2, 16384), (64, 12, 192, 2, 16384), (64, 16, 128, 2, 16384), (64, 16, 64, 2, 16384),
    (256, 16, 128, 2, 16384), (256, 32, 128, 2, 16384), (256, 16, 256, 2, 16384),
    (64, 8, 128, 2, 8), (256, 32, 128, 2, 8), (64, 16, 64, 2, 100), (64, 4, 192, 1, 8)])
def test_sketch_identical_across_sampler_shapes(skis, threads, slots, visited, qpl, big_row):
    # big_row = 8 sends most samples through the second tier
    g = inputs.workload_graph("cl15k_wc")
    T = 30000
    _say("shape", threads, slots, visited, big_row)
    ora = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=11, j0=0, j1=T, nthreads=8)
    sk = skis.build_sketch(g.row_ptr, g.col, g.w, T, 11, threads_per_block=threads, slots_per_block=slots,
                           visited_threshold=visited, quads_per_lane=qpl, big_row=big_row)
    inf = sk.info()
    _assert_tiers_add_up(inf)
    if big_row == 8:
        assert inf.deferred > T // 4
    _assert_sketch_equal(sk, ora)


@pytest.mark.parametrize("scale,n,m", [(2.5, 30000, 300000), (4.0, 30000, 300000), (4.0, 60000, 600000)])
def test_large_cascades_global_tier(skis, scale, n, m):
    # heavier weights give samples of thousands of nodes: LDS overflow -> the HBM hash tier;
    # at scale 4 most samples exceed the LDS sort limit (8192 nodes) and are sorted through
    # the compaction's node bitmap; on the 60k-node graph most also exceed the hash tier's
    # 6144 nodes and finish in the bitmap tier, resumed from the hash tier's handover
    g = inputs.chung_lu_graph(n, m, 2.1, 77, "wc", cache=False)
    w = np.minimum(g.w * scale, 1.0).astype(np.float32)
    T = 2000
    _say("large cascades", scale, n)
    ora = oracle.build_sketch(g.row_ptr, g.col, w, seed=5, j0=0, j1=T, nthreads=8)
    sizes = np.diff(ora.sample_ptr)
    if scale > 3:
        assert (sizes > 8192).mean() > 0.5
    else:
        assert (sizes > 256).mean() > 0.5 and sizes.max() <= 8192
    sk = skis.build_sketch(g.row_ptr, g.col, w, T, 5)
    inf = sk.info()
    _say("large cascades info", inf)
    assert inf.deferred > 0 and inf.deferred_global > 0  # samples above 1024 nodes reach the HBM tiers
    _assert_tiers_add_up(inf)
    assert inf.tier_samples[2] + inf.tier_samples[3] == inf.deferred_global
    assert inf.tier_samples[3] == inf.deferred_bitmap
    assert (inf.deferred_bitmap > 0) == bool((sizes > 6144).any())
    if n > 30000:
        assert (sizes > 6144).mean() > 0.5
    _assert_sketch_equal(sk, ora)


@pytest.mark.parametrize("which", ["cl15k", "large", "large4"])
def test_plain_form_matches_oracle_and_persistent(skis, which):
    # the one-launch-per-level form gives the same sketch, bit for bit; at weight scale 4
    # most samples exceed 8192 nodes, so the compaction's bitmap sort orders them
    if which == "cl15k":
        g = inputs.workload_graph("cl15k_wc")
        rp, c, w, T = g.row_ptr, g.col, g.w, 30000
    else:
        scale = 2.5 if which == "large" else 4.0
        g = inputs.chung_lu_graph(30000, 300000, 2.1, 77, "wc", cache=False)
        rp, c, w, T = g.row_ptr, g.col, np.minimum(g.w * scale, 1.0).astype(np.float32), 2000
    _say("plain form", which)
    ora = oracle.build_sketch(rp, c, w, seed=13, j0=0, j1=T, nthreads=8)
    if which == "large4":
        assert (np.diff(ora.sample_ptr) > 8192).mean() > 0.5
    plain = skis.build_sketch(rp, c, w, T, 13, form=1)
    assert plain.info().plain_levels > 0
    _assert_tiers_add_up(plain.info())
    _assert_sketch_equal(plain, ora)
    pers = skis.build_sketch(rp, c, w, T, 13)
    for x, y in zip(plain.export(), pers.export()):
        assert torch.equal(x, y)


@pytest.mark.parametrize("which,chunk", [("cl15k", 0), ("cl15k", 4096), ("cl15k", 1000), ("large", 300),
                                         ("large4", 700)])
def test_captured_form_matches_oracle_and_persistent(skis, which, chunk):
    # the captured chain (chunk bounds, roots, three tiers) replayed once per chunk of ids,
    # the last chunk ragged, gives the same sketch bit for bit; two builds in a row
    # instantiate and replay two graphs over the same kind of buffers
    if which == "cl15k":
        g = inputs.workload_graph("cl15k_wc")
        rp, c, w, T = g.row_ptr, g.col, g.w, 30000
    else:
        scale, gn = (2.5, 30000) if which == "large" else (4.0, 60000)
        g = inputs.chung_lu_graph(gn, 10 * gn, 2.1, 77, "wc", cache=False)
        rp, c, w, T = g.row_ptr, g.col, np.minimum(g.w * scale, 1.0).astype(np.float32), 2000
    _say("captured form", which, chunk)
    ora = oracle.build_sketch(rp, c, w, seed=13, j0=0, j1=T, nthreads=8)
    pers = skis.build_sketch(rp, c, w, T, 13)
    for rep in range(2):
        cap = skis.build_sketch(rp, c, w, T, 13, form=2, chunk_samples=chunk)
        inf = cap.info()
        _say("captured info", rep, inf)
        eff = min(chunk or (1 << 24), T)
        assert inf.graph_replays == (T + eff - 1) // eff
        _assert_tiers_add_up(inf)
        assert list(inf.tier_samples) == list(pers.info().tier_samples)
        _assert_sketch_equal(cap, ora)
        for x, y in zip(cap.export(), pers.export()):
            assert torch.equal(x, y)
        assert inf.deferred == pers.info().deferred
        assert inf.deferred_global == pers.info().deferred_global
        assert inf.deferred_bitmap == pers.info().deferred_bitmap
        if which == "large":
            assert inf.deferred_global > 0
        if which == "large4":
            assert inf.deferred_bitmap > 0


def test_tiny_and_degenerate_shapes(skis):
    cases = []
    # two-edge star, single edge, deterministic weights, multi-edges, empty rows
    cases.append((np.array([0, 2, 2, 2], np.int32), np.array([1, 2], np.int32), np.array([0.5, 0.5], np.float32)))
    cases.append((np.array([0, 0, 1], np.int32), np.array([0], np.int32), np.array([0.25], np.float32)))
    cases.append((np.array([0, 3, 3, 4, 4], np.int32), np.array([1, 1, 2, 0], np.int32),
                  np.array([0.3, 0.3, 1.0, 1.0], np.float32)))
    cases.append((np.array([0, 0, 0, 1], np.int32), np.array([0], np.int32), np.array([1.0], np.float32)))
    rng = np.random.Generator(np.random.PCG64(12))
    for _ in range(6):
        g = inputs.random_tiny_graph(rng, n=int(rng.integers(3, 9)), m=int(rng.integers(2, 12)))
        cases.append((g.row_ptr, g.col, g.w))
    for i, (rp, c, w) in enumerate(cases):
        for T in [1, 7, 1000]:
            _say("tiny case", i, "T", T)
            ora = oracle.build_sketch(rp, c, w, seed=3, j0=0, j1=T)
            sk = skis.build_sketch(rp, c, w, T, 3)
            _assert_sketch_equal(sk, ora)
            _assert_sketch_equal(skis.build_sketch(rp, c, w, T, 3, form=1), ora)
            _assert_sketch_equal(skis.build_sketch(rp, c, w, T, 3, form=2, chunk_samples=3), ora)


def test_coin_ties_of_the_high_halves(skis):
    # edge weights that put the coin threshold's high half on the coin of one planted sample
    # per edge: those samples take the low-half draw; all three forms match the oracle
    import coin_ties
    seed = 21
    rp, c, w, planted = coin_ties.tie_star(seed)
    T = 8192
    _say("coin ties", len(planted), "planted, T", T)
    ora = oracle.build_sketch(rp, c, w, seed=seed, j0=0, j1=T)
    _assert_sketch_equal(skis.build_sketch(rp, c, w, T, seed), ora)
    _assert_sketch_equal(skis.build_sketch(rp, c, w, T, seed, form=1), ora)
    _assert_sketch_equal(skis.build_sketch(rp, c, w, T, seed, form=2, chunk_samples=1000), ora)
    _assert_sketch_equal(skis.build_sketch(rp, c, w, T, seed, threads_per_block=256, slots_per_block=16,
                                           visited_threshold=128, quads_per_lane=2), ora)
    # in-degree 64 above big_row: every sample is handed on to the second tier
    sk = skis.build_sketch(rp, c, w, T, seed, big_row=8)
    assert sk.info().tier_samples[1] == T
    _assert_sketch_equal(sk, ora)


def test_staging_overflow_retry(skis):
    g = inputs.workload_graph("cl15k_wc")
    T = 20000
    ora = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=2, j0=0, j1=T, nthreads=8)
    sk = skis.build_sketch(g.row_ptr, g.col, g.w, T, 2, staging_entries=1000)
    _assert_sketch_equal(sk, ora)
    sk = skis.build_sketch(g.row_ptr, g.col, g.w, T, 2, staging_entries=1000, form=2, chunk_samples=3000)
    _assert_sketch_equal(sk, ora)


def test_deterministic_repeat(skis):
    g = inputs.workload_graph("cl15k_wc")
    a = skis.build_sketch(g.row_ptr, g.col, g.w, 50000, 9)
    b = skis.build_sketch(g.row_ptr, g.col, g.w, 50000, 9)
    for x, y in zip(a.export(), b.export()):
        assert torch.equal(x, y)
    na, sa = a.inverse()
    nb, sb = b.inverse()
    assert torch.equal(na, nb)


# ---------------------------------------------------------------------------------------
# a8-a10: inverse index, estimate, greedy
# ---------------------------------------------------------------------------------------
def test_inverse_index(cl15k):
    g, ora, sk = cl15k
    node_ptr, ns = (_np(x) for x in sk.inverse())
    onp, ons = oracle.inverse(g.n, ora.sample_ptr, ora.nodes)
    # each list H(v) ascending by sample id, as the oracle fills it
    assert np.array_equal(node_ptr, onp)
    assert np.array_equal(ns, ons)


def test_estimate_parity_config_sets(cl15k):
    g, ora, sk = cl15k
    sets = inputs.random_sets(g.n, 100, 50, seed=7)
    sets += [np.array([], np.int32), np.array([3, 3, 3, 9, 9], np.int32), np.arange(g.n, dtype=np.int32),
             np.array([g.n - 1, 0], np.int32)]
    set_ptr, set_nodes = inputs.sets_to_csr(sets)
    cov, est = sk.estimate(set_ptr, set_nodes)
    _, q = oracle.row_prefix(g.row_ptr, g.w)
    ocov, oest = oracle.estimate(g.n, ora.sample_ptr, ora.nodes, q, ora.Gamma, set_ptr=set_ptr, set_nodes=set_nodes)
    assert np.array_equal(_np(cov).astype(np.uint64), ocov)
    e = _np(est)
    assert np.all(np.abs(e - oest) <= REL * np.maximum(np.abs(oest), 1e-300)), np.max(np.abs(e - oest) / np.abs(oest))
    # repeated calls reuse cleared scratch
    cov2, est2 = sk.estimate(set_ptr, set_nodes)
    assert torch.equal(cov, cov2) and torch.equal(est, est2)


def test_estimate_heavy_sets(cl15k):
    # sets whose sample lists hold more than 32768 entries (hubs), 80 of them in one call
    g, ora, sk = cl15k
    node_ptr, _ = (_np(x) for x in sk.inverse())
    deg = np.diff(node_ptr)
    order = np.argsort(-deg, kind="stable").astype(np.int32)
    rng = np.random.Generator(np.random.PCG64(31))
    sets = [order[:k] for k in (1, 2, 3, 5, 10, 50, 300, 4096)]
    for _ in range(80):
        hub = np.concatenate([order[:2], order[rng.integers(2, 20, size=2)]])
        sets.append(np.concatenate([hub, rng.choice(g.n, 30, replace=False).astype(np.int32)]))
    heavy = sum(int(deg[np.unique(S)].sum()) > 32768 for S in sets)
    _say("heavy sets", heavy, "top deg", int(deg[order[0]]))
    assert heavy > 64
    set_ptr, set_nodes = inputs.sets_to_csr(sets)
    cov, est = sk.estimate(set_ptr, set_nodes)
    _, q = oracle.row_prefix(g.row_ptr, g.w)
    ocov, oest = oracle.estimate(g.n, ora.sample_ptr, ora.nodes, q, ora.Gamma, set_ptr=set_ptr, set_nodes=set_nodes)
    assert np.array_equal(_np(cov).astype(np.uint64), ocov)
    e = _np(est)
    assert np.all(np.abs(e - oest) <= REL * np.abs(oest))
    # the walks leave their bitmaps clear: a second call gives the same
    cov2, est2 = sk.estimate(set_ptr, set_nodes)
    assert torch.equal(cov, cov2) and torch.equal(est, est2)
    # and each set alone gives the same bits as in the batch
    for i in (0, 5, 7, 40):
        c1, e1 = sk.estimate(np.array([0, len(sets[i])]), sets[i])
        assert int(c1[0]) == int(cov[i]) and float(e1[0]) == float(est[i])


def test_greedy_parity(cl15k):
    g, ora, sk = cl15k
    _, q = oracle.row_prefix(g.row_ptr, g.w)
    for k in [1, 50]:
        seeds, marg, cov, est = sk.greedy(k)
        oseeds, omarg, ocov, oest = oracle.greedy(g.n, ora.sample_ptr, ora.nodes, q, ora.Gamma, k)
        assert np.array_equal(_np(seeds), oseeds)
        assert np.array_equal(_np(marg).astype(np.uint64), omarg)
        assert cov == ocov
        assert abs(est - oest) <= REL * abs(oest)


def test_errors_and_degenerate(skis):
    g = inputs.workload_graph("cl15k_wc")
    bad_col = g.col.copy()
    bad_col[5] = g.n
    with pytest.raises(skis.SkisError) as ei:
        skis.build_sketch(g.row_ptr, bad_col, g.w, 10, 1)
    assert ei.value.code == skis.SKIS_EINVAL
    bad_w = g.w.copy()
    bad_w[7] = np.nan
    with pytest.raises(skis.SkisError):
        skis.build_sketch(g.row_ptr, g.col, bad_w, 10, 1)
    loop = g.col.copy()
    v = int(np.argmax(np.diff(g.row_ptr) > 0))
    loop[g.row_ptr[v]] = v
    with pytest.raises(skis.SkisError):
        skis.build_sketch(g.row_ptr, loop, g.w, 10, 1)
    with pytest.raises(skis.SkisError):
        skis.build_sketch(g.row_ptr, g.col, g.w, 0, 1)
    with pytest.raises(skis.SkisError) as ei:
        skis.build_sketch(g.row_ptr, g.col, g.w, 1000, 1, max_device_bytes=1 << 16)
    assert ei.value.code == skis.SKIS_ENOMEM
    sk = skis.build_sketch(g.row_ptr, g.col, g.w, 1000, 1)
    with pytest.raises(skis.SkisError):
        sk.greedy(0)
    with pytest.raises(skis.SkisError):
        sk.greedy(g.n + 1)
    with pytest.raises(skis.SkisError):
        sk.estimate(np.array([0, 1]), np.array([g.n], np.int32))
    nb = skis.build_sketch(g.row_ptr, g.col, g.w, 1000, 1, build_inverse_index=0)
    with pytest.raises(skis.SkisError):
        nb.estimate(np.array([0, 1]), np.array([0], np.int32))
    # Gamma = 0: empty sketch, warning status, I_hat(S) = |S|
    rp = np.array([0, 1, 2, 2], np.int32)
    c = np.array([1, 2], np.int32)
    w0 = np.zeros(2, np.float32)
    d = skis.build_sketch(rp, c, w0, 100, 1)
    assert d.status == skis.SKIS_WDEGENERATE and d.info().T == 0
    cov, est = d.estimate(np.array([0, 2, 3]), np.array([0, 1, 2], np.int32))
    assert _np(cov).tolist() == [0, 0] and _np(est).tolist() == [2.0, 1.0]
    seeds, marg, cov, est = d.greedy(2)
    assert _np(seeds).tolist() == [0, 1] and cov == 0 and est == 2.0


# ---------------------------------------------------------------------------------------
# Full-size workloads (1M nodes / 20M edges / 2^24 samples, WC; 4M nodes / 70M edges / 2^25
# samples, TRI), in the launch configuration the benchmark times: the whole sketch against
# the oracle's, bit for bit, and the greedy k = 100 against the oracle's greedy
# ---------------------------------------------------------------------------------------
def _host_threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["cl1m_wc", "cl4m_tri"])
def test_full_size_against_oracle(skis, name):
    g = inputs.workload_graph(name)
    T = inputs.WORKLOADS[name]["T"]
    _say("full-size build", name, T)
    sk = skis.build_sketch(g.row_ptr, g.col, g.w, T, inputs.SAMPLE_SEED)
    inf = sk.info()
    _say("info", inf)
    _assert_tiers_add_up(inf)
    sp, nodes, roots, probed = (_np(x) for x in sk.export())
    _say("oracle sketch", name, "threads", _host_threads())
    prep = oracle.Prepared(g.row_ptr, g.col, g.w)
    ora = prep.sample(inputs.SAMPLE_SEED, 0, T, nthreads=_host_threads())
    _say("oracle entries", len(ora.nodes))
    assert inf.Gamma == ora.Gamma and inf.C == ora.C
    assert np.array_equal(sp, ora.sample_ptr)
    assert np.array_equal(nodes, ora.nodes)
    assert np.array_equal(roots, ora.roots)
    assert np.array_equal(probed.astype(np.uint64), ora.probed)
    del sp, nodes, roots, probed
    # the captured form (four replays of its chain) writes the same sketch
    cap = skis.build_sketch(g.row_ptr, g.col, g.w, T, inputs.SAMPLE_SEED, form=2, chunk_samples=T // 4 + 1,
                            build_inverse_index=0)
    _say("captured info", cap.info())
    assert cap.info().graph_replays == 4
    for x, y in zip(cap.export(), sk.export()):
        assert torch.equal(x, y)
    cap.free()
    q = prep.q()
    # estimates of a few sets against the oracle's
    sets = inputs.random_sets(g.n, 4, 30, seed=5)
    set_ptr, set_nodes = inputs.sets_to_csr(sets)
    cov, est = sk.estimate(set_ptr, set_nodes)
    ocov, oest = oracle.estimate(g.n, ora.sample_ptr, ora.nodes, q, ora.Gamma, set_ptr=set_ptr, set_nodes=set_nodes)
    assert np.array_equal(_np(cov).astype(np.uint64), ocov)
    assert np.all(np.abs(_np(est) - oest) <= REL * np.abs(oest))
    # greedy k = 100 (Alg. 3) at full size, where the first rounds each cover more than T/32
    # samples: seeds, marginals, Cov and I_hat against the oracle's greedy
    k = 100
    _say("greedy", name)
    seeds, marg, gcov, gest = sk.greedy(k)
    oseeds, omarg, ocov, oest = oracle.greedy(g.n, ora.sample_ptr, ora.nodes, q, ora.Gamma, k)
    assert np.array_equal(_np(seeds), oseeds)
    assert np.array_equal(_np(marg).astype(np.uint64), omarg)
    assert gcov == ocov and abs(gest - oest) <= REL * abs(oest)
    _say("greedy", name, "first picks", oseeds[:4].tolist(), "marg", omarg[:4].tolist())


def test_estimate_dense_list_every_lane_boundary(skis):
    # a centre node c = n - 1 with a certain edge into every other node: every sample, rooted at
    # a leaf, is {leaf, c}, so H(c) holds every sample id and a wave of the walk meets runs of
    # 32 lanes on one bitmap word.  Sets {0 .. k-1, c} start c's list at every lane of a wave
    # (their leaf lists come first), including lanes 62 and 63 and word 0 of the bitmap.
    n, T, seed = 97, 6000, 5
    rp = np.concatenate([np.arange(n, dtype=np.int32), np.array([n - 1], np.int32)])
    col = np.full(n - 1, n - 1, np.int32)
    w = np.ones(n - 1, np.float32)
    _say("dense list: star n=%d T=%d" % (n, T))
    ora = oracle.build_sketch(rp, col, w, seed=seed, j0=0, j1=T, nthreads=4)
    sk = skis.build_sketch(rp, col, w, T, seed)
    _assert_sketch_equal(sk, ora)
    sets = [np.array(list(range(k)) + [n - 1], np.int32) for k in range(0, n - 1)]
    sets += [np.array([n - 1], np.int32), np.arange(n, dtype=np.int32), np.array([0, 1, 2], np.int32)]
    set_ptr, set_nodes = inputs.sets_to_csr(sets)
    cov, est = sk.estimate(set_ptr, set_nodes)
    _, q = oracle.row_prefix(rp, w)
    ocov, oest = oracle.estimate(n, ora.sample_ptr, ora.nodes, q, ora.Gamma, set_ptr=set_ptr, set_nodes=set_nodes)
    assert np.array_equal(_np(cov).astype(np.uint64), ocov)
    assert int(ocov[0]) == T  # {c} alone covers every sample
    e = _np(est)
    assert np.all(np.abs(e - oest) <= REL * np.maximum(np.abs(oest), 1e-300))
    sk.free()
