"""RIS mode (Sec. 2.3.1) on the GPU through the C ABI: plain reverse-reachable samples with a
uniform root and independent coins on all of the root's in-edges, singular samples kept.
Bit-exact against the oracle's RIS mode (sample_ptr, nodes, roots, probed) in all three sampler
forms; the estimate n * Cov / T (Eq. ris_prob) and the greedy on gains n * Delta / T against the
oracle's with Gamma = n and no q term; the singular fraction against 1 - Gamma / n (Sec. 3.1)."""
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
    print("[gpu-ris]", *a, flush=True)
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


def _equal(sk, ora):
    sp, nodes, roots, probed = (_np(x) for x in sk.export())
    assert np.array_equal(sp, ora.sample_ptr)
    assert np.array_equal(nodes, ora.nodes)
    assert np.array_equal(roots, ora.roots)
    assert np.array_equal(probed.astype(np.uint64), ora.probed)


def test_ris_cl15k_bit_exact_all_forms(skis):
    g = inputs.workload_graph("cl15k_wc")
    T = 50000
    _say("cl15k RIS T=%d" % T)
    ora = oracle.build_sketch(g.row_ptr, g.col, g.w, seed=3, j0=0, j1=T, nthreads=8, ris_mode=True)
    sk = skis.build_sketch(g.row_ptr, g.col, g.w, T, 3, ris_mode=1)
    inf = sk.info()
    assert inf.T == T and inf.entries == len(ora.nodes)
    assert sum(inf.tier_samples) == T
    _equal(sk, ora)
    _equal(skis.build_sketch(g.row_ptr, g.col, g.w, T, 3, ris_mode=1, form=1, build_inverse_index=0), ora)
    _equal(skis.build_sketch(g.row_ptr, g.col, g.w, T, 3, ris_mode=1, form=2, chunk_samples=7000,
                             build_inverse_index=0), ora)
    _equal(skis.build_sketch(g.row_ptr, g.col, g.w, T, 3, ris_mode=1, big_row=8), ora)
    # the singular fraction (samples {root}) against its expectation 1 - Gamma / n: a binomial
    # proportion within 6 standard deviations
    sizes = np.diff(ora.sample_ptr)
    p = 1.0 - ora.Gamma / g.n
    frac = float((sizes == 1).mean())
    assert abs(frac - p) <= 6 * math.sqrt(p * (1 - p) / T), (frac, p)
    # estimates and greedy: n * Cov / T, gains n * Delta / T
    sets = inputs.random_sets(g.n, 60, 40, seed=7) + [np.array([], np.int32), np.arange(g.n, dtype=np.int32)]
    set_ptr, set_nodes = inputs.sets_to_csr(sets)
    cov, est = sk.estimate(set_ptr, set_nodes)
    zq = np.zeros(g.n)
    ocov, oest = oracle.estimate(g.n, ora.sample_ptr, ora.nodes, zq, float(g.n), set_ptr=set_ptr, set_nodes=set_nodes)
    assert np.array_equal(_np(cov).astype(np.uint64), ocov)
    assert np.all(np.abs(_np(est) - oest) <= REL * np.maximum(np.abs(oest), 1e-300))
    assert int(_np(cov)[-1]) == T and float(_np(est)[-1]) == float(g.n)  # every sample meets V
    seeds, marg, c, e = sk.greedy(20)
    oseeds, omarg, oc, oe = oracle.greedy(g.n, ora.sample_ptr, ora.nodes, zq, float(g.n), 20)
    assert np.array_equal(_np(seeds), oseeds) and np.array_equal(_np(marg).astype(np.uint64), omarg)
    assert c == oc and abs(e - oe) <= REL * abs(oe)


def test_ris_tiny_and_degenerate(skis):
    cases = [
        (np.array([0, 2, 2, 2], np.int32), np.array([1, 2], np.int32), np.array([0.5, 0.5], np.float32)),
        (np.array([0, 0, 1], np.int32), np.array([0], np.int32), np.array([0.25], np.float32)),
        (np.array([0, 3, 3, 4, 4], np.int32), np.array([1, 1, 2, 0], np.int32),
         np.array([0.3, 0.3, 1.0, 1.0], np.float32)),
        # Gamma = 0: every RIS sample is its root alone (IIS would have no sample at all)
        (np.array([0, 1, 2, 2], np.int32), np.array([1, 2], np.int32), np.zeros(2, np.float32)),
    ]
    rng = np.random.Generator(np.random.PCG64(12))
    for _ in range(4):
        g = inputs.random_tiny_graph(rng, n=int(rng.integers(3, 9)), m=int(rng.integers(2, 12)))
        cases.append((g.row_ptr, g.col, g.w))
    for i, (rp, c, w) in enumerate(cases):
        for T in (1, 7, 1000):
            _say("tiny RIS case", i, "T", T)
            ora = oracle.build_sketch(rp, c, w, seed=5, j0=0, j1=T, ris_mode=True)
            sk = skis.build_sketch(rp, c, w, T, 5, ris_mode=1)
            assert sk.status == skis.SKIS_OK
            _equal(sk, ora)
            _equal(skis.build_sketch(rp, c, w, T, 5, ris_mode=1, form=1), ora)
            _equal(skis.build_sketch(rp, c, w, T, 5, ris_mode=1, form=2, chunk_samples=3), ora)
            if not w.any():
                assert np.all(np.diff(ora.sample_ptr) == 1)
