"""Parity at the 1.4B-edge shape (cl40m_wc: 40M nodes, 1.4B edges, WC, T = 2^26), in the
launch configuration the benchmark times: the first 2^20 sample ids and 16 random windows of
4096 ids of the GPU sketch against the CPU oracle on the same graph, bit for bit, and the
captured form's whole sketch against the eager form's.  The oracle's preprocessing of the
graph is done once and serves every id range."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1709_03565_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[full-scale]", *a, flush=True)


@pytest.mark.timeout(900)
def test_cl40m_sample_ranges_match_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_03565_amd import skis
    wl = inputs.WORKLOADS["cl40m_wc"]
    T = wl["T"]
    _say("graph n=%d m=%d" % (wl["n"], wl["m"]))
    rp, col, w = inputs.chung_lu_graph_device(wl["n"], wl["m"], wl["beta"], wl["seed"], wl["model"], "cuda")
    # the generator is reproducible: a second draw gives the same graph
    rp2, col2, w2 = inputs.chung_lu_graph_device(wl["n"], wl["m"], wl["beta"], wl["seed"], wl["model"], "cuda")
    assert torch.equal(rp, rp2) and torch.equal(col, col2) and torch.equal(w, w2)
    del rp2, col2, w2
    torch.cuda.empty_cache()
    _say("build T=%d" % T)
    sk = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED, build_inverse_index=0)
    inf = sk.info()
    _say("info", inf)
    assert sum(inf.tier_samples) == T and sum(inf.tier_entries) == inf.entries
    sp, nodes, roots, probed = sk.export()
    sk.free()
    # the captured form (4 replays of its chain over chunks of 2^24 ids) writes the same sketch
    _say("captured form")
    cap = skis.build_sketch(rp, col, w, T, inputs.SAMPLE_SEED, form=2, build_inverse_index=0)
    cinf = cap.info()
    _say("captured info", cinf)
    assert cinf.graph_replays == T >> 24 and cinf.deferred_global > 0
    for x, y in zip(cap.export(), (sp, nodes, roots, probed)):
        assert torch.equal(x, y)
    cap.free()
    hrp, hcol, hw = rp.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy()
    del rp, col, w
    torch.cuda.empty_cache()
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    _say("oracle preprocessing, %d host threads for sampling" % threads)
    prep = oracle.Prepared(hrp, hcol, hw)
    assert prep.Gamma == inf.Gamma and prep.C == inf.C
    rng = np.random.Generator(np.random.PCG64(2024))
    ranges = [(0, 1 << 20)] + [(int(s), int(s) + 4096) for s in rng.integers(1 << 20, T - 4096, 16)]
    for j0, j1 in ranges:
        _say("oracle ids", j0, j1)
        ora = prep.sample(inputs.SAMPLE_SEED, j0, j1, nthreads=threads)
        a, b = int(sp[j0]), int(sp[j1])
        assert np.array_equal((sp[j0:j1 + 1] - a).cpu().numpy(), ora.sample_ptr)
        assert np.array_equal(nodes[a:b].cpu().numpy(), ora.nodes)
        assert np.array_equal(roots[j0:j1].cpu().numpy(), ora.roots)
        assert np.array_equal(probed[j0:j1].cpu().numpy().astype(np.uint64), ora.probed)
    prep.close()
