"""D-SSA on SKIS sketches through the C ABI (skis_im_dssa) against the oracle's D-SSA on the
same graph, seed stream and parameters: the same iterations, sample counts, stop decision,
seeds and coverages; the estimates within 1e-12 relative."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1709_03565_amd import inputs

pytestmark = pytest.mark.gpu

REL = 1e-12


def _say(*a):
    print("[gpu-dssa]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def skis():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_03565_amd import skis as s
    s.lib()
    return s


@pytest.mark.parametrize("name,k,eps,delta", [("cl15k_wc", 1, 0.3, 0.01), ("cl15k_wc", 10, 0.3, 0.01),
                                              ("cl15k_wc", 50, 0.1, 1e-4), ("cl1m_wc", 50, 0.2, 1e-6)])
def test_dssa_matches_oracle(skis, name, k, eps, delta):
    g = inputs.workload_graph(name)
    _say(name, k, eps, delta)
    seeds, info, st = skis.im_dssa(g.row_ptr, g.col, g.w, k, eps, delta, 7)
    oseeds, oinfo = oracle.dssa(g.row_ptr, g.col, g.w, k, eps, delta, 7, nthreads=8)
    _say("gpu", info)
    _say("oracle", oinfo)
    assert st == skis.SKIS_OK
    for key in ("T", "iterations", "stopped", "cov_select", "cov_check"):
        assert info[key] == oinfo[key], key
    for key in ("Lambda", "N_max", "t_max", "Gamma"):
        assert info[key] == oinfo[key], key
    assert np.array_equal(seeds, oseeds)
    for key in ("est_select", "est_check"):
        assert abs(info[key] - oinfo[key]) <= REL * abs(oinfo[key]), key
    for key in ("eps1", "eps2", "eps3", "eps_t"):
        assert abs(info[key] - oinfo[key]) <= 1e-9, key


def test_dssa_degenerate_and_errors(skis):
    rp = np.array([0, 1, 2, 2], np.int32)
    c = np.array([1, 2], np.int32)
    seeds, info, st = skis.im_dssa(rp, c, np.zeros(2, np.float32), 2, 0.3, 0.1, 1)
    assert st == skis.SKIS_WDEGENERATE and seeds.tolist() == [0, 1] and info["est_select"] == 2.0
    g = inputs.workload_graph("cl15k_wc")
    for k, eps, delta in [(0, 0.3, 0.1), (g.n + 1, 0.3, 0.1), (5, 0.0, 0.1), (5, 0.7, 0.1), (5, 0.3, 1.0)]:
        with pytest.raises(skis.SkisError):
            skis.im_dssa(g.row_ptr, g.col, g.w, k, eps, delta, 1)
