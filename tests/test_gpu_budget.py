"""Size-budgeted sketches (Sec. 7: samples until their total size reaches h * n * log n, here
h = 5 and the natural log) through the C ABI: the sketch holds exactly the oracle's smallest
leading T samples reaching the budget, bit for bit, whatever rounds the build took, and answers
estimates from that cut; a cap below the budget keeps every sample up to the cap."""
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
    print("[gpu-budget]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def skis():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_03565_amd import skis as s
    s.lib()
    return s


@pytest.mark.parametrize("name,h", [("cl15k_wc", 5), ("cl15k_wc", 0.01)])
def test_budgeted_sketch_matches_oracle(skis, name, h):
    g = inputs.workload_graph(name)
    budget = int(math.ceil(h * g.n * math.log(g.n)))
    cap = 1 << 22
    prep = oracle.Prepared(g.row_ptr, g.col, g.w)
    T = oracle.first_T_reaching(prep, 1, budget, cap, chunk=1 << 16, nthreads=8)
    _say(name, "budget", budget, "oracle T", T)
    ora = prep.sample(1, 0, T, nthreads=8)
    assert ora.sample_ptr[-1] >= budget and (T == 1 or ora.sample_ptr[-2] < budget)
    sk = skis.build_sketch(g.row_ptr, g.col, g.w, cap, 1, entry_budget=budget)
    inf = sk.info()
    assert inf.T == T and inf.entries == ora.sample_ptr[-1] and inf.probed_total == int(ora.probed.sum())
    sp, nodes, roots, probed = (x.cpu().numpy() for x in sk.export())
    assert np.array_equal(sp, ora.sample_ptr) and np.array_equal(nodes, ora.nodes)
    assert np.array_equal(roots, ora.roots) and np.array_equal(probed.astype(np.uint64), ora.probed)
    sets = inputs.random_sets(g.n, 30, 40, seed=3)
    set_ptr, set_nodes = inputs.sets_to_csr(sets)
    cov, est = sk.estimate(set_ptr, set_nodes)
    ocov, oest = oracle.estimate(g.n, ora.sample_ptr, ora.nodes, prep.q(), ora.Gamma, set_ptr=set_ptr,
                                 set_nodes=set_nodes)
    assert np.array_equal(cov.cpu().numpy().astype(np.uint64), ocov)
    assert np.all(np.abs(est.cpu().numpy() - oest) <= REL * np.abs(oest))
    # a cap the budget is not reached under: every sample up to the cap
    small = skis.build_sketch(g.row_ptr, g.col, g.w, 1000, 1, entry_budget=10 ** 12)
    assert small.info().T == 1000
    ref = prep.sample(1, 0, 1000, nthreads=4)
    assert np.array_equal(small.export()[1].cpu().numpy(), ref.nodes)
