"""The serving workload at full size through the C ABI: Poisson arrivals at 50,000 queries/s,
set sizes Zipf(1.5) on 1..1000 with members uniform over the nodes of the 4M-node, 70M-edge TRI
graph, answered by the continuous-batching server against the resident 2^25-sample sketch.  Each
answer equals skis_estimate of the set alone (bit for bit: a result must not depend on the batch
it ran in), and the oracle's Eq. (eq21) on its own sketch of the same 2^25 samples (Cov exact,
I_hat within 1e-12 relative) on a spread of the queries and on the largest ones."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_1709_03565_amd import inputs

pytestmark = pytest.mark.gpu

REL = 1e-12


def _say(*a):
    print("[gpu-serve-trace]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def skis():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_03565_amd import skis as s
    s.lib()
    return s


def test_poisson_zipf_trace_on_the_tri_sketch(skis):
    name = "cl4m_tri"
    g = inputs.workload_graph(name)
    T = inputs.WORKLOADS[name]["T"]
    _say("gpu build", name, T)
    sk = skis.build_sketch(g.row_ptr, g.col, g.w, T, inputs.SAMPLE_SEED)
    Q = 3000
    set_ptr, set_nodes, arrival = inputs.serving_trace(g.n, Q, 50000.0, seed=11, zipf_a=1.5, max_size=1000)
    srv = skis.Server(sk)
    cov, est, lat = srv.replay(set_ptr, set_nodes, arrival)
    st = srv.stats()
    srv.close()
    _say("replay", st, "p50 %.1f us p99 %.1f us" % (np.percentile(lat, 50), np.percentile(lat, 99)))
    assert st["queries"] == Q and st["max_batch"] > 1
    acov, aest = (x.cpu().numpy() for x in sk.estimate(set_ptr, set_nodes))
    assert np.array_equal(cov, acov.astype(np.uint64)) and np.array_equal(est, aest)
    # the oracle's sketch of the same samples, and its estimates of 96 spread queries and the
    # 32 largest, in parallel calls
    _say("oracle build", name, T)
    prep = oracle.Prepared(g.row_ptr, g.col, g.w)
    ora = prep.sample(inputs.SAMPLE_SEED, 0, T, nthreads=16)
    q = prep.q()
    prep.close()
    sizes = np.diff(set_ptr)
    idx = np.unique(np.concatenate([np.linspace(0, Q - 1, 96).astype(np.int64), np.argsort(-sizes)[:32]]))
    chunks = np.array_split(idx, 16)

    def run(ch):
        sub = [set_nodes[set_ptr[i]:set_ptr[i + 1]] for i in ch]
        sp2, sn2 = inputs.sets_to_csr(sub)
        return oracle.estimate(g.n, ora.sample_ptr, ora.nodes, q, ora.Gamma, set_ptr=sp2, set_nodes=sn2)

    _say("oracle estimates", len(idx))
    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(run, chunks))
    ocov = np.concatenate([r[0] for r in res])
    oest = np.concatenate([r[1] for r in res])
    assert np.array_equal(cov[idx], ocov)
    assert np.all(np.abs(est[idx] - oest) <= REL * np.abs(oest))
