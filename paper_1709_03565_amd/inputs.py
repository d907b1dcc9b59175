"""Seeded synthetic inputs: directed Chung-Lu graphs in in-CSR form, edge-probability
models and seed-set query streams.

This module holds none of the method's arithmetic; it only produces inputs.  The paper
evaluates on six SNAP / Kwak graphs (Sec. 7, Table 2) that are not available here, so
power-law Chung-Lu graphs of the stated shapes stand in for them, with the two edge
probability models of Sec. 7 ("Weight Settings"):
  * weighted cascade (WC): w(u,v) = 1 / d_in(v), computed in fp32;
  * trivalency (TRI):      w(u,v) drawn uniformly from {0.1, 0.01, 0.001} (fp32);
  * linear threshold (LT): the in-weights of v normalised and scaled by one number U_v
    uniform in [0,1) per node, w(u,v) = U_v / d_in(v) (binary64, rounded once to fp32), the
    setting of the paper's LT experiment (Sec. 7); a row's weights then sum to at most
    U_v (1 + 2^-24).

Chung-Lu recipe (directed): expected-degree weights x_i = (i+1)^(-1/(beta-1)), scaled to
sum to m, are assigned to nodes through two independent random permutations (one for
out-weights, one for in-weights).  Edges are dropped as balls: in each round B balls get
their sources from a multinomial over the out-weights and their targets from a
multinomial over the in-weights, and the targets are shuffled by a uniform random
permutation (this pairs independent draws, so every ball is an i.i.d. (source, target)
draw).  Self-loops and pairs already present are rejected; if a round yields more new
distinct pairs than are still missing, a uniform random subset of them of the missing
size is kept.  Rounds repeat until exactly m distinct edges exist.  Rows are then sorted
by (target, source).  All draws use numpy's PCG64 with the seed given.

Generated graphs are cached as .npz files under $SKIS_INPUT_CACHE (default
/tmp/skis_inputs), keyed by every parameter of the recipe.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

RECIPE_VERSION = 2


@dataclass
class Graph:
    n: int
    m: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[m], source u of edge u->v in row v
    w: np.ndarray        # float32[m]
    name: str = ""

    @property
    def indeg(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def _cache_dir() -> str:
    d = os.environ.get("SKIS_INPUT_CACHE", "/tmp/skis_inputs")
    os.makedirs(d, exist_ok=True)
    return d


def chung_lu_edges(n: int, m: int, beta: float, seed: int):
    """(src, dst) int64 arrays of m distinct directed non-loop edges, sorted by src*n+dst."""
    if m > n * (n - 1):
        raise ValueError("m exceeds the number of possible directed edges")
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (beta - 1.0))
    x *= m / x.sum()
    w_out = np.empty(n, np.float64)
    w_out[rng.permutation(n)] = x
    w_in = np.empty(n, np.float64)
    w_in[rng.permutation(n)] = x
    p_out = w_out / w_out.sum()
    p_in = w_in / w_in.sum()
    ids = np.arange(n, dtype=np.int64)
    keys = np.zeros(0, np.int64)
    while keys.size < m:
        need = m - keys.size
        B = int(need * 1.05) + 4096
        src = np.repeat(ids, rng.multinomial(B, p_out))
        dst = np.repeat(ids, rng.multinomial(B, p_in))[rng.permutation(B)]
        ok = src != dst
        cand = np.unique(src[ok] * n + dst[ok])
        del src, dst, ok
        if keys.size:
            pos = np.minimum(np.searchsorted(keys, cand), keys.size - 1)
            cand = cand[keys[pos] != cand]
        if cand.size > need:
            cand = np.sort(rng.choice(cand, size=need, replace=False))
        keys = np.concatenate([keys, cand])
        keys.sort(kind="stable")
    return keys // n, keys % n


def edges_to_in_csr(n: int, src, dst, w=None):
    """In-CSR with rows by target and, within a row, sources ascending (stable for
    repeated (u, v) pairs).  Returns (row_ptr int32[n+1], col int32[m], w or None)."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    if w is None:
        key = dst * n + src
        key.sort()
        col = (key % n).astype(np.int32)
        cnt = np.bincount(key // n, minlength=n).astype(np.int64)
        ww = None
    else:
        order = np.lexsort((src, dst))
        col = src[order].astype(np.int32)
        cnt = np.bincount(dst, minlength=n).astype(np.int64)
        ww = np.asarray(w, np.float32)[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(cnt, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("m does not fit int32 row offsets")
    return row_ptr.astype(np.int32), col, ww


def wc_weights(row_ptr) -> np.ndarray:
    """Weighted cascade: every in-edge of v gets 1/d_in(v) (fp32 division)."""
    deg = np.diff(np.asarray(row_ptr, np.int64))
    per_row = np.float32(1.0) / np.maximum(deg, 1).astype(np.float32)
    return np.repeat(per_row, deg).astype(np.float32)


TRI_VALUES = np.array([0.1, 0.01, 0.001], np.float32)


def tri_weights(m: int, seed: int) -> np.ndarray:
    """Trivalency: each edge's w uniform from {0.1, 0.01, 0.001} (fp32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return TRI_VALUES[rng.integers(0, 3, size=m)]


def lt_weights(row_ptr, seed: int) -> np.ndarray:
    """Linear threshold: w(u,v) = U_v / d_in(v), U_v uniform in [0,1) per node (PCG64)."""
    deg = np.diff(np.asarray(row_ptr, np.int64))
    rng = np.random.Generator(np.random.PCG64(seed))
    U = rng.random(len(deg))
    per_row = U / np.maximum(deg, 1).astype(np.float64)
    return np.repeat(per_row, deg).astype(np.float32)


def chung_lu_graph(n: int, m: int, beta: float, seed: int, model: str, cache: bool = True) -> Graph:
    """Directed Chung-Lu graph with WC, TRI or LT weights; weight seed = graph seed + 1000."""
    name = "cl_n%d_m%d_b%g_s%d_%s_v%d" % (n, m, beta, seed, model, RECIPE_VERSION)
    path = os.path.join(_cache_dir(), name + ".npz") if cache else None
    if path and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return Graph(n, m, z["row_ptr"], z["col"], z["w"], name)
    src, dst = chung_lu_edges(n, m, beta, seed)
    row_ptr, col, _ = edges_to_in_csr(n, src, dst)
    del src, dst
    if model == "wc":
        w = wc_weights(row_ptr)
    elif model == "tri":
        w = tri_weights(m, seed + 1000)
    elif model == "lt":
        w = lt_weights(row_ptr, seed + 1000)
    else:
        raise ValueError("unknown weight model %r" % model)
    if path:
        tmp = path + ".tmp%d.npz" % os.getpid()
        np.savez(tmp, row_ptr=row_ptr, col=col, w=w)
        os.replace(tmp, path)
    return Graph(n, m, row_ptr, col, w, name)


def chung_lu_graph_device(n: int, m: int, beta: float, seed: int, model: str, device="cuda"):
    """The Chung-Lu recipe above drawn on the GPU with torch, for graphs whose host build
    would take minutes (1.4B edges): the same expected-degree weights and node permutations,
    balls as i.i.d. (source, target) draws by inverse CDF over the cumulative weights, self-
    loops and repeated pairs rejected, a uniform random subset kept when a round yields more
    than are missing, rounds until exactly m distinct edges exist, rows by (target, source).
    torch's generators (seeded with `seed`) replace PCG64, so the graph is another draw of the
    same recipe, not the host function's graph.  The weights, permutations and cumulative sums
    are formed on the CPU: a floating-point scan on the GPU may add its partial sums in an
    order that depends on timing, and one rounding changes which node some draws land on.
    Returns (row_ptr int32[n+1], col int32[m], w fp32[m]) as device tensors."""
    import torch
    if m > n * (n - 1):
        raise ValueError("m exceeds the number of possible directed edges")
    dev = torch.device(device)
    gh = torch.Generator(device="cpu")
    gh.manual_seed(seed)
    x = torch.arange(1, n + 1, dtype=torch.float64) ** (-1.0 / (beta - 1.0))
    x *= m / x.sum()
    cdf = []
    for _ in range(2): # out-weights, then in-weights, each through its own permutation
        wv = torch.empty(n, dtype=torch.float64)
        wv[torch.randperm(n, generator=gh)] = x
        c = torch.cumsum(wv, 0)
        cdf.append((c / c[-1]).to(dev))
    del x, wv, c
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    keys = torch.zeros(0, dtype=torch.int64, device=dev)
    chunk = 1 << 27
    while keys.numel() < m:
        need = m - keys.numel()
        B = int(need * 1.05) + 4096
        parts = []
        for b0 in range(0, B, chunk):
            b = min(chunk, B - b0)
            src = torch.searchsorted(cdf[0], torch.rand(b, dtype=torch.float64, generator=g, device=dev), right=True)
            dst = torch.searchsorted(cdf[1], torch.rand(b, dtype=torch.float64, generator=g, device=dev), right=True)
            src.clamp_(max=n - 1)
            dst.clamp_(max=n - 1)
            ok = src != dst
            parts.append(torch.unique(src[ok] * n + dst[ok]))
            del src, dst, ok
        cand = torch.unique(torch.cat(parts))
        del parts
        if keys.numel():
            cand = cand[~torch.isin(cand, keys)]
        if cand.numel() > need:
            pick = torch.randperm(cand.numel(), generator=g, device=dev)[:need]
            cand = torch.sort(cand[pick]).values
        keys = torch.sort(torch.cat([keys, cand])).values
        del cand
    src = keys // n
    dst = keys % n
    del keys
    order = torch.sort(dst * n + src).values
    del src, dst
    col = (order % n).to(torch.int32)
    dsts = order // n
    del order
    deg = torch.bincount(dsts, minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    torch.cumsum(deg, 0, out=row_ptr[1:])
    if model == "wc":
        w = (1.0 / deg.clamp(min=1).to(torch.float64)).to(torch.float32)[dsts]
    elif model == "tri":
        vals = torch.tensor(TRI_VALUES, device=dev)
        w = vals[torch.randint(0, 3, (m,), generator=g, device=dev)]
    elif model == "lt":
        U = torch.rand(n, dtype=torch.float64, generator=g, device=dev)
        w = (U / deg.clamp(min=1).to(torch.float64)).to(torch.float32)[dsts]
        del U
    else:
        raise ValueError("unknown weight model %r" % model)
    del dsts, deg
    return row_ptr.to(torch.int32), col, w


def random_sets(n: int, count: int, max_size: int, seed: int):
    """`count` seed sets, sizes uniform in {1..max_size}, members uniform without
    replacement."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(1, max_size + 1, size=count)
    return [rng.choice(n, size=int(s), replace=False).astype(np.int32) for s in sizes]


def sets_to_csr(sets):
    set_ptr = np.zeros(len(sets) + 1, np.int64)
    for i, s in enumerate(sets):
        set_ptr[i + 1] = set_ptr[i] + len(s)
    flat = np.concatenate([np.asarray(s, np.int32) for s in sets]) if len(sets) else np.zeros(0, np.int32)
    return set_ptr, flat.astype(np.int32)


def zipf_sizes(count: int, a: float, lo: int, hi: int, rng) -> np.ndarray:
    """Sizes with P(k) proportional to k^-a on {lo..hi} (a truncated Zipf law)."""
    k = np.arange(lo, hi + 1, dtype=np.float64)
    p = k ** (-a)
    p /= p.sum()
    return rng.choice(k.astype(np.int64), size=count, p=p)


def serving_trace(n: int, num_queries: int, rate_per_s: float, seed: int = 11, zipf_a: float = 1.5,
                  max_size: int = 1000):
    """An open-loop query stream: arrival gaps exponential with mean 1/rate (a Poisson
    process), set sizes from a Zipf law of exponent zipf_a truncated to {1..max_size},
    members uniform over the n nodes without replacement.  Returns (set_ptr int64[Q+1],
    set_nodes int32, arrival_us float64[Q])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1e6 / rate_per_s, size=num_queries)
    arrival = np.cumsum(gaps) - gaps[0]
    sizes = zipf_sizes(num_queries, zipf_a, 1, max_size, rng)
    set_ptr = np.zeros(num_queries + 1, np.int64)
    np.cumsum(sizes, out=set_ptr[1:])
    nodes = np.empty(int(set_ptr[-1]), np.int32)
    for i, k in enumerate(sizes):
        nodes[set_ptr[i]:set_ptr[i + 1]] = rng.choice(n, size=int(k), replace=False)
    return set_ptr, nodes, arrival


def random_tiny_graph(rng, n: int, m: int, wset=None):
    """A random graph on n nodes with m distinct non-loop edges (for exact tests)."""
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    idx = rng.choice(len(pairs), size=m, replace=False)
    src = np.array([pairs[i][0] for i in idx], np.int64)
    dst = np.array([pairs[i][1] for i in idx], np.int64)
    if wset is None:
        w = rng.uniform(0.05, 0.95, size=m).astype(np.float32)
    else:
        w = np.asarray(wset, np.float32)[rng.integers(0, len(wset), size=m)]
    row_ptr, col, ww = edges_to_in_csr(n, src, dst, w)
    return Graph(n, m, row_ptr, col, ww, "tiny")


def random_tiny_lt_graph(rng, n: int, m: int, full_rows: bool = False):
    """A random graph on n nodes with m distinct non-loop edges and linear threshold weights
    that are multiples of 1/64 (so every sum is exact): row v's weights sum to at most 1, to
    exactly 1 when full_rows is set."""
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    idx = rng.choice(len(pairs), size=m, replace=False)
    src = np.array([pairs[i][0] for i in idx], np.int64)
    dst = np.array([pairs[i][1] for i in idx], np.int64)
    w = np.zeros(m, np.float32)
    for v in range(n):
        es = np.nonzero(dst == v)[0]
        if len(es) == 0:
            continue
        # d + 1 parts of 64 (the last one is the "no in-neighbour" share), each at least 1
        cuts = np.sort(rng.choice(np.arange(1, 64), size=len(es), replace=False))
        parts = np.diff(np.concatenate([[0], cuts, [64]]))
        k = parts[:-1].copy()
        if full_rows:
            k[-1] += parts[-1]
        w[es] = k.astype(np.float32) / np.float32(64)
    row_ptr, col, ww = edges_to_in_csr(n, src, dst, w)
    return Graph(n, m, row_ptr, col, ww, "tiny_lt")


# Workloads (sizes of the synthetic stand-ins).  Sample seed 1 everywhere.
WORKLOADS = {
    "cl15k_wc": dict(n=15_000, m=60_000, beta=2.3, seed=101, model="wc", T=200_000),
    "cl1m_wc": dict(n=1_000_000, m=20_000_000, beta=2.1, seed=102, model="wc", T=1 << 24),
    "cl4m_tri": dict(n=4_000_000, m=70_000_000, beta=2.0, seed=103, model="tri", T=1 << 25),
    # built on the GPU (chung_lu_graph_device); the step there is the build alone
    "cl40m_wc": dict(n=40_000_000, m=1_400_000_000, beta=2.2, seed=104, model="wc", T=1 << 26,
                     device_graph=True, build_only=True),
    # linear threshold model (Sec. 6) with the LT experiment's weights (Sec. 7)
    "cl15k_lt": dict(n=15_000, m=60_000, beta=2.3, seed=101, model="lt", T=200_000),
    "cl1m_lt": dict(n=1_000_000, m=20_000_000, beta=2.1, seed=102, model="lt", T=1 << 24),
    "cl40m_lt": dict(n=40_000_000, m=1_400_000_000, beta=2.2, seed=104, model="lt", T=1 << 26,
                     device_graph=True, build_only=True),
}
SAMPLE_SEED = 1


def workload_graph(name: str, cache: bool = True) -> Graph:
    c = WORKLOADS[name]
    return chung_lu_graph(c["n"], c["m"], c["beta"], c["seed"], c["model"], cache=cache)
