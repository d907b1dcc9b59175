"""Exact enumeration over live-edge graphs for tiny graphs -- TEST INFRASTRUCTURE ONLY.

Every probability is an exact rational (fractions.Fraction of the fp32 edge weights), so
these are the paper's definitions evaluated without rounding:
  * Pr[g] = prod_{live} w * prod_{dead} (1 - w)                       (Sec. 2.1)
  * I(S)  = sum_g |eta_g(S)| Pr[g]                                     (Sec. 2.1)
  * gamma_v = 1 - prod_{u in N_in(v)} (1 - w(u,v)), Gamma = sum gamma_v (Eq. gamma_v)
  * the IIS sample distribution: root v with probability gamma_v / Gamma, then the RIS
    sample of v conditioned on being non-singular (Lemma 2):
        P_IIS(A) = (1/Gamma) sum_v sum_{g : eta^-_g(v) = A, |A| >= 2} Pr[g]
  * the RIS sample distribution (Eq. ris_prob): P_RIS(A) = (1/n) sum_v sum_{g: eta^-_g(v)=A} Pr[g]
Only for graphs of at most ~14 edges (2^m live-edge graphs).

The linear threshold model (Sec. 6) in its live-edge form: every node v keeps at most one
in-edge, edge (u,v) with probability w(u,v) and none with probability 1 - sum_u w(u,v), all
nodes independently; gamma_v = sum_u w(u,v).  ``lt_threshold_influence_mc`` simulates the
model's own definition instead (uniform thresholds, activation once the active in-weight
reaches the threshold), which ties the live-edge form to it.
"""
from __future__ import annotations

from collections import defaultdict
from fractions import Fraction
from itertools import product

import numpy as np


def _frac(w) -> Fraction:
    return Fraction(float(np.float32(w)))


def live_edge_graphs(edges):
    """Yields (live mask tuple, Pr[g]) over all 2^m live-edge graphs."""
    ws = [_frac(w) for (_, _, w) in edges]
    for mask in product((0, 1), repeat=len(edges)):
        p = Fraction(1)
        for b, w in zip(mask, ws):
            p *= w if b else (1 - w)
            if p == 0:
                break
        if p:
            yield mask, p


def _reach(n, edges, mask, start, reverse):
    adj = [[] for _ in range(n)]
    for b, (u, v, _) in zip(mask, edges):
        if b:
            if reverse:
                adj[v].append(u)
            else:
                adj[u].append(v)
    seen = set(start)
    stack = list(start)
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return frozenset(seen)


def exact_influence(n, edges, S) -> Fraction:
    S = list(set(int(s) for s in S))
    tot = Fraction(0)
    for mask, p in live_edge_graphs(edges):
        tot += len(_reach(n, edges, mask, S, reverse=False)) * p
    return tot


def exact_gamma(n, edges):
    q = [Fraction(1)] * n
    for (u, v, w) in edges:
        q[v] *= (1 - _frac(w))
    gam = [1 - x for x in q]
    return gam, sum(gam, Fraction(0))


def exact_iis_distribution(n, edges):
    """dict frozenset(R) -> exact probability under IIS (Lemma 2)."""
    gam, Gamma = exact_gamma(n, edges)
    dist = defaultdict(Fraction)
    for mask, p in live_edge_graphs(edges):
        for v in range(n):
            A = _reach(n, edges, mask, [v], reverse=True)
            if len(A) >= 2:
                dist[A] += p / Gamma
    return dict(dist)


def exact_ris_distribution(n, edges):
    """dict frozenset(R) -> exact probability of a plain RIS sample (Eq. ris_prob)."""
    dist = defaultdict(Fraction)
    for mask, p in live_edge_graphs(edges):
        for v in range(n):
            dist[_reach(n, edges, mask, [v], reverse=True)] += p / n
    return dict(dist)


def exact_hit_probability(dist, S) -> Fraction:
    S = set(int(s) for s in S)
    return sum((p for A, p in dist.items() if A & S), Fraction(0))


# ---------------------------------------------------------------------------------------
# Linear threshold model (Sec. 6)
# ---------------------------------------------------------------------------------------

def lt_live_edge_graphs(n, edges):
    """Yields (live mask tuple, Pr[g]) over the LT live-edge graphs: each node keeps at most
    one in-edge (Sec. 6).  Requires sum_u w(u,v) <= 1 exactly for every v."""
    rows = [[] for _ in range(n)]
    for i, (_, v, _) in enumerate(edges):
        rows[v].append(i)
    options = []
    for v in range(n):
        ws = [(i, _frac(edges[i][2])) for i in rows[v]]
        none = 1 - sum((w for _, w in ws), Fraction(0))
        if none < 0:
            raise ValueError("row %d: in-weights sum above 1" % v)
        opt = [(None, none)] if none else []
        opt += [(i, w) for i, w in ws if w]
        options.append(opt)
    m = len(edges)
    for combo in product(*options):
        p = Fraction(1)
        mask = [0] * m
        for (i, w) in combo:
            p *= w
            if i is not None:
                mask[i] = 1
        if p:
            yield tuple(mask), p


def exact_lt_gamma(n, edges):
    gam = [Fraction(0)] * n
    for (u, v, w) in edges:
        gam[v] += _frac(w)
    return gam, sum(gam, Fraction(0))


def exact_lt_influence(n, edges, S) -> Fraction:
    S = list(set(int(s) for s in S))
    return sum((len(_reach(n, edges, mask, S, reverse=False)) * p for mask, p in lt_live_edge_graphs(n, edges)),
               Fraction(0))


def exact_lt_iis_distribution(n, edges):
    """dict frozenset(R) -> exact probability of an LT IIS sample (Sec. 6): root v with
    probability gamma_v / Gamma, then v's RIS sample conditioned on being non-singular."""
    _, Gamma = exact_lt_gamma(n, edges)
    dist = defaultdict(Fraction)
    for mask, p in lt_live_edge_graphs(n, edges):
        for v in range(n):
            A = _reach(n, edges, mask, [v], reverse=True)
            if len(A) >= 2:
                dist[A] += p / Gamma
    return dict(dist)


def lt_threshold_influence_mc(n, edges, S, runs: int, seed: int) -> tuple[float, float]:
    """(mean, standard error) of |activated| over runs of the threshold process: every node
    draws lambda_v uniform in [0,1]; starting from S, an inactive v turns active once the
    weights of its active in-neighbours sum to at least lambda_v; repeat until nothing
    changes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ins = [[] for _ in range(n)]
    for (u, v, w) in edges:
        ins[v].append((u, float(np.float32(w))))
    S = set(int(s) for s in S)
    tot = 0.0
    tot2 = 0.0
    for _ in range(runs):
        lam = rng.random(n)
        active = set(S)
        changed = True
        while changed:
            changed = False
            for v in range(n):
                if v in active:
                    continue
                if sum(w for (u, w) in ins[v] if u in active) >= lam[v]:
                    active.add(v)
                    changed = True
        x = float(len(active))
        tot += x
        tot2 += x * x
    mean = tot / runs
    var = max(tot2 / runs - mean * mean, 0.0)
    return mean, (var / runs) ** 0.5
