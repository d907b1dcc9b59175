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
