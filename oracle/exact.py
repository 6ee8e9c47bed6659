"""Exact (un-sampled) quantities of the Panther model, in rational arithmetic.

TEST INFRASTRUCTURE: used only to pin the sampling oracle on tiny graphs.

* ``path_distribution`` enumerates every T-path (Sec. 3.1) with its exact
  sampling probability: a uniform start over the start set times the product
  of transition probabilities t_ij = w_ij / sum_k w_ik (Eq. 3).  This is
  phi(p) = w(p) / sum_{p in Pi} w(p) of Sec. 3.2, since each start's
  outgoing path weights sum to one.
* ``exact_similarity`` evaluates Eq. 1, S_RP(i, j) = phi(P_ij), by summing
  the enumeration.
* ``avoid_prob`` / ``similarity_by_avoidance`` compute the same quantity a
  second, independent way: A(X) = Pr[path avoids every vertex of X] by a
  T-step dynamic programme restricted to V \\ X, and inclusion-exclusion
  S(i, j) = 1 - A({i}) - A({j}) + A({i, j}).
* ``sample_size`` restates Theorem 1 with Lemma 1's VC bound.
"""
from __future__ import annotations

import math
from fractions import Fraction
from itertools import product


def _adj(g):
    rp = [int(x) for x in g.row_ptr]
    col = [int(x) for x in g.col]
    w = [int(x) for x in g.w]
    rows = []
    for v in range(g.n):
        rows.append([(col[e], w[e]) for e in range(rp[v], rp[v + 1])])
    return rows


def start_set(g, start_all=False):
    rows = _adj(g)
    return [v for v in range(g.n) if start_all or sum(w for _, w in rows[v]) > 0]


def transition(g):
    """t[v] = list of (u, Fraction t_vu) for edges of positive weight."""
    rows = _adj(g)
    t = []
    for v in range(g.n):
        tot = sum(w for _, w in rows[v])
        acc = {}
        if tot > 0:
            for u, w in rows[v]:
                if w > 0:
                    acc[u] = acc.get(u, Fraction(0)) + Fraction(w, tot)
        t.append(sorted(acc.items()))
    return t


def path_distribution(g, T, start_all=False):
    """dict path-tuple -> exact probability."""
    t = transition(g)
    starts = start_set(g, start_all)
    p0 = Fraction(1, len(starts))
    dist = {}

    def rec(path, prob):
        if len(path) == T + 1:
            dist[tuple(path)] = dist.get(tuple(path), Fraction(0)) + prob
            return
        v = path[-1]
        if not t[v]:  # zero-weight row (start_all form): the walk stays
            rec(path + [v], prob)
            return
        for u, tp in t[v]:
            rec(path + [u], prob * tp)

    for s in starts:
        rec([s], p0)
    return dist


def exact_similarity(g, T, i, j, dist=None):
    """Eq. 1: total probability of the T-paths containing both i and j."""
    if dist is None:
        dist = path_distribution(g, T)
    return sum((p for path, p in dist.items() if i in path and j in path), Fraction(0))


def avoid_prob(g, T, X, start_all=False):
    """Pr[a sampled T-path visits no vertex of X], by dynamic programming."""
    X = set(X)
    t = transition(g)
    starts = start_set(g, start_all)
    a = {v: Fraction(1, len(starts)) for v in starts if v not in X}
    for _ in range(T):
        nxt = {}
        for v, pv in a.items():
            if not t[v]:
                nxt[v] = nxt.get(v, Fraction(0)) + pv
                continue
            for u, tp in t[v]:
                if u in X:
                    continue
                nxt[u] = nxt.get(u, Fraction(0)) + pv * tp
        a = nxt
    return sum(a.values(), Fraction(0))


def similarity_by_avoidance(g, T, i, j):
    if i == j:
        return 1 - avoid_prob(g, T, {i})
    return 1 - avoid_prob(g, T, {i}) - avoid_prob(g, T, {j}) + avoid_prob(g, T, {i, j})


def avoid_prob_float(g, T, X, start_all=False):
    """Same DP in double precision, for graphs too large for rationals."""
    import numpy as np

    n = g.n
    rp = g.row_ptr.astype(np.int64)
    W = np.add.reduceat(g.w.astype(np.float64), rp[:-1]) if g.m else np.zeros(n)
    W[rp[:-1] == rp[1:]] = 0.0
    starts = np.array(start_set(g, start_all))
    mask = np.ones(n, bool)
    mask[list(X)] = False
    a = np.zeros(n)
    a[starts] = 1.0 / len(starts)
    a *= mask
    src = np.repeat(np.arange(n), np.diff(rp))
    tp = np.where(W[src] > 0, g.w.astype(np.float64) / np.where(W[src] > 0, W[src], 1.0), 0.0)
    for _ in range(T):
        nxt = np.zeros(n)
        np.add.at(nxt, g.col, a[src] * tp)
        nxt += np.where(W == 0, a, 0.0)
        a = nxt * mask
    return float(a.sum())


def sample_size(eps, c, delta, T):
    """Theorem 1 + Lemma 1: R = c/eps^2 (log2 C(T,2) + 1 + ln 1/delta)."""
    return math.ceil(c / eps ** 2 * (math.log2(math.comb(T, 2)) + 1 + math.log(1 / delta)))


def epsilon_for(R, c, delta, vc):
    """Invert Theorem 1 for the error bound at R samples and VC bound vc."""
    return math.sqrt(c * (vc + math.log(1 / delta)) / R)
