"""Pins the oracle's index and counts (Algorithm 1, Eq. 4) against exact
path similarity (Eq. 1), closed forms and Theorem 1's error bound."""
import math
from fractions import Fraction

import numpy as np
import pytest


def _all_counts(oracle, g, paths):
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    C = np.zeros((g.n, g.n), np.int64)
    for q in range(g.n):
        C[q] = oracle.counts_dense(g.n, paths, inv_ptr, inv_pid, q)
    return C, inv_ptr, inv_pid


def _tiny(inputs, seed, n=6):
    rng = np.random.default_rng(seed)
    edges, ws = [], []
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < 0.5:
                edges.append((u, v)); ws.append(int(rng.integers(1, 9)))
    edges.append((0, 1)); ws.append(2)
    return inputs.graph_from_edges(n, edges, ws)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_enumeration_equals_avoidance_dp(inputs, seed):
    """Two independent exact evaluations of Eq. 1 agree as rationals."""
    from oracle import exact

    g = _tiny(inputs, seed)
    T = 3
    dist = exact.path_distribution(g, T)
    for i in range(g.n):
        for j in range(g.n):
            assert exact.exact_similarity(g, T, i, j, dist) == exact.similarity_by_avoidance(g, T, i, j)


@pytest.mark.parametrize("m,weights", [(10, None), (4, [1, 2, 3, 10])])
def test_star_closed_form(inputs, m, weights):
    """K_{1,m}, T=5: S(center, l) = 1 - (1-p_l)^2 (m - p_l) / (m+1)."""
    from oracle import exact

    g = inputs.graph_from_edges(m + 1, [(0, i + 1) for i in range(m)], weights)
    w = np.ones(m) if weights is None else np.array(weights)
    for l in range(m):
        p = Fraction(int(w[l]), int(w.sum()))
        want = 1 - (1 - p) ** 2 * (m - p) / (m + 1)
        assert exact.similarity_by_avoidance(g, 5, 0, l + 1) == want
    if weights is None:
        assert exact.similarity_by_avoidance(g, 5, 0, 1) == 1 - Fraction(m - 1, m) ** 3
        assert exact.similarity_by_avoidance(g, 5, 1, 2) == (
            1 - 2 * Fraction(m - 1, m) ** 3 + Fraction(m - 2, m) ** 3)


def test_star_center_counts_equal_list_sizes(oracle, inputs):
    """Every path of a star contains the centre, so c(0, l) = |P_l|."""
    m = 10
    g = inputs.graph_from_edges(m + 1, [(0, i + 1) for i in range(m)],
                                list(range(1, m + 1)))
    paths = oracle.walk(g, 5, 50_000, seed=1)
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    c = oracle.counts_dense(g.n, paths, inv_ptr, inv_pid, 0)
    sizes = np.diff(inv_ptr)
    assert (c[1:] == sizes[1:]).all()
    assert sizes[0] == 50_000 and c[0] == 0


def test_k2_and_disjoint_components(oracle, inputs):
    g = inputs.graph_from_edges(2, [(0, 1)], [5])
    paths = oracle.walk(g, 5, 1000, seed=1)
    inv_ptr, inv_pid = oracle.index(2, paths)
    assert oracle.counts_dense(2, paths, inv_ptr, inv_pid, 0)[1] == 1000
    # two triangles: no path crosses
    g = inputs.graph_from_edges(6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)],
                                [1, 2, 3, 4, 5, 6])
    paths = oracle.walk(g, 5, 5000, seed=2)
    C, _, _ = _all_counts(oracle, g, paths)
    assert C[:3, 3:].sum() == 0 and C[3:, :3].sum() == 0
    assert C[0, 1] > 0


@pytest.mark.parametrize("seed", [1, 4])
def test_estimator_within_theorem_bound(oracle, inputs, seed):
    """c(i,j)/R vs exact S(i,j): per-pair binomial z-scores, and the
    Theorem 1 bound with c = 0.5, delta = 0.1 and the conservative VC bound
    log2 C(T+1, 2) + 1 (a T-path has T+1 vertices)."""
    from oracle import exact

    g = _tiny(inputs, seed, n=7)
    T, R = 4, 100_000
    dist = exact.path_distribution(g, T)
    paths = oracle.walk(g, T, R, seed=seed + 100)
    C, _, _ = _all_counts(oracle, g, paths)
    eps = exact.epsilon_for(R, 0.5, 0.1, math.log2(math.comb(T + 1, 2)) + 1)
    worst = 0.0
    for i in range(g.n):
        for j in range(g.n):
            if i == j:
                continue
            S = float(exact.exact_similarity(g, T, i, j, dist))
            est = C[i, j] / R
            worst = max(worst, abs(est - S))
            if 0 < S < 1:
                z = (C[i, j] - R * S) / math.sqrt(R * S * (1 - S))
                assert abs(z) < 5.0, (i, j, z)
            else:
                assert C[i, j] == round(R * S)
    assert worst <= eps, (worst, eps)


def test_estimator_ba1k_vs_float_dp(oracle, ba1k, ba1k_paths):
    """On the 1,000-vertex BA graph, sampled S for 8 queries x 60 vertices
    vs the exact avoidance DP in double precision (binomial z-scores)."""
    from oracle import exact

    paths, inv_ptr, inv_pid = ba1k_paths
    R = paths.shape[0]
    rng = np.random.default_rng(0)
    qs = rng.choice(ba1k.n, 8, replace=False)
    A1 = {}
    for q in qs:
        c = oracle.counts_dense(ba1k.n, paths, inv_ptr, inv_pid, int(q))
        others = rng.choice(ba1k.n, 60, replace=False)
        aq = A1.setdefault(int(q), exact.avoid_prob_float(ba1k, 5, {int(q)}))
        for v in others:
            v = int(v)
            if v == q:
                continue
            av = A1.setdefault(v, exact.avoid_prob_float(ba1k, 5, {v}))
            S = 1 - aq - av + exact.avoid_prob_float(ba1k, 5, {int(q), v})
            z = (int(c[v]) - R * S) / math.sqrt(max(R * S * (1 - S), 1e-12))
            assert abs(z) < 5.5, (q, v, z)
