"""Pins the oracle's Panther++ steps (Sec. 3.3, Algorithm 2): the feature
vectors theta(v) and the exact Euclidean k-nearest-neighbour search."""
import math
from fractions import Fraction

import numpy as np
import pytest


def test_features_vs_sorted_counts(oracle, ba1k, ba1k_paths):
    paths, inv_ptr, inv_pid = ba1k_paths
    R = paths.shape[0]
    D = 50
    theta = oracle.features(ba1k.n, paths, inv_ptr, inv_pid, D)
    for v in range(0, ba1k.n, 29):
        c = oracle.counts_dense(ba1k.n, paths, inv_ptr, inv_pid, v).astype(np.int64)
        c[v] = 0
        top = np.sort(c)[::-1][:D]
        want = (top.astype(np.float32) / np.float32(R)).astype(np.float32)
        assert (theta[v] == want).all()
        assert (np.diff(theta[v]) <= 0).all()


def test_features_zero_rows_for_unvisited(oracle, inputs):
    g = inputs.graph_from_edges(6, [(0, 1), (1, 2), (2, 0)], [1, 2, 3])
    paths = oracle.walk(g, 5, 1000, seed=1)
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    th = oracle.features(g.n, paths, inv_ptr, inv_pid, 4)
    assert (th[3:] == 0).all()
    assert (th[0, :2] > 0).all() and (th[0, 2:] == 0).all()  # two others only


def _exact_knn(theta, q, k):
    n, D = theta.shape
    rows = [[Fraction(float(x)) for x in theta[v]] for v in range(n)]
    d2 = []
    for v in range(n):
        if v == q:
            continue
        d2.append((sum((a - b) ** 2 for a, b in zip(rows[q], rows[v])), v))
    d2.sort()
    return d2[:k]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_knn_vs_exact_rationals(oracle, seed):
    rng = np.random.default_rng(seed)
    n, D, k = 60, 7, 9
    theta = (rng.integers(0, 40, (n, D)) / 1000.0).astype(np.float32)
    theta = -np.sort(-theta, axis=1)
    theta[5] = theta[9]  # identical rows -> exact ties broken by id
    theta[11] = theta[9]
    theta[20:23] = 0.0
    qs = np.array([0, 9, 20, 33], np.int32)
    ids, dist = oracle.knn(theta, qs, k)
    for i, q in enumerate(qs):
        want = _exact_knn(theta, int(q), k)
        wd = np.array([math.sqrt(float(d)) for d, _ in want])
        assert np.allclose(dist[i], wd, rtol=1e-12, atol=0)
        # ids agree wherever the exact distance separates neighbours
        for j, (d, v) in enumerate(want):
            others = [dd for dd, _ in want if dd != d]
            assert ids[i, j] == v or any(abs(float(d - dd)) < 1e-12 for dd in others)
    # identical rows: query 9 sees 5 and 11 at distance 0, in id order
    assert ids[1, 0] == 5 and ids[1, 1] == 11 and dist[1, 0] == 0.0
    # zero rows: query 20 sees 21, 22 first
    assert ids[2, 0] == 21 and ids[2, 1] == 22


def test_knn_padding(oracle):
    theta = np.ones((3, 4), np.float32)
    ids, dist = oracle.knn(theta, np.array([1], np.int32), 5)
    assert ids[0].tolist() == [0, 2, -1, -1, -1]
    assert np.isinf(dist[0, 2:]).all() and (dist[0, :2] == 0).all()


def _exact_cross(tq, tdb, k):
    rq = [Fraction(float(x)) for x in tq]
    d2 = sorted((sum((a - Fraction(float(b))) ** 2 for a, b in zip(rq, tdb[v])), v)
                for v in range(tdb.shape[0]))
    return d2[:k]


@pytest.mark.parametrize("seed", [0, 1])
def test_knn_cross_vs_exact_rationals(oracle, seed):
    """Cross-graph kNN: a query row of one graph against every row of the
    other, ranked by exact rational squared distance, ties by id."""
    rng = np.random.default_rng(10 + seed)
    D, k = 6, 8
    tdb = (rng.integers(0, 30, (45, D)) / 1000.0).astype(np.float32)
    tq = (rng.integers(0, 30, (4, D)) / 1000.0).astype(np.float32)
    tq[1] = tdb[17]            # an exact twin: distance 0, rank first ...
    tdb[3] = tdb[17]           # ... behind an identical row of smaller id
    ids, dist = oracle.knn_cross(tq, tdb, k)
    for i in range(tq.shape[0]):
        want = _exact_cross(tq[i], tdb, k)
        assert np.allclose(dist[i], [math.sqrt(float(d)) for d, _ in want], rtol=1e-12, atol=0)
        for j, (d, v) in enumerate(want):
            others = [dd for dd, _ in want if dd != d]
            assert ids[i, j] == v or any(abs(float(d - dd)) < 1e-12 for dd in others)
    assert ids[1, 0] == 3 and ids[1, 1] == 17 and dist[1, 0] == 0.0 and dist[1, 1] == 0.0


def test_knn_cross_reduces_to_single_graph(oracle, ba1k, ba1k_paths):
    """With both sides the same graph, dropping the query itself from its
    cross-graph list of k+1 leaves exactly its single-graph list of k."""
    paths, inv_ptr, inv_pid = ba1k_paths
    theta = oracle.features(ba1k.n, paths, inv_ptr, inv_pid, 12)
    qs = np.array([0, 3, 77, 500, 999], np.int32)
    k = 10
    ci, cd = oracle.knn_cross(theta[qs], theta, k + 1)
    si, sd = oracle.knn(theta, qs, k)
    for i, q in enumerate(qs):
        keep = ci[i] != q
        assert (ci[i][keep][:k] == si[i]).all()
        assert (cd[i][keep][:k] == sd[i]).all()


def test_two_copy_twins(oracle, inputs):
    """Two copies of one graph with permuted ids, each with its own paths:
    a vertex's twin in the other copy ranks among its nearest neighbours
    across the graphs, and more often as R grows (the estimates converge,
    Theorem 1).  This is the identity-resolution use of Panther++."""
    g = inputs.ba_graph(1000, 5)
    gb, perm = inputs.permuted_copy(g, 4)
    assert gb.m == g.m
    qs = np.arange(0, g.n, 7, dtype=np.int32)
    rate = {}
    for R in (100_000, 400_000):
        pa = oracle.walk(g, 5, R, 1)
        pb = oracle.walk(gb, 5, R, 2)
        ta = oracle.features(g.n, pa, *oracle.index(g.n, pa), 20)
        tb = oracle.features(gb.n, pb, *oracle.index(gb.n, pb), 20)
        ids, _ = oracle.knn_cross(ta[qs], tb, 10)
        rate[R] = np.mean([perm[q] in ids[i] for i, q in enumerate(qs)])
    assert rate[400_000] >= 0.9 and rate[400_000] > rate[100_000]


def test_knn_cross_padding(oracle):
    ids, dist = oracle.knn_cross(np.zeros((1, 3), np.float32), np.ones((2, 3), np.float32), 4)
    assert ids[0].tolist() == [0, 1, -1, -1] and np.isinf(dist[0, 2:]).all()


def test_dist2_is_fma_chain(oracle):
    """Squared distance of float32 rows in double, one fma per coordinate:
    exact for values whose differences square without rounding."""
    a = np.array([0.5, 0.25, 3.0], np.float32)
    b = np.array([0.0, 0.75, 1.0], np.float32)
    assert oracle.dist2(a, b) == 0.25 + 0.25 + 4.0


def test_sample_size_closed_forms(oracle):
    """Theorem 1 with Lemma 1: R = c/eps^2 (log2 C(T,2) + 1 + ln 1/delta)."""
    e = math.exp(1.0)
    # T = 2: C(2,2) = 1 -> log term vanishes; delta = 1/e -> ln term is 1
    assert oracle.sample_size(0.01, 1.0, 1 / e, 2) in (20000, 20001)
    # T = 3: C(3,2) = 3; c = 0.5, delta = 0.1, eps = 0.1
    want = 0.5 / 0.01 * (math.log2(3) + 1 + math.log(10))
    assert oracle.sample_size(0.1, 0.5, 0.1, 3) == math.ceil(want)
    # the paper's setting (c=0.5, delta=0.1, T=5, eps=sqrt(1/|E|)) gives
    # R ~= 3.3123 |E| (Section 3.4 parameters)
    for E in (10_000, 1_000_000):
        assert abs(oracle.sample_size(math.sqrt(1 / E), 0.5, 0.1, 5) / E - 3.3123) < 1e-3
    # quartering eps^2 quadruples R
    a = oracle.sample_size(0.02, 0.5, 0.1, 5)
    b = oracle.sample_size(0.01, 0.5, 0.1, 5)
    assert abs(b - 4 * a) <= 4
    assert oracle.sample_size(0.1, 0.5, 0.1, 1) < 0  # C(1,2) = 0: undefined
