"""Pins the oracle's neighbour choice (Eq. 3) with closed forms.

u = floor(r * W / 2^64) takes value u for exactly the r in
[ceil(u 2^64 / W), ceil((u+1) 2^64 / W)), and edge e is chosen for
u in [P_{e-1}, P_e) where P is the inclusive weight prefix of the row.
So edge e is chosen exactly for r in [ceil(P_{e-1} 2^64/W), ceil(P_e 2^64/W)),
i.e. with probability w_e / W up to one part in 2^64 / W.
"""
import numpy as np
import pytest

TWO64 = 1 << 64


def ceil_div(a, b):
    return -(-a // b)


def test_scale_boundaries(oracle):
    rng = np.random.default_rng(5)
    for W in [1, 2, 3, 7, 100, 65537, (1 << 32) - 1, 1 << 32, (1 << 40) + 3]:
        for u in set([0, 1, W - 1] + [int(x) for x in rng.integers(0, W, 20)]):
            if u >= W:
                continue
            lo = ceil_div(u * TWO64, W)
            assert oracle.scale(lo, W) == u
            if lo > 0:
                assert oracle.scale(lo - 1, W) == u - 1
        assert oracle.scale(0, W) == 0
        assert oracle.scale(TWO64 - 1, W) == W - 1


def test_preimage_counts_exhaustive_small(oracle):
    # each u has floor(2^64/W) or ceil(2^64/W) preimages
    for W in range(1, 65):
        for u in range(W):
            cnt = ceil_div((u + 1) * TWO64, W) - ceil_div(u * TWO64, W)
            assert cnt in (TWO64 // W, ceil_div(TWO64, W))
            # and the oracle agrees at both ends of the preimage interval
            a = ceil_div(u * TWO64, W)
            b = ceil_div((u + 1) * TWO64, W) - 1
            assert oracle.scale(a, W) == u and oracle.scale(b, W) == u


def _star_row_graph(inputs, weights):
    # vertex 0 joined to 1..d with the given weights (zero allowed)
    d = len(weights)
    return inputs.graph_from_edges(d + 1, [(0, i + 1) for i in range(d)], weights)


@pytest.mark.parametrize("weights", [[5], [1, 1], [3, 0, 4], [0, 0, 7, 0, 2, 0],
                                     [100] * 17, list(range(1, 40)), [0, 1]])
def test_pick_edge_interval_ends(oracle, inputs, weights):
    g = _star_row_graph(inputs, weights)
    W = sum(weights)
    P = np.cumsum(weights)
    prev = 0
    for e, w in enumerate(weights):
        lo = ceil_div(prev * TWO64, W)
        hi = ceil_div(int(P[e]) * TWO64, W)  # exclusive
        if w == 0:
            assert lo == hi  # empty interval: never chosen
        else:
            assert oracle.pick_edge(g, 0, lo) == e
            assert oracle.pick_edge(g, 0, hi - 1) == e
        prev = int(P[e])
    first_pos = next(i for i, w in enumerate(weights) if w > 0)
    last_pos = max(i for i, w in enumerate(weights) if w > 0)
    assert oracle.pick_edge(g, 0, 0) == first_pos
    assert oracle.pick_edge(g, 0, TWO64 - 1) == last_pos


def test_pick_edge_matches_linear_scan(oracle, inputs):
    """Bisection == the plain definition (first prefix > u) on random rows."""
    rng = np.random.default_rng(9)
    for trial in range(30):
        d = int(rng.integers(1, 300))
        weights = [int(x) for x in rng.integers(0, 5, d)]
        if sum(weights) == 0:
            weights[-1] = 1
        g = _star_row_graph(inputs, weights)
        W = sum(weights)
        for _ in range(50):
            r = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
            u = (r * W) >> 64
            s, want = 0, None
            for e, w in enumerate(weights):
                s += w
                if s > u:
                    want = e
                    break
            assert oracle.pick_edge(g, 0, r) == want


def test_zero_weight_row_returns_none(oracle, inputs):
    g = inputs.graph_from_edges(3, [(0, 1), (1, 2)], [0, 0])
    assert oracle.pick_edge(g, 1, 12345) == -1
