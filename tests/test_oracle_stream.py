"""Pins the oracle's sampled-path helpers used for runs too large to replay
whole: ``walk_pids`` (chosen path ids, Algorithm 3) and ``stream_counts``
(the list lengths of the inverted index and the counts of Algorithm 1,
streamed over every path without storing it).

``walk_pids`` is checked against ``walk`` (every pid of a run, random and
extreme pids, both start readings) and, for path ids at or above 2^32 that
no stored run reaches, against a step-by-step composition of the pinned
primitives (Philox draw, start-set scaling, edge pick).  ``stream_counts``
is checked against a numpy count of the definition over the stored paths
(c(q, v) = number of paths whose vertex set holds both q and v; |P_v| =
number of paths holding v)."""
import numpy as np
import pytest


def _numpy_counts(paths, n, q):
    """c(q, v) for every v straight from the definition (Eq. 4 numerator)."""
    rows = paths[(paths == q).any(1)]
    s = np.sort(rows, 1)
    first = np.ones_like(s, dtype=bool)
    first[:, 1:] = s[:, 1:] != s[:, :-1]
    c = np.bincount(s[first], minlength=n).astype(np.uint32)
    c[q] = 0
    return c


def _numpy_list_len(paths, n):
    s = np.sort(paths, 1)
    first = np.ones_like(s, dtype=bool)
    first[:, 1:] = s[:, 1:] != s[:, :-1]
    return np.bincount(s[first], minlength=n).astype(np.uint64)


@pytest.mark.parametrize("start_all", [False, True])
def test_walk_pids_equals_walk(oracle, inputs, start_all):
    g = inputs.graph_from_edges(60, [(i, (i * 7 + 3) % 50) for i in range(50)] + [(0, 1)],
                                [1 + (i % 9) for i in range(51)])  # vertices 50..59 isolated
    T, R, seed = 4, 20_000, 123
    full = oracle.walk(g, T, R, seed, start_all=start_all)
    rng = np.random.default_rng(5)
    pids = np.concatenate([[0, 1, R - 2, R - 1], rng.integers(0, R, 500)]).astype(np.int64)
    got = oracle.walk_pids(g, T, seed, pids, start_all=start_all)
    assert (got == full[pids]).all()
    # every id of the run, in order
    assert (oracle.walk_pids(g, T, seed, np.arange(R), start_all=start_all) == full).all()


def test_walk_pids_beyond_2_32(oracle, ba1k):
    """Path ids with a non-zero high word take Philox counter word 3; the
    path is the composition of the pinned draw, start scaling and edge
    pick."""
    T, seed = 5, 77
    starts = oracle.start_set(ba1k)
    pids = np.array([1 << 32, (1 << 32) + 12345, (1 << 40) + 9, (1 << 63) - 1], np.int64)
    got = oracle.walk_pids(ba1k, T, seed, pids)
    for row, pid in zip(got, pids.tolist()):
        v = int(starts[oracle.scale(oracle.draw(seed, pid, 0), len(starts))])
        want = [v]
        for t in range(1, T + 1):
            e = oracle.pick_edge(ba1k, v, oracle.draw(seed, pid, t))
            v = int(ba1k.col[e])
            want.append(v)
        assert row.tolist() == want
    # the high word matters: pid 2^32 is not pid 0
    assert not (got[0] == oracle.walk_pids(ba1k, T, seed, np.array([0]))[0]).all()


def test_stream_counts_equal_definition(oracle, ba1k, ba1k_paths):
    paths, inv_ptr, inv_pid = ba1k_paths
    T, R, seed = 5, paths.shape[0], 1
    rng = np.random.default_rng(9)
    qs = np.concatenate([[0, ba1k.n - 1], rng.choice(ba1k.n, 10, replace=False)]).astype(np.int32)
    ln, cnt = oracle.stream_counts(ba1k, T, R, seed, qs)
    assert (ln == _numpy_list_len(paths, ba1k.n)).all()
    assert (ln == np.diff(inv_ptr)).all()
    for i, q in enumerate(qs.tolist()):
        assert (cnt[i] == _numpy_counts(paths, ba1k.n, q)).all(), q
    # symmetry between two queries
    assert cnt[2][qs[3]] == cnt[3][qs[2]]
    # top-k from dense counts equals the oracle's top-k
    want = oracle.topk(ba1k.n, paths, inv_ptr, inv_pid, qs, 15)
    for i, q in enumerate(qs.tolist()):
        ids, c, m = oracle.topk_from_counts(cnt[i], q, 15)
        assert (ids == want[0][i]).all() and (c == want[1][i]).all() and m == want[2][i]


def test_stream_counts_start_all(oracle, inputs):
    g = inputs.graph_from_edges(40, [(i, i + 1) for i in range(25)] + [(0, 7)],
                                list(range(1, 27)))  # 26..39 isolated
    T, R, seed = 3, 30_000, 4
    paths = oracle.walk(g, T, R, seed, start_all=True)
    qs = np.array([0, 3, 30, 39], np.int32)  # two isolated queries
    ln, cnt = oracle.stream_counts(g, T, R, seed, qs, start_all=True)
    assert (ln == _numpy_list_len(paths, g.n)).all()
    for i, q in enumerate(qs.tolist()):
        assert (cnt[i] == _numpy_counts(paths, g.n, q)).all()
    assert cnt[2].sum() == 0 and cnt[3].sum() == 0  # an isolated start stays put
