"""Pins the oracle's inverted index and top-k step with brute force and
invariants (set semantics of P_v; c(q,v) = |P_q intersect P_v|)."""
import numpy as np
import pytest


def test_index_brute_force(oracle, ba1k, ba1k_paths):
    paths, inv_ptr, inv_pid = ba1k_paths
    R = paths.shape[0]
    sets = [set(map(int, row)) for row in paths[:20000]]
    # nnz = sum of distinct vertices per path
    assert inv_ptr[-1] == sum(len(set(map(int, r))) for r in paths)
    for v in range(0, ba1k.n, 37):
        lst = inv_pid[inv_ptr[v]:inv_ptr[v + 1]]
        assert (np.diff(lst.astype(np.int64)) > 0).all()  # ascending, no duplicates
        want = [pid for pid in range(20000) if v in sets[pid]]
        got = lst[lst < 20000].tolist()
        assert got == want


def test_count_invariants(oracle, ba1k, ba1k_paths):
    paths, inv_ptr, inv_pid = ba1k_paths
    sizes = np.diff(inv_ptr)
    rng = np.random.default_rng(1)
    qs = [int(x) for x in rng.choice(ba1k.n, 12, replace=False)]
    dense = {q: oracle.counts_dense(ba1k.n, paths, inv_ptr, inv_pid, q) for q in qs}
    for q in qs:
        c = dense[q].astype(np.int64)
        assert c[q] == 0
        assert (c <= np.minimum(sizes[q], sizes)).all()
        Pq = inv_pid[inv_ptr[q]:inv_ptr[q + 1]]
        want_total = sum(len(set(map(int, paths[p]))) - 1 for p in Pq)
        assert c.sum() == want_total
        for v in rng.choice(ba1k.n, 40, replace=False):
            v = int(v)
            if v == q:
                continue
            Pv = inv_pid[inv_ptr[v]:inv_ptr[v + 1]]
            assert c[v] == np.intersect1d(Pq, Pv).size
    for a in qs:
        for b in qs:
            if a != b:
                assert dense[a][b] == dense[b][a]


def _brute_topk(c, q, k):
    c = c.astype(np.int64).copy()
    c[q] = 0
    cand = np.nonzero(c)[0]
    order = np.lexsort((cand, -c[cand]))  # count desc, id asc
    sel = cand[order][:k]
    ids = np.full(k, -1, np.int32)
    cnt = np.zeros(k, np.uint32)
    ids[:len(sel)] = sel
    cnt[:len(sel)] = c[sel]
    return ids, cnt, len(sel)


@pytest.mark.parametrize("k", [1, 10, 50, 200, 2000])
def test_topk_vs_full_sort(oracle, ba1k, ba1k_paths, k):
    paths, inv_ptr, inv_pid = ba1k_paths
    qs = np.arange(0, ba1k.n, 53, dtype=np.int32)
    ids, cnt, ln = oracle.topk(ba1k.n, paths, inv_ptr, inv_pid, qs, k)
    for i, q in enumerate(qs):
        c = oracle.counts_dense(ba1k.n, paths, inv_ptr, inv_pid, int(q))
        wi, wc, wl = _brute_topk(c, int(q), k)
        assert (ids[i] == wi).all() and (cnt[i] == wc).all() and ln[i] == wl


def test_topk_ties_star(oracle, inputs):
    """Uniform star, tiny R: many leaves share a count; order by id."""
    m = 30
    g = inputs.graph_from_edges(m + 1, [(0, i + 1) for i in range(m)])
    paths = oracle.walk(g, 5, 40, seed=3)
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    ids, cnt, ln = oracle.topk(g.n, paths, inv_ptr, inv_pid, np.array([0], np.int32), 10)
    c = oracle.counts_dense(g.n, paths, inv_ptr, inv_pid, 0)
    wi, wc, wl = _brute_topk(c, 0, 10)
    assert (ids[0] == wi).all() and (cnt[0] == wc).all()
    assert len(set(cnt[0].tolist())) < 10  # ties present


def test_topk_padding_and_unvisited_query(oracle, inputs):
    g = inputs.graph_from_edges(5, [(0, 1), (1, 2)], [1, 1])  # 3, 4 isolated
    paths = oracle.walk(g, 3, 100, seed=1)
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    ids, cnt, ln = oracle.topk(g.n, paths, inv_ptr, inv_pid, np.array([1, 3], np.int32), 5)
    assert ln[0] == 2 and set(ids[0, :2]) == {0, 2} and (ids[0, 2:] == -1).all()
    assert ln[1] == 0 and (ids[1] == -1).all() and (cnt[1] == 0).all()
