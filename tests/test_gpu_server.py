"""Serving loop: each result equals the same request run alone.

A mixed stream (80% Panther / 20% Panther++, k uniform over {10, 50, 200},
query vertices proportional to degree) is submitted while batches are in
flight on three lanes.  Panther results must be bit-identical to the
standalone panther_topk_similar call with the same k; Panther++ results
must match the standalone panther_pp_topk call (distances within 1e-9
relative, ids equal outside ties)."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def setup(oracle, inputs):
    from paper_1504_02577_amd.panther import Panther

    g = inputs.rmat_graph(14)
    P = Panther(0)
    P.load_graph(g)
    P.sample_paths(5, 400_000, 7)
    rng = np.random.default_rng(21)
    n_req = 3000
    kinds = (rng.random(n_req) < 0.2).astype(np.int32)
    ks = rng.choice([10, 50, 200], n_req).astype(np.int32)
    qs = inputs.queries_by_degree(g, n_req, 22)
    # standalone answers, one call per distinct (kind, k)
    alone = {}
    for kind in (0, 1):
        for k in (10, 50, 200):
            sel = np.nonzero((kinds == kind) & (ks == k))[0]
            if sel.size == 0:
                continue
            if kind == 0:
                ids, cnt, ln = P.topk(qs[sel], int(k))
                for j, i in enumerate(sel):
                    alone[i] = (ids[j], cnt[j].astype(np.float64))
            else:
                ids, dist = P.pp_topk(qs[sel], 50, int(k))
                for j, i in enumerate(sel):
                    alone[i] = (ids[j], dist[j])
    yield g, P, kinds, ks, qs, alone
    P.close()


def _compare(i, kind, got_ids, got_sc, want_ids, want_sc):
    if kind == 0:
        assert (got_ids == want_ids).all() and (got_sc == want_sc).all(), i
        return
    fin = np.isfinite(want_sc)
    assert (np.isfinite(got_sc) == fin).all(), i
    assert np.allclose(got_sc[fin], want_sc[fin], rtol=1e-9, atol=0), i
    for j in range(len(want_ids)):
        if got_ids[j] != want_ids[j]:
            assert np.isclose(want_sc, want_sc[j], rtol=1e-9, atol=0).sum() > 1, (i, j)


def _run(srv, kinds, ks, qs, pace_s=0.0):
    results = {}
    for i in range(len(qs)):
        st = srv.submit(int(kinds[i]), int(qs[i]), int(ks[i]), i)
        assert st == 0, st
        if pace_s:
            time.sleep(pace_s)
        for r in srv.poll(0):
            results[r["tag"]] = r
    t0 = time.time()
    while len(results) < len(qs) and time.time() - t0 < 60:
        for r in srv.poll(20000):
            results[r["tag"]] = r
    return results


@pytest.mark.parametrize("lanes,max_batch", [(3, 256), (1, 16), (2, 1)])
def test_mixed_stream_equals_alone(setup, lanes, max_batch):
    from paper_1504_02577_amd.panther import Server

    g, P, kinds, ks, qs, alone = setup
    _say(f"case: server lanes={lanes} max_batch={max_batch}")
    srv = Server(P, mem_budget_bytes=1 << 30, max_batch=max_batch, lanes=lanes, D=50)
    try:
        res = _run(srv, kinds, ks, qs)
        assert len(res) == len(qs)
        for i, r in res.items():
            assert r["status"] == 0 and r["query"] == qs[i] and r["k"] == ks[i]
            _compare(i, r["kind"], r["ids"], r["scores"], *alone[i])
        st = srv.stats()
        _say(f"  p50 {st['p50_ms']:.3f} ms  p99 {st['p99_ms']:.3f} ms  qps {st['qps']:.0f}")
        assert st["completed"] == len(qs) and st["p99_ms"] >= st["p50_ms"] > 0
    finally:
        assert srv.stop() == 0


def test_memory_admission(setup):
    from paper_1504_02577_amd.panther import PANTHER_ENOMEM, Server

    g, P, kinds, ks, qs, alone = setup
    _say("case: server memory admission")
    # room for about one Panther++ request with k = 200 at a time
    srv = Server(P, mem_budget_bytes=40_000, max_batch=64, lanes=3, D=50)
    try:
        sel = np.arange(300)
        res = _run(srv, kinds[sel], ks[sel], qs[sel])
        assert len(res) == len(sel)
        for i, r in res.items():
            _compare(i, r["kind"], r["ids"], r["scores"], *alone[sel[i]])
    finally:
        srv.stop()
    tiny = Server(P, mem_budget_bytes=4096, max_batch=8, lanes=1, D=50)
    try:
        assert tiny.submit(1, 0, 200, 0) == PANTHER_ENOMEM
    finally:
        tiny.stop()
