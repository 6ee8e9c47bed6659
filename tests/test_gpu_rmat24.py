"""Parity at R-MAT scale 24, the batched workload: 16,777,216 vertices,
520,759,432 CSR entries, lognormal weights, T=5, R=10^8, Philox seed 1,
10^5 query vertices drawn proportional to degree (heavy-tailed path lists),
k=50 -- the launch configuration bench.py times (batched form, device
buffers, the caller's stream; its hub queries take several staging chunks).

Every path (Algorithm 3), every index list (Sec. 3.1) and all 10^5 top-k
rows (Algorithm 1) are compared bit for bit with the oracle; a replay of the
captured launch and the plain form on the longest lists are checked too."""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1500)]


@pytest.fixture(scope="module")
def c3(oracle, inputs, progress):
    _say = progress
    import time

    t0 = time.time()
    _say("case: rmat24: generating the inputs")
    g, q, p = inputs.workload("rmat24")
    _say(f"case: rmat24 n={g.n} m={g.m} R={p['R']} queries={len(q)} "
         f"(inputs {time.time() - t0:.0f} s)")
    t0 = time.time()
    paths = oracle.walk(g, p["T"], p["R"], p["seed"])
    _say(f"  oracle walk {time.time() - t0:.0f} s")
    t0 = time.time()
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    _say(f"  oracle index {time.time() - t0:.0f} s, nnz {len(inv_pid)}")
    t0 = time.time()
    want = oracle.topk(g.n, paths, inv_ptr, inv_pid, q, p["k"])
    _say(f"  oracle top-k {time.time() - t0:.0f} s")
    return g, q, p, paths, inv_ptr, inv_pid, want


def _check_rows(got, want, tag, rows=None):
    gi, gc, gl = got
    wi, wc, wl = want
    if rows is not None:
        wi, wc, wl = wi[rows], wc[rows], wl[rows]
    bad = np.nonzero((gi != wi).any(1) | (gc != wc).any(1) | (gl != wl))[0]
    assert bad.size == 0, f"{tag}: {bad.size} rows differ, first {bad[:5]}"


def test_rmat24_full_parity(c3, progress):
    _say = progress
    import torch
    from paper_1504_02577_amd.panther import Panther

    g, q, p, paths, inv_ptr, inv_pid, want = c3
    T, R, seed, k = p["T"], p["R"], p["seed"], p["k"]
    P = Panther(0)
    try:
        P.load_graph(g)
        P.sample_paths(T, R, seed)
        assert np.array_equal(P.paths(), paths), "paths differ"
        _say("  paths equal the oracle's")
        gp, gid = P.index(g.n)
        assert np.array_equal(gp, inv_ptr) and np.array_equal(gid, inv_pid), "index differs"
        del gp, gid
        _say("  index equals the oracle's")
        lens = np.diff(inv_ptr)[q]
        _say(f"  sum |P_q| = {int(lens.sum())}, max {int(lens.max())}")
        # the benchmarked launch: batched form, device buffers, torch's stream
        P.set_option("topk.form", 1)
        dq = torch.from_numpy(q).cuda()
        out = (torch.empty((len(q), k), dtype=torch.int32, device="cuda"),
               torch.empty((len(q), k), dtype=torch.uint32, device="cuda"),
               torch.empty(len(q), dtype=torch.int32, device="cuda"))
        stream = torch.cuda.current_stream().cuda_stream
        for rep in range(3):  # the third call replays the captured launch
            for t in out:
                t.fill_(7)
            P.topk(dq, k, out=out, stream=stream)
            torch.cuda.synchronize()
            _check_rows(tuple(t.cpu().numpy() for t in out), want, f"batched call {rep}")
            _say(f"  batched call {rep}: all {len(q)} rows equal the oracle's")
        # plain form (one launch per query) on the 200 longest lists and 300 others
        P.set_option("topk.form", 0)
        rows = np.concatenate([np.argsort(-lens, kind="stable")[:200],
                               np.random.default_rng(3).choice(len(q), 300, replace=False)])
        _check_rows(P.topk(q[rows], k), want, "plain", rows)
    finally:
        P.close()
