"""Sample-size-driven R with more than 2^32 index entries (Theorem 1 with
Lemma 1, Sec. 3.2: R of the order of c / eps^2 grows past what 32-bit list
offsets address).  The 1,000-vertex BA graph is sampled with T=5 and
R = 8.5*10^8 paths (about 5.45 distinct vertices each), so the inverted index
holds about 4.6*10^9 entries and
the offsets of the higher vertex ids exceed 2^32.

Checked against the oracle, which streams over every path without storing
it: every list offset (inv_ptr, from the oracle's |P_v|), 4,096 sampled
paths (including the first and last id), every list restricted to three
windows of path ids (the oracle's index of the window's paths), and the
top-50 of eight queries, among them the highest ids, whose lists start past
2^32."""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1500)]

T, R, SEED, K = 5, 850_000_000, 3, 50


def test_index_beyond_2_32(oracle, inputs, progress):
    _say = progress
    import time

    import torch
    from paper_1504_02577_amd.panther import Panther

    g = inputs.ba_graph(1000, 5)
    qs = np.array([0, 1, 17, 500, 996, 997, 998, 999], np.int32)
    _say(f"case: bigR ba1k T={T} R={R}")
    P = Panther(0)
    try:
        P.load_graph(g)
        P.sample_paths(T, R, SEED)
        nnz = P.nnz()
        _say(f"  nnz {nnz}")
        assert nnz > 1 << 32
        ptr, pid = P.index_device(g.n)
        h_ptr = ptr.cpu().numpy()
        ids, cnt, ln = P.topk(qs, K)
        t0 = time.time()
        o_len, o_cnt = oracle.stream_counts(g, T, R, SEED, qs)
        _say(f"  oracle stream over {R} paths {time.time() - t0:.0f} s")
        want_ptr = np.concatenate([[0], np.cumsum(o_len.astype(np.int64))])
        assert np.array_equal(h_ptr, want_ptr), "list offsets differ"
        assert h_ptr[qs[-1]] > 1 << 32  # the last queries' lists start past 2^32
        for i, q in enumerate(qs.tolist()):
            wi, wc, wl = oracle.topk_from_counts(o_cnt[i], q, K)
            assert (ids[i] == wi).all() and (cnt[i] == wc).all() and ln[i] == wl, q
        # sampled paths
        rng = np.random.default_rng(11)
        pids = np.concatenate([[0, R - 1], rng.integers(0, R, 4094)]).astype(np.int64)
        paths = P.paths_device()
        got = paths[torch.from_numpy(pids).cuda()].cpu().numpy()
        assert np.array_equal(got, oracle.walk_pids(g, T, SEED, pids)), "sampled paths differ"
        del paths
        # every list, restricted to windows of path ids
        for a in (0, 372_000_000, R - 200_000):
            b = a + 200_000
            wp = oracle.walk_pids(g, T, SEED, np.arange(a, b, dtype=np.int64))
            w_ptr, w_pid = oracle.index(g.n, wp)
            for v in range(g.n):  # path ids < 2^31: the int32 view sorts as uint32
                seg = pid[int(h_ptr[v]):int(h_ptr[v + 1])]
                x = int(torch.searchsorted(seg, torch.tensor([a], dtype=torch.int32,
                                                             device="cuda")).item())
                y = int(torch.searchsorted(seg, torch.tensor([b], dtype=torch.int32,
                                                             device="cuda")).item())
                got_v = seg[x:y].cpu().numpy().astype(np.int64) - a
                want_v = w_pid[w_ptr[v]:w_ptr[v + 1]].astype(np.int64)
                assert np.array_equal(got_v, want_v), (a, v)
    finally:
        P.close()
