"""The allocation-free top-k entry point (panther_topk_similar_noalloc),
called through the C ABI with device buffers, against the existing
panther_topk_similar: two calls in a row on one context, the second with a
smaller input, then calls on a second context of another size sharing the
GPU's scratch array, an out-of-range query, and a graph above the scratch
limit."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _noalloc(P, dq, k, stream):
    import torch

    from paper_1504_02577_amd import panther as pm

    nq = dq.shape[0]
    out = (torch.full((nq, k), 7, dtype=torch.int32, device="cuda"),
           torch.full((nq, k), 7, dtype=torch.int32, device="cuda"),  # uint32 bits
           torch.full((nq,), 7, dtype=torch.int32, device="cuda"))
    st = pm.panther_topk_similar_noalloc(P.h, ctypes.c_void_p(dq.data_ptr()), nq, k,
                                         ctypes.c_void_p(out[0].data_ptr()),
                                         ctypes.c_void_p(out[1].data_ptr()),
                                         ctypes.c_void_p(out[2].data_ptr()),
                                         ctypes.c_void_p(stream))
    assert st == 0, pm.panther_last_error(P.h)
    torch.cuda.synchronize()
    ids, cnt, ln = (t.cpu().numpy() for t in out)
    return ids, cnt.view(np.uint32), ln


def _same(got, want, tag):
    for a, b, name in zip(got, want, ("ids", "counts", "len")):
        assert np.array_equal(np.asarray(a), np.asarray(b)), (tag, name)


def test_noalloc_equals_topk_similar(oracle, inputs):
    import torch

    from paper_1504_02577_amd.panther import PANTHER_EINVAL, Panther

    stream = torch.cuda.current_stream().cuda_stream
    g = inputs.rmat_graph(14)
    A = Panther(0)
    B = Panther(0)
    try:
        A.load_graph(g)
        A.sample_paths(5, 400_000, 7)
        A.set_option("topk.form", 1)
        q1 = np.concatenate([inputs.queries_by_degree(g, 700, 41),
                             np.arange(0, g.n, 211, dtype=np.int32)]).astype(np.int32)
        want1 = A.topk(q1, 60)
        got1 = _noalloc(A, torch.from_numpy(q1).cuda(), 60, stream)
        _same(got1, want1, "first call")
        # a second, smaller call with another k
        q2 = q1[::9].copy()
        want2 = A.topk(q2, 13)
        got2 = _noalloc(A, torch.from_numpy(q2).cuda(), 13, stream)
        _same(got2, want2, "second call")
        # another context of another size on the same GPU's array, then back
        gb = inputs.ba_graph(1000, 5)
        B.load_graph(gb)
        B.sample_paths(5, 100_000, 1)
        qb = np.arange(0, gb.n, 7, dtype=np.int32)
        _same(_noalloc(B, torch.from_numpy(qb).cuda(), 10, stream), B.topk(qb, 10), "ba1k")
        _same(_noalloc(A, torch.from_numpy(q2).cuda(), 13, stream), want2, "after ba1k")
        # the oracle agrees
        paths = oracle.walk(g, 5, 400_000, 7)
        ip, pid = oracle.index(g.n, paths)
        _same(got2, oracle.topk(g.n, paths, ip, pid, q2, 13), "oracle")
        # an out-of-range id pads its row; the others are unaffected
        q3 = np.array([q2[0], g.n + 5, -1, q2[1]], np.int32)
        ids, cnt, ln = _noalloc(A, torch.from_numpy(q3).cuda(), 13, stream)
        assert ln[1] == -1 and ln[2] == -1 and (ids[1:3] == -1).all() and (cnt[1:3] == 0).all()
        _same((ids[[0, 3]], cnt[[0, 3]], ln[[0, 3]]),
              tuple(np.asarray(w)[[0, 1]] for w in want2), "valid rows")
        # a graph with more vertices than the array holds is refused
        n_big = 8_388_601
        big = inputs.Graph(n=n_big, row_ptr=np.concatenate(
            [np.zeros(1, np.int32), np.full(n_big, 2, np.int32)]).astype(np.int32),
            col=np.array([1, 0], np.int32), w=np.array([3, 3], np.uint32))
        big.row_ptr[1] = 1
        B.load_graph(big)
        B.sample_paths(2, 1000, 1)
        from paper_1504_02577_amd import panther as pm

        dq = torch.zeros(1, dtype=torch.int32, device="cuda")
        out = torch.zeros(16, dtype=torch.int32, device="cuda")
        st = pm.panther_topk_similar_noalloc(B.h, ctypes.c_void_p(dq.data_ptr()), 1, 4,
                                             ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()), None)
        assert st == PANTHER_EINVAL and "8388600" in pm.panther_last_error(B.h)
    finally:
        A.close()
        B.close()
