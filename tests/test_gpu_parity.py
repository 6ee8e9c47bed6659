"""GPU parity: the HIP path through the C ABI against the oracle.

Paths, the inverted index and top-k lists are integer results and must be
bit-exact.  Sizes: a 1,000-vertex BA graph (all of it), an R-MAT scale-14
graph (all paths, all lists, thousands of queries, lists long enough for
every sort tier), and edge cases.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P():
    from paper_1504_02577_amd.panther import Panther

    p = Panther(0)
    yield p
    p.close()


def _check_topk(got, want, tag):
    gi, gc, gl = got
    wi, wc, wl = want
    bad = np.nonzero((gi != wi).any(1) | (gc != wc).any(1) | (gl != wl))[0]
    assert bad.size == 0, f"{tag}: {bad.size} rows differ, first row {bad[:5]}"


@pytest.fixture(scope="module")
def ba_state(oracle, inputs, P):
    g = inputs.ba_graph(1000, 5)
    T, R, seed = 5, 100_000, 1
    paths = oracle.walk(g, T, R, seed)
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    return g, T, R, seed, paths, inv_ptr, inv_pid


def test_ba1k_paths_and_index(P, ba_state):
    g, T, R, seed, paths, inv_ptr, inv_pid = ba_state
    _say("case: ba1k paths/index")
    P.load_graph(g)
    P.sample_paths(T, R, seed)
    assert (P.paths() == paths).all()
    gp, gid = P.index(g.n)
    assert (gp == inv_ptr).all()
    assert (gid == inv_pid).all()


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("k", [1, 10, 200, 1024])
def test_ba1k_topk_all_vertices(P, oracle, ba_state, form, k):
    g, T, R, seed, paths, inv_ptr, inv_pid = ba_state
    _say(f"case: ba1k topk form={form} k={k}")
    P.load_graph(g)
    P.sample_paths(T, R, seed)
    P.set_option("topk.form", form)
    q = np.arange(g.n, dtype=np.int32)
    want = oracle.topk(g.n, paths, inv_ptr, inv_pid, q, k)
    _check_topk(P.topk(q, k), want, f"form={form} k={k}")


@pytest.fixture(scope="module")
def rmat14(oracle, inputs):
    g = inputs.rmat_graph(14)
    T, R, seed = 5, 400_000, 7
    paths = oracle.walk(g, T, R, seed)
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    return g, T, R, seed, paths, inv_ptr, inv_pid


def test_rmat14_full_parity(P, oracle, inputs, rmat14):
    g, T, R, seed, paths, inv_ptr, inv_pid = rmat14
    _say("case: rmat14 paths/index/topk")
    assert np.diff(inv_ptr).max() > 4096 * 2  # exercises chunk sort + merges
    P.load_graph(g)
    P.sample_paths(T, R, seed)
    assert (P.paths() == paths).all()
    gp, gid = P.index(g.n)
    assert (gp == inv_ptr).all() and (gid == inv_pid).all()
    qs = np.concatenate([inputs.queries_by_degree(g, 3000, 5),
                         np.argsort(-np.diff(inv_ptr))[:20].astype(np.int32)])
    for form in (0, 1):
        P.set_option("topk.form", form)
        want = oracle.topk(g.n, paths, inv_ptr, inv_pid, qs, 50)
        _check_topk(P.topk(qs, 50), want, f"rmat14 form={form}")


def test_start_all_vertices_and_isolated(P, oracle, inputs):
    from paper_1504_02577_amd.panther import PANTHER_START_ALL_VERTICES

    _say("case: start-all flag")
    g = inputs.graph_from_edges(50, [(i, i + 1) for i in range(30)] + [(0, 5), (3, 9)],
                                list(range(1, 33)))
    for flags, start_all in ((0, False), (PANTHER_START_ALL_VERTICES, True)):
        P.load_graph(g, flags=flags)
        P.sample_paths(3, 20_000, 99)
        want = oracle.walk(g, 3, 20_000, 99, start_all=start_all)
        assert (P.paths() == want).all()
        inv_ptr, inv_pid = oracle.index(g.n, want)
        gp, gid = P.index(g.n)  # empty lists of isolated vertices
        assert (gp == inv_ptr).all() and (gid == inv_pid).all()
        q = np.arange(g.n, dtype=np.int32)  # includes isolated vertices
        P.set_option("topk.form", 1)
        _check_topk(P.topk(q, 7), oracle.topk(g.n, want, inv_ptr, inv_pid, q, 7), "start")


def test_long_paths_and_wide_weights(P, oracle, inputs):
    """T = 20 (stride 32) and row weight sums >= 2^32 (64-bit prefixes)."""
    _say("case: T=20 and 64-bit prefixes")
    rng = np.random.default_rng(3)
    edges = [(int(a), int(b)) for a, b in rng.integers(0, 200, (1500, 2))]
    w = rng.integers(1 << 30, (1 << 32) - 1, len(edges), dtype=np.uint64).astype(np.uint32)
    g = inputs.graph_from_edges(200, edges, w)
    assert oracle.row_weights(g).max() >= 1 << 32
    P.load_graph(g)
    for T in (20, 1, 63):
        P.sample_paths(T, 30_000, 5)
        want = oracle.walk(g, T, 30_000, 5)
        assert (P.paths() == want).all(), T
        inv_ptr, inv_pid = oracle.index(g.n, want)
        gp, gid = P.index(g.n)
        assert (gp == inv_ptr).all() and (gid == inv_pid).all()
        q = np.arange(0, 200, 3, dtype=np.int32)
        _check_topk(P.topk(q, 30), oracle.topk(g.n, want, inv_ptr, inv_pid, q, 30), f"T={T}")


def test_duplicates_and_device_buffers(P, oracle, ba_state):
    import torch

    g, T, R, seed, paths, inv_ptr, inv_pid = ba_state
    _say("case: duplicate queries, device buffers")
    P.load_graph(g)
    P.sample_paths(T, R, seed)
    q = np.array([3, 3, 17, 3, 999, 17], np.int32)
    want = oracle.topk(g.n, paths, inv_ptr, inv_pid, q, 25)
    dq = torch.from_numpy(q).cuda()
    out = (torch.empty((6, 25), dtype=torch.int32, device="cuda"),
           torch.empty((6, 25), dtype=torch.uint32, device="cuda"),
           torch.empty(6, dtype=torch.int32, device="cuda"))
    stream = torch.cuda.current_stream().cuda_stream
    for form in (0, 1):
        P.set_option("topk.form", form)
        P.topk(dq, 25, out=out, stream=stream)
        torch.cuda.synchronize()
        got = tuple(t.cpu().numpy() for t in out)
        _check_topk(got, want, f"device form={form}")
    assert (got[0][0] == got[0][1]).all() and (got[0][0] == got[0][3]).all()


def test_errors_leave_context_usable(P, oracle, inputs, ba_state):
    from paper_1504_02577_amd.panther import (PANTHER_EINVAL, PANTHER_ENOMEM, PANTHER_ERANGE,
                                              PANTHER_ESTATE, Panther, PantherError)

    g, T, R, seed, paths, inv_ptr, inv_pid = ba_state
    _say("case: error paths")
    fresh = Panther(0)
    with pytest.raises(PantherError) as e:
        fresh.sample_paths(5, 100, 1)
    assert e.value.code == PANTHER_ESTATE
    # malformed CSR
    bad = inputs.Graph(n=g.n, row_ptr=g.row_ptr.copy(), col=g.col.copy(), w=g.w)
    bad.col[7] = g.n + 3
    with pytest.raises(PantherError) as e:
        fresh.load_graph(bad)
    assert e.value.code == PANTHER_EINVAL
    bad = inputs.Graph(n=g.n, row_ptr=g.row_ptr.copy(), col=g.col, w=g.w)
    bad.row_ptr[10], bad.row_ptr[11] = bad.row_ptr[11], bad.row_ptr[10] - 1
    with pytest.raises(PantherError) as e:
        fresh.load_graph(bad)
    assert e.value.code == PANTHER_EINVAL
    fresh.load_graph(g)
    for T_, R_ in ((0, 10), (64, 10), (5, 0), (5, 1 << 32)):
        with pytest.raises(PantherError) as e:
            fresh.sample_paths(T_, R_, 1)
        assert e.value.code == PANTHER_EINVAL
    with pytest.raises(PantherError) as e:
        fresh.topk(np.array([1], np.int32), 5)
    assert e.value.code == PANTHER_ESTATE
    # allocation failure injected during sampling, then recovery
    fresh.set_option("test.fail_alloc_after", 2)
    with pytest.raises(PantherError) as e:
        fresh.sample_paths(T, R, seed)
    assert e.value.code == PANTHER_ENOMEM
    fresh.set_option("test.fail_alloc_after", -1)
    fresh.sample_paths(T, R, seed)
    # out-of-range query: nothing written
    ids = np.full((2, 5), 77, np.int32)
    from paper_1504_02577_amd import panther as pm
    import ctypes
    q = np.array([1, g.n], np.int32)
    cnt = np.full((2, 5), 77, np.uint32)
    ln = np.full(2, 77, np.int32)
    st = pm.panther_topk_similar(fresh.h, q.ctypes.data_as(ctypes.c_void_p), 2, 5,
                                 ids.ctypes.data_as(ctypes.c_void_p),
                                 cnt.ctypes.data_as(ctypes.c_void_p),
                                 ln.ctypes.data_as(ctypes.c_void_p), pm.PANTHER_MEM_HOST, None)
    assert st == PANTHER_ERANGE and (ids == 77).all() and (ln == 77).all()
    for kk in (0, 1025):
        with pytest.raises(PantherError) as e:
            fresh.topk(np.array([1], np.int32), kk)
        assert e.value.code == PANTHER_EINVAL
    # still usable
    qq = np.array([0, 5], np.int32)
    _check_topk(fresh.topk(qq, 10), oracle.topk(g.n, paths, inv_ptr, inv_pid, qq, 10), "after")
    fresh.close()


@pytest.mark.parametrize("block,wgs,ta,tb,hb,budget", [
    (512, 1, -1, -1, -1, 0), (256, 1, -1, -1, -1, 0), (512, 2, -1, -1, -1, 0),
    (256, 2, -1, -1, -1, 0),
    (512, 1, 0, 0, -1, 0),     # every non-empty list goes to the split hub pipeline
    (256, 1, 4, 0, -1, 0),     # wave tier + hub pipeline
    (512, 2, 1, 60, -1, 0),    # all three tiers, small tables
    (512, 1, 0, 0, 0, 0),      # one bucket per hub: large ones overflow the LDS table
    (512, 1, -1, 60, 1, 0),    # two buckets per hub, overflow and sub-range splits
    # a staging budget of 64 KiB splits the hub queries into many chunks
    # (each at least the longest list's T * L slots), as at R-MAT 24
    (512, 1, 0, 0, -1, 1 << 16),
    (512, 1, -1, 60, 1, 1 << 16),
    (256, 2, 4, 0, 0, 1 << 16),
])
def test_batched_tiers_rmat14(P, oracle, inputs, rmat14, block, wgs, ta, tb, hb, budget):
    g, T, R, seed, paths, inv_ptr, inv_pid = rmat14
    _say(f"case: batched tiers block={block} wgs={wgs} ta={ta} tb={tb} hub_bits={hb} "
         f"hub_budget={budget}")
    P.load_graph(g)
    P.sample_paths(T, R, seed)
    P.set_option("topk.form", 1)
    P.set_option("batch.block", block)
    P.set_option("batch.wgs_per_cu", wgs)
    P.set_option("batch.tier_a", ta)
    P.set_option("batch.tier_b", tb)
    P.set_option("batch.hub_bits", hb)
    P.set_option("test.hub_budget", budget)
    try:
        qs = np.concatenate([inputs.queries_by_degree(g, 1500, 11),
                             np.arange(0, g.n, 97, dtype=np.int32)])
        for k in (1, 50, 300):
            want = oracle.topk(g.n, paths, inv_ptr, inv_pid, qs, k)
            _check_topk(P.topk(qs, k), want, f"tiers {block}/{wgs}/{ta}/{tb}/{hb}/{budget} k={k}")
    finally:
        for key, v in (("batch.block", 0), ("batch.wgs_per_cu", 0), ("batch.tier_a", -1),
                       ("batch.tier_b", -1), ("batch.hub_bits", -1), ("test.hub_budget", 0)):
            P.set_option(key, v)


@pytest.mark.parametrize("div,bias", [(2, 0), (1, 1), (2, 1)])
def test_batched_tuner_choices_rmat14(P, oracle, inputs, rmat14, div, bias):
    """Each (tier B divisor, bucket bias) the autotuner may pick gives the
    same lists."""
    g, T, R, seed, paths, inv_ptr, inv_pid = rmat14
    _say(f"case: batched tuner choice tier_b_div={div} bucket_bias={bias}")
    P.load_graph(g)
    P.sample_paths(T, R, seed)
    P.set_option("topk.form", 1)
    P.set_option("batch.tier_b_div", div)
    P.set_option("batch.bucket_bias", bias)
    try:
        qs = np.concatenate([inputs.queries_by_degree(g, 1500, 13),
                             np.arange(0, g.n, 89, dtype=np.int32)])
        for k in (1, 50, 300):
            want = oracle.topk(g.n, paths, inv_ptr, inv_pid, qs, k)
            _check_topk(P.topk(qs, k), want, f"tuner choice {div}/{bias} k={k}")
    finally:
        P.set_option("batch.tier_b_div", 0)
        P.set_option("batch.bucket_bias", -1)


def test_autotune_cache_rmat14(P, oracle, inputs, rmat14, tmp_path, monkeypatch):
    """The autotuner stores one line per shape class, a later call reuses it,
    and malformed lines are skipped."""
    g, T, R, seed, paths, inv_ptr, inv_pid = rmat14
    _say("case: autotune cache")
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PANTHER_TUNE_CACHE", str(cache))
    P.load_graph(g)
    P.sample_paths(T, R, seed)
    P.set_option("topk.form", 1)
    P.set_option("autotune", 1)
    P.set_option("batch.block", 0)  # drops the lane's tuned choice
    qs = np.concatenate([inputs.queries_by_degree(g, 1500, 17),
                         np.arange(0, g.n, 83, dtype=np.int32)])
    want = oracle.topk(g.n, paths, inv_ptr, inv_pid, qs, 50)
    _check_topk(P.topk(qs, 50), want, "autotuned")
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    f = lines[0].split()
    assert len(f) == 5 and int(f[1]) in (256, 512) and int(f[2]) in (1, 2)
    assert int(f[3]) in (1, 2) and int(f[4]) in (0, 1)
    key = f[0]
    # a stored line (here the short form of earlier caches) is reused: no
    # new line is appended
    text = f"{key} 512 9 1 0\n{key} 300 1\n{key} 256 2\n"
    cache.write_text(text)
    P.set_option("batch.block", 0)
    _check_topk(P.topk(qs, 50), want, "cached")
    assert cache.read_text() == text
    # only malformed lines: the tuner runs again and appends its choice
    cache.write_text(f"{key} 512 1 3 0\n{key} 512\n")
    P.set_option("batch.block", 0)
    _check_topk(P.topk(qs, 50), want, "retuned")
    assert len(cache.read_text().splitlines()) == 3


def test_device_planned_batch_rmat14(P, oracle, inputs, rmat14, tmp_path, monkeypatch):
    """A batch of 2^20 queries is planned on the device (digit keys sorted by
    the index's radix pass, only the hubs' lengths downloaded); the
    autotuner, run afresh, times host-planned prefixes of it.  Every row
    equals the oracle's, in host and device outputs, with the tuned and the
    forced configurations."""
    import torch

    g, T, R, seed, paths, inv_ptr, inv_pid = rmat14
    _say("case: device-planned batch of 2^20 queries")
    monkeypatch.setenv("PANTHER_TUNE_CACHE", str(tmp_path / "tune.txt"))
    P.load_graph(g)
    P.sample_paths(T, R, seed)
    P.set_option("topk.form", 1)
    P.set_option("autotune", 1)
    P.set_option("batch.block", 0)
    rng = np.random.default_rng(23)
    qs = np.concatenate([rng.integers(0, g.n, (1 << 20) - 4096),
                         inputs.queries_by_degree(g, 4096, 29)]).astype(np.int32)
    uq, inv = np.unique(qs, return_inverse=True)
    k = 10
    wu = oracle.topk(g.n, paths, inv_ptr, inv_pid, uq, k)
    want = (wu[0][inv], wu[1][inv], wu[2][inv])
    assert (np.diff(inv_ptr)[qs] > 400).any()  # hubs among them
    _check_topk(P.topk(qs, k), want, "device plan, tuned")
    assert (tmp_path / "tune.txt").exists()
    dq = torch.from_numpy(qs).cuda()
    out = (torch.full((len(qs), k), 7, dtype=torch.int32, device="cuda"),
           torch.full((len(qs), k), 7, dtype=torch.uint32, device="cuda"),
           torch.full((len(qs),), 7, dtype=torch.int32, device="cuda"))
    for blk, wgs in ((256, 2), (512, 1)):
        P.set_option("batch.block", blk)
        P.set_option("batch.wgs_per_cu", wgs)
        P.topk(dq, k, out=out, stream=torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        _check_topk(tuple(t.cpu().numpy() for t in out), want, f"device plan {blk}x{wgs}")
    P.set_option("batch.block", 0)
    P.set_option("batch.wgs_per_cu", 0)


@pytest.mark.parametrize("k", [5, 50])
def test_all_vertex_topk(P, oracle, rmat14, k):
    """panther_topk_all equals the oracle's top-k of every vertex (the
    paper's all-vertex workload), host and device outputs."""
    import torch

    g, T, R, seed, paths, inv_ptr, inv_pid = rmat14
    _say(f"case: all-vertex top-{k}")
    P.load_graph(g)
    P.sample_paths(T, R, seed)
    q = np.arange(g.n, dtype=np.int32)
    want = oracle.topk(g.n, paths, inv_ptr, inv_pid, q, k)
    _check_topk(P.topk_all(g.n, k), want, f"all-vertex k={k}")
    out = (torch.full((g.n, k), 7, dtype=torch.int32, device="cuda"),
           torch.full((g.n, k), 7, dtype=torch.uint32, device="cuda"),
           torch.full((g.n,), 7, dtype=torch.int32, device="cuda"))
    P.topk_all(g.n, k, out=out, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    _check_topk(tuple(t.cpu().numpy() for t in out), want, f"all-vertex device k={k}")


def test_batched_graph_replays(P, oracle, inputs, rmat14):
    """Repeated calls with the same buffers replay the captured graph; each
    replay, with other device work and synchronisations in between, must
    equal the oracle."""
    import torch

    g, T, R, seed, paths, inv_ptr, inv_pid = rmat14
    _say("case: batched graph replays")
    P.load_graph(g)
    P.sample_paths(T, R, seed)
    P.set_option("topk.form", 1)
    qs = inputs.queries_by_degree(g, 2000, 12)
    want = oracle.topk(g.n, paths, inv_ptr, inv_pid, qs, 40)
    dq = torch.from_numpy(qs).cuda()
    out = (torch.empty((len(qs), 40), dtype=torch.int32, device="cuda"),
           torch.empty((len(qs), 40), dtype=torch.uint32, device="cuda"),
           torch.empty(len(qs), dtype=torch.int32, device="cuda"))
    stream = torch.cuda.current_stream().cuda_stream
    x = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        for t in out:
            t.fill_(7)
        P.topk(dq, 40, out=out, stream=stream)
        torch.cuda.synchronize()
        _check_topk(tuple(t.cpu().numpy() for t in out), want, f"replay {rep}")
        x = (x * 1.0001).sin()  # unrelated eager work between replays
        torch.cuda.synchronize()


def test_check_symmetric_flag(P, inputs, ba_state):
    """PANTHER_CHECK_SYMMETRIC (Definition 1: undirected edges, stored in
    both rows with one weight): asymmetric entries, mismatched weights and
    unmatched parallel entries are rejected with EINVAL before anything is
    loaded; symmetric input passes, also with rows not in column order."""
    from paper_1504_02577_amd.panther import (PANTHER_CHECK_SYMMETRIC, PANTHER_EINVAL,
                                              PANTHER_ESTATE, PantherError)

    g, T, R, seed, paths, inv_ptr, inv_pid = ba_state
    _say("case: symmetric check")
    P.load_graph(g, flags=PANTHER_CHECK_SYMMETRIC)  # the BA graph is symmetric
    P.sample_paths(T, 1000, seed)

    def rejected(gg):
        with pytest.raises(PantherError) as e:
            P.load_graph(gg, flags=PANTHER_CHECK_SYMMETRIC)
        assert e.value.code == PANTHER_EINVAL, e.value
        with pytest.raises(PantherError) as e2:  # nothing loaded
            P.sample_paths(T, 10, seed)
        assert e2.value.code == PANTHER_ESTATE

    # one weight changed on one side only
    bad = inputs.Graph(n=g.n, row_ptr=g.row_ptr, col=g.col, w=g.w.copy())
    bad.w[123] += 1
    rejected(bad)
    # a directed edge: 0 -> 1 only
    d = inputs.Graph(n=3, row_ptr=np.array([0, 1, 1, 1], np.int32),
                     col=np.array([1], np.int32), w=np.array([5], np.uint32))
    rejected(d)
    # parallel entries: two 0->1 of weight 2, one 1->0
    mm = inputs.Graph(n=2, row_ptr=np.array([0, 2, 3], np.int32),
                      col=np.array([1, 1, 0], np.int32), w=np.array([2, 2, 2], np.uint32))
    rejected(mm)
    # the same with both copies on the other side passes; so do unsorted
    # rows and a self-loop
    ok = inputs.Graph(n=3, row_ptr=np.array([0, 3, 5, 6], np.int32),
                      col=np.array([2, 1, 1, 0, 0, 0], np.int32),
                      w=np.array([7, 2, 2, 2, 2, 7], np.uint32))
    P.load_graph(ok, flags=PANTHER_CHECK_SYMMETRIC)
    loop = inputs.Graph(n=2, row_ptr=np.array([0, 2, 3], np.int32),
                        col=np.array([0, 1, 0], np.int32), w=np.array([4, 3, 3], np.uint32))
    P.load_graph(loop, flags=PANTHER_CHECK_SYMMETRIC)
    # without the flag a directed CSR is walked as given
    P.load_graph(d)
    P.sample_paths(2, 100, 1)
    assert (P.paths()[:, 0] == 0).all() and (P.paths()[:, 1:] == 1).all()


def test_resample_with_new_stride_after_capture(P, oracle, inputs, rmat14):
    """A captured batched launch must not be replayed over paths of another
    row stride: T = 9 (stride 16) twice on device buffers captures the
    launch; after sampling T = 5 (stride 8) the same call must use the
    stride-8 kernels."""
    import torch

    g, T, R, seed, paths, inv_ptr, inv_pid = rmat14
    _say("case: resample with a new stride after graph capture")
    P.load_graph(g)
    P.set_option("topk.form", 1)
    qs = inputs.queries_uniform(g, 600, 31)
    dq = torch.from_numpy(qs).cuda()
    k = 20
    out = (torch.empty((len(qs), k), dtype=torch.int32, device="cuda"),
           torch.empty((len(qs), k), dtype=torch.uint32, device="cuda"),
           torch.empty(len(qs), dtype=torch.int32, device="cuda"))
    stream = torch.cuda.current_stream().cuda_stream
    R9 = 60_000
    paths9 = oracle.walk(g, 9, R9, seed)
    p9, i9 = oracle.index(g.n, paths9)
    want9 = oracle.topk(g.n, paths9, p9, i9, qs, k)
    P.sample_paths(9, R9, seed)
    for _ in range(3):
        P.topk(dq, k, out=out, stream=stream)
        torch.cuda.synchronize()
        _check_topk(tuple(t.cpu().numpy() for t in out), want9, "T=9")
    R5 = 90_000  # fewer path bytes than the T=9 run: the buffers are reused
    paths5 = oracle.walk(g, 5, R5, seed)
    p5, i5 = oracle.index(g.n, paths5)
    want5 = oracle.topk(g.n, paths5, p5, i5, qs, k)
    P.sample_paths(5, R5, seed)
    for _ in range(3):
        P.topk(dq, k, out=out, stream=stream)
        torch.cuda.synchronize()
        _check_topk(tuple(t.cpu().numpy() for t in out), want5, "T=5 after T=9")
