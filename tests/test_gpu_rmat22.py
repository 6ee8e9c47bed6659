"""Parity at R-MAT scale 22, the Panther++ workload: 4,194,304 vertices,
T=5, R=5*10^7, Philox seed 1, D=50, 65,536 queries uniform over the start
set, k=20, candidate pool 256.

Features (Algorithm 2: the D largest c(v, u) / R over u != v in IEEE single
precision) are compared bit for bit for every vertex.  The BF16 form runs
the benchmarked call (all 65,536 queries in one call, device buffers) and a
1,024-query call; on a seeded sample of 1,024 queries both must return the
oracle's exact FP64 neighbours (Sec. 3.3): the same ids and bit-identical
distances.  The FP64 form is checked on 128 of them."""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1500)]


@pytest.fixture(scope="module")
def c4(oracle, inputs, progress):
    _say = progress
    import time

    t0 = time.time()
    _say("case: rmat22_pp: generating the inputs")
    g, q, p = inputs.workload("rmat22_pp")
    _say(f"case: rmat22_pp n={g.n} m={g.m} R={p['R']} (inputs {time.time() - t0:.0f} s)")
    t0 = time.time()
    paths = oracle.walk(g, p["T"], p["R"], p["seed"])
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    _say(f"  oracle walk + index {time.time() - t0:.0f} s")
    t0 = time.time()
    theta = oracle.features(g.n, paths, inv_ptr, inv_pid, p["D"])
    del paths, inv_pid
    _say(f"  oracle features {time.time() - t0:.0f} s")
    rng = np.random.default_rng(1024)
    sample = np.sort(rng.choice(len(q), 1024, replace=False))
    t0 = time.time()
    wi, wd = oracle.knn(theta, q[sample], p["k"])
    _say(f"  oracle kNN of 1,024 queries {time.time() - t0:.0f} s")
    return g, q, p, theta, sample, wi, wd


def _exact(gi, gd, wi, wd, tag):
    bad = np.nonzero((gi != wi).any(1))[0]
    assert bad.size == 0, f"{tag}: ids differ in {bad.size} rows, first {bad[:5]}"
    g = np.ascontiguousarray(gd, np.float64).view(np.uint64)
    w = np.ascontiguousarray(wd, np.float64).view(np.uint64)
    bad = np.nonzero((g != w).any(1))[0]
    assert bad.size == 0, f"{tag}: distances differ in {bad.size} rows, first {bad[:5]}"


def test_rmat22_features_and_knn(c4, progress):
    _say = progress
    import torch
    from paper_1504_02577_amd.panther import Panther

    g, q, p, theta, sample, wi, wd = c4
    T, R, seed, k, D = p["T"], p["R"], p["seed"], p["k"], p["D"]
    P = Panther(0)
    try:
        P.load_graph(g)
        P.sample_paths(T, R, seed)
        got = P.features(g.n, D)
        bad = np.nonzero((got.view(np.uint32) != theta.view(np.uint32)).any(1))[0]
        assert bad.size == 0, f"features differ in {bad.size} rows, first {bad[:5]}"
        del got
        # the benchmarked call: every query at once, device buffers
        P.set_option("pp.form", 1)
        P.set_option("pp.pool", p["pool"])
        dq = torch.from_numpy(q).cuda()
        out = (torch.empty((len(q), k), dtype=torch.int32, device="cuda"),
               torch.empty((len(q), k), dtype=torch.float64, device="cuda"))
        P.pp_topk(dq, D, k, out=out, stream=torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        ids, dist = out[0].cpu().numpy(), out[1].cpu().numpy()
        _exact(ids[sample], dist[sample], wi, wd, "bf16 65,536-query call")
        nq, redo = P.pp_certified()
        _say(f"  certified {nq - redo} of {nq}, recomputed {redo}")
        # a 1,024-query call (sliced scan with the bound pass)
        gi, gd = P.pp_topk(q[sample], D, k)
        _exact(gi, gd, wi, wd, "bf16 1,024-query call")
        P.set_option("pp.form", 0)
        gi, gd = P.pp_topk(q[sample[:128]], D, k)
        _exact(gi, gd, wi[:128], wd[:128], "fp64 form")
    finally:
        P.close()
