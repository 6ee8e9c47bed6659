"""Full-size parity at the benchmarked workload: R-MAT scale 20 (1,048,576
vertices, ~31.4M CSR entries, lognormal weights), T=5, R=10^7, Philox seed
1, 10,000 queries uniform over the start set, k=50 -- the exact launch
configuration bench.py times (batched form) plus the plain form.  Every
path, every index list and every top-k row is compared bit for bit with
the oracle."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full(oracle, inputs):
    os.environ.setdefault("PANTHER_INPUT_CACHE", "/tmp/panther_inputs")
    g, q, p = inputs.workload("rmat20")
    print(f"case: rmat20 full size n={g.n} m={g.m} R={p['R']}", file=sys.__stderr__, flush=True)
    paths = oracle.walk(g, p["T"], p["R"], p["seed"])
    inv_ptr, inv_pid = oracle.index(g.n, paths)
    want = oracle.topk(g.n, paths, inv_ptr, inv_pid, q, p["k"])
    return g, q, p, paths, inv_ptr, inv_pid, want


def test_rmat20_full_parity(full):
    from paper_1504_02577_amd.panther import Panther

    g, q, p, paths, inv_ptr, inv_pid, want = full
    P = Panther(0)
    P.load_graph(g)
    P.sample_paths(p["T"], p["R"], p["seed"])
    assert (P.paths() == paths).all()
    gp, gid = P.index(g.n)
    assert (gp == inv_ptr).all() and (gid == inv_pid).all()
    for form in (1, 0):
        P.set_option("topk.form", form)
        ids, cnt, ln = P.topk(q, p["k"])
        assert (ids == want[0]).all() and (cnt == want[1]).all() and (ln == want[2]).all(), form
    # a second sampling into the reused buffers gives the same paths
    P.sample_paths(p["T"], p["R"], p["seed"])
    assert (P.paths()[::997] == paths[::997]).all()
    P.close()


def test_rmat20_all_vertex(full, oracle):
    """All 1,048,576 vertices as queries (planned on the device): every row
    equals the oracle's top-5."""
    from paper_1504_02577_amd.panther import Panther

    g, q, p, paths, inv_ptr, inv_pid, want = full
    print("case: rmat20 all-vertex top-5", file=sys.__stderr__, flush=True)
    wall = oracle.topk(g.n, paths, inv_ptr, inv_pid, np.arange(g.n, dtype=np.int32), 5)
    P = Panther(0)
    P.load_graph(g)
    P.sample_paths(p["T"], p["R"], p["seed"])
    ids, cnt, ln = P.topk_all(g.n, 5)
    bad = np.nonzero((ids != wall[0]).any(1) | (cnt != wall[1]).any(1) | (ln != wall[2]))[0]
    assert bad.size == 0, f"{bad.size} rows differ, first {bad[:5]}"
    P.close()
