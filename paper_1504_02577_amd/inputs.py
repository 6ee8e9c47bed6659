"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only *produces* inputs: graphs in CSR form, edge weights and
query-vertex lists.  It contains none of the method's arithmetic (no
transition probabilities, no sampling, no counting), so the oracle and the
GPU path can both consume its output without sharing any computation.

Graph families (stand-ins for the paper's Tencent / Twitter / Mobile /
co-author networks, which are not available):

* Barabasi-Albert graphs (``networkx.barabasi_albert_graph``) with uniform
  integer weights in [1, 100].
* R-MAT graphs (Chakrabarti et al.) with quadrant probabilities
  a=0.57, b=0.19, c=0.19, d=0.05, edge factor 16, self-loops dropped,
  duplicate undirected pairs merged, vertex ids randomly relabelled, and
  weights ``rint(lognormal(0, 1) * 100) + 1``.

Every graph is undirected (Section 2, Definition 1): each undirected edge is
stored twice in the CSR with the same weight, neighbours ascending.
"""
from __future__ import annotations

import dataclasses
import os
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[m]
    w: np.ndarray        # uint32[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def _csr_from_undirected(n: int, u: np.ndarray, v: np.ndarray, w: np.ndarray,
                         name: str) -> Graph:
    """Symmetrise a list of undirected edges (u != v, unique pairs) into CSR.

    Every directed (row, col) pair is distinct, so sorting by the key
    row * n + col orders the entries uniquely (rows ascending, neighbours
    ascending).  When the key fits 48 bits and the weights 16 bits, the
    weight rides in the low bits of one sorted 64-bit word; otherwise an
    argsort carries it."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.uint32)
    m = 2 * u.shape[0]
    if m >= 2 ** 31:
        raise ValueError("graph too large for int32 CSR")
    wmax = int(w.max()) if w.size else 0
    if n <= (1 << 24) and wmax < (1 << 16):
        key = np.empty(m, dtype=np.uint64)
        h = u.shape[0]
        np.multiply(u, n, out=key[:h], casting="unsafe")
        key[:h] += v.astype(np.uint64)
        np.multiply(v, n, out=key[h:], casting="unsafe")
        key[h:] += u.astype(np.uint64)
        key <<= np.uint64(16)
        wk = w.astype(np.uint64)
        key[:h] |= wk
        key[h:] |= wk
        del wk
        key.sort()
        ws = (key & np.uint64(0xFFFF)).astype(np.uint32)
        key >>= np.uint64(16)
        rows = key // np.uint64(n)
        cols = (key - rows * np.uint64(n)).astype(np.int32)
        del key
        counts = np.bincount(rows.astype(np.int64), minlength=n)
        del rows
    else:
        rows = np.concatenate([u, v])
        cols = np.concatenate([v, u])
        ws = np.concatenate([w, w])
        key = rows * np.int64(n) + cols
        order = np.argsort(key)  # keys are distinct: any sort gives this order
        del key
        rows = rows[order]
        cols = cols[order].astype(np.int32)
        ws = ws[order]
        del order
        counts = np.bincount(rows, minlength=n)
        del rows
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr.astype(np.int32), col=cols, w=ws,
                 name=name)


def graph_from_edges(n: int, edges, weights=None, name: str = "custom") -> Graph:
    """Build an undirected CSR graph from explicit (u, v) pairs.

    Pairs are canonicalised (min, max); self-loops and duplicates are dropped
    (the first weight given for a pair is kept).  ``weights`` defaults to 1.
    """
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if weights is None:
        weights = np.ones(e.shape[0], dtype=np.uint32)
    weights = np.asarray(weights, dtype=np.uint32)
    a = np.minimum(e[:, 0], e[:, 1])
    b = np.maximum(e[:, 0], e[:, 1])
    keep = a != b
    a, b, weights = a[keep], b[keep], weights[keep]
    key = a * n + b
    _, first = np.unique(key, return_index=True)
    first = np.sort(first)
    return _csr_from_undirected(n, a[first], b[first], weights[first], name)


def ba_graph(n: int, m: int, seed: int = 7, weight_seed: int = 11) -> Graph:
    """Barabasi-Albert graph with uniform integer weights in [1, 100]."""
    import networkx as nx

    g = nx.barabasi_albert_graph(n, m, seed=seed)
    e = np.array(sorted((min(a, b), max(a, b)) for a, b in g.edges()),
                 dtype=np.int64).reshape(-1, 2)
    rng = np.random.default_rng(weight_seed)
    w = rng.integers(1, 101, size=e.shape[0], dtype=np.int64).astype(np.uint32)
    return _csr_from_undirected(n, e[:, 0], e[:, 1], w, f"ba{n}_m{m}")


def rmat_graph(scale: int, edge_factor: int = 16, a: float = 0.57,
               b: float = 0.19, c: float = 0.19, seed: int = 20,
               weight_seed: int = 21, perm_seed: int = 22) -> Graph:
    """R-MAT graph, lognormal weights ``rint(lognormal(0,1)*100)+1``."""
    n = 1 << scale
    n_edges = edge_factor * n
    rng = np.random.default_rng(seed)
    src = np.zeros(n_edges, dtype=np.uint32)
    dst = np.zeros(n_edges, dtype=np.uint32)
    ab = np.float32(a + b)
    abc = np.float32(a + b + c)
    fa = np.float32(a)
    chunk = 1 << 24

    def assemble(s, d, levels):
        # quadrant of each level, most significant bit first: row bit =
        # (r >= a+b); column bit = (a <= r < a+b) or (r >= a+b+c)
        b1 = np.empty(s.shape[0], dtype=bool)
        b2 = np.empty(s.shape[0], dtype=bool)
        for r in levels:
            np.left_shift(s, 1, out=s)
            np.greater_equal(r, ab, out=b1)
            np.bitwise_or(s, b1, out=s, casting="unsafe")
            np.greater_equal(r, fa, out=b2)
            np.logical_not(b1, out=b1)
            np.logical_and(b2, b1, out=b2)
            np.greater_equal(r, abc, out=b1)
            np.logical_or(b2, b1, out=b2)
            np.left_shift(d, 1, out=d)
            np.bitwise_or(d, b2, out=d, casting="unsafe")

    # the draws stay in one sequential stream (chunk by chunk, level by
    # level); the bit assembly of each chunk runs on a worker thread
    import concurrent.futures as cf

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        pending = []
        for lo in range(0, n_edges, chunk):
            hi = min(n_edges, lo + chunk)
            levels = [rng.random(hi - lo, dtype=np.float32) for _ in range(scale)]
            pending.append(ex.submit(assemble, src[lo:hi], dst[lo:hi], levels))
            del levels
            if len(pending) >= 4:
                pending.pop(0).result()
        for f in pending:
            f.result()
    lo_v = np.minimum(src, dst).astype(np.uint64)
    hi_v = np.maximum(src, dst).astype(np.uint64)
    del src, dst
    keep = lo_v != hi_v
    key = (lo_v[keep] << np.uint64(32)) | hi_v[keep]
    del lo_v, hi_v, keep
    key = np.unique(key)
    u = (key >> np.uint64(32)).astype(np.int64)
    v = (key & np.uint64(0xFFFFFFFF)).astype(np.int64)
    del key
    perm = np.random.default_rng(perm_seed).permutation(n).astype(np.int64)
    u = perm[u]
    v = perm[v]
    wr = np.random.default_rng(weight_seed)
    w = (np.rint(wr.lognormal(0.0, 1.0, size=u.shape[0]) * 100.0) + 1.0)
    w = w.astype(np.uint32)
    return _csr_from_undirected(n, u, v, w, f"rmat{scale}")


def permuted_copy(g: Graph, seed: int):
    """An isomorphic copy of g with vertex ids permuted: vertex v of g is
    perm[v] of the copy, and every edge keeps its weight.  Returns (copy,
    perm)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(g.n).astype(np.int32)
    deg = np.diff(g.row_ptr.astype(np.int64))
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    keep = src < g.col  # each undirected pair once; pairs stay distinct under perm
    u = perm[src[keep]].astype(np.int64)
    v = perm[g.col[keep]].astype(np.int64)
    return _csr_from_undirected(g.n, u, v, g.w[keep], g.name + "_perm"), perm


def start_vertices(g: Graph) -> np.ndarray:
    """Vertices with at least one incident edge of positive weight."""
    rp = g.row_ptr.astype(np.int64)
    pos = (g.w > 0).astype(np.int64)
    csum = np.concatenate([[0], np.cumsum(pos)])
    has = csum[rp[1:]] - csum[rp[:-1]] > 0
    return np.nonzero(has)[0].astype(np.int32)


def queries_uniform(g: Graph, count: int, seed: int,
                    over: str = "start") -> np.ndarray:
    """Distinct query vertices, uniform over V ('all') or over V_start."""
    rng = np.random.default_rng(seed)
    pool = np.arange(g.n, dtype=np.int32) if over == "all" else start_vertices(g)
    count = min(count, pool.shape[0])
    return np.sort(rng.choice(pool, size=count, replace=False)).astype(np.int32)


def queries_by_degree(g: Graph, count: int, seed: int) -> np.ndarray:
    """Query vertices drawn proportional to degree, with replacement.

    Each draw takes the source vertex of a uniformly random CSR entry.
    """
    rng = np.random.default_rng(seed)
    e = rng.integers(0, g.m, size=count, dtype=np.int64)
    q = np.searchsorted(g.row_ptr.astype(np.int64), e, side="right") - 1
    return q.astype(np.int32)


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the evaluated configurations: a small
# BA graph, and R-MAT scale 20 / 22 / 24 graphs.
# ---------------------------------------------------------------------------
WORKLOADS = {
    "ba1k": dict(graph=("ba", 1000, 5), T=5, R=100_000, seed=1,
                 queries=("uniform_all", 16, 101), k=10),
    "rmat20": dict(graph=("rmat", 20), T=5, R=10_000_000, seed=1,
                   queries=("uniform_start", 10_000, 102), k=50),
    "rmat24": dict(graph=("rmat", 24), T=5, R=100_000_000, seed=1,
                   queries=("degree", 100_000, 103), k=50),
    "rmat22_pp": dict(graph=("rmat", 22), T=5, R=50_000_000, seed=1,
                      queries=("uniform_start", 65_536, 104), k=20, D=50,
                      pool=256),
}


def _cache_path(name: str) -> Optional[str]:
    d = os.environ.get("PANTHER_INPUT_CACHE")
    if not d:
        return None
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, f"{name}.npz")


def make_graph(spec) -> Graph:
    kind = spec[0]
    if kind == "ba":
        name = f"ba{spec[1]}_m{spec[2]}"
    else:
        name = f"rmat{spec[1]}"
    path = _cache_path(name)
    if path and os.path.exists(path):
        z = np.load(path)
        return Graph(n=int(z["n"]), row_ptr=z["row_ptr"], col=z["col"],
                     w=z["w"], name=name)
    if kind == "ba":
        g = ba_graph(spec[1], spec[2])
    elif kind == "rmat":
        g = rmat_graph(spec[1])
    else:
        raise ValueError(kind)
    if path:
        np.savez(path, n=np.int64(g.n), row_ptr=g.row_ptr, col=g.col, w=g.w)
    return g


def make_queries(g: Graph, spec) -> np.ndarray:
    kind, count, seed = spec
    if kind == "uniform_all":
        return queries_uniform(g, count, seed, over="all")
    if kind == "uniform_start":
        return queries_uniform(g, count, seed, over="start")
    if kind == "degree":
        return queries_by_degree(g, count, seed)
    raise ValueError(kind)


def workload(name: str):
    """Return (graph, queries, params) for a named workload."""
    p = dict(WORKLOADS[name])
    g = make_graph(p["graph"])
    q = make_queries(g, p["queries"])
    return g, q, p
