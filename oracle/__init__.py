"""The oracle: a plain CPU implementation of the Panther hot path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package.  The product path (the
HIP library in ``paper_1504_02577_amd``) never imports it, and it never
imports the product path.

``oracle.c`` holds the arithmetic (compiled with gcc into ``liboracle.so``);
this module only marshals numpy arrays through ctypes.  ``exact.py`` holds
the exact (un-sampled) quantities used to pin the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(openmp: bool = True) -> str:
    """Compile oracle.c with gcc -O2 into liboracle.so."""
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", _SO + ".tmp", src, "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64, u32, u64, dbl = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_draw.argtypes = [u64, u64, u32]
        L.or_draw.restype = u64
        L.or_scale.argtypes = [u64, u64]
        L.or_scale.restype = u64
        L.or_validate.argtypes = [i32, i64, P, P]
        L.or_row_weights.argtypes = [i32, P, P, P]
        L.or_row_prefix.argtypes = [i32, P, P, P]
        L.or_start_set.argtypes = [i32, P, ctypes.c_int, P]
        L.or_start_set.restype = i32
        L.or_pick_edge.argtypes = [P, P, P, i32, u64]
        L.or_pick_edge.restype = i64
        L.or_walk.argtypes = [i32, i64, P, P, P, i32, i64, u64, ctypes.c_int, P]
        L.or_walk_pids.argtypes = [i32, i64, P, P, P, i32, u64, ctypes.c_int, P, i64, P]
        L.or_index_ptr.argtypes = [i32, i32, i64, P, P]
        L.or_index_ptr.restype = i64
        L.or_index_fill.argtypes = [i32, i32, i64, P, P, P]
        L.or_counts_dense.argtypes = [i32, i32, P, P, P, i32, P]
        L.or_topk.argtypes = [i32, i32, P, P, P, P, i64, i32, P, P, P]
        L.or_features.argtypes = [i32, i32, i64, P, P, P, i32, P]
        L.or_dist2.argtypes = [P, P, i32]
        L.or_dist2.restype = dbl
        L.or_knn.argtypes = [i32, i32, P, P, i64, i32, P, P]
        L.or_knn_cross.argtypes = [i32, i64, P, i32, P, i32, P, P]
        L.or_stream_counts.argtypes = [i32, i64, P, P, P, i32, i64, u64, ctypes.c_int, P, i32,
                                       P, P]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_get_threads.restype = ctypes.c_int
        L.or_sample_size.argtypes = [dbl, dbl, dbl, i32]
        L.or_sample_size.restype = i64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _check(status: int, what: str):
    if status != 0:
        raise RuntimeError(f"oracle {what} failed with status {status}")


# -- random bits -------------------------------------------------------------
def philox4x32_10(counter, key) -> np.ndarray:
    c = _c(counter, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def draw(seed: int, pid: int, step: int) -> int:
    return int(lib().or_draw(seed, pid, step))


def scale(r: int, n: int) -> int:
    return int(lib().or_scale(r, n))


# -- graph -------------------------------------------------------------------
def validate(g) -> bool:
    rp = _c(g.row_ptr, np.int32)
    col = _c(g.col, np.int32)
    return lib().or_validate(g.n, g.m, _p(rp), _p(col)) == 0


def row_weights(g) -> np.ndarray:
    W = np.zeros(g.n, np.uint64)
    lib().or_row_weights(g.n, _p(_c(g.row_ptr, np.int32)), _p(_c(g.w, np.uint32)), _p(W))
    return W


def start_set(g, start_all: bool = False) -> np.ndarray:
    W = row_weights(g)
    out = np.zeros(g.n, np.int32)
    k = lib().or_start_set(g.n, _p(W), int(start_all), _p(out))
    return out[:k].copy()


def pick_edge(g, v: int, r: int) -> int:
    rp = _c(g.row_ptr, np.int32)
    w = _c(g.w, np.uint32)
    W = row_weights(g)
    pfx = np.zeros(max(g.m, 1), np.uint64)
    lib().or_row_prefix(g.n, _p(rp), _p(w), _p(pfx))
    return int(lib().or_pick_edge(_p(rp), _p(pfx), _p(W), v, r))


# -- hot path ----------------------------------------------------------------
def walk(g, T: int, R: int, seed: int, start_all: bool = False) -> np.ndarray:
    rp = _c(g.row_ptr, np.int32)
    col = _c(g.col, np.int32)
    w = _c(g.w, np.uint32)
    paths = np.zeros((R, T + 1), np.int32)
    _check(lib().or_walk(g.n, g.m, _p(rp), _p(col), _p(w), T, R, seed,
                         int(start_all), _p(paths)), "walk")
    return paths


def walk_pids(g, T: int, seed: int, pids, start_all: bool = False) -> np.ndarray:
    rp = _c(g.row_ptr, np.int32)
    col = _c(g.col, np.int32)
    w = _c(g.w, np.uint32)
    p = _c(pids, np.int64)
    out = np.zeros((p.shape[0], T + 1), np.int32)
    _check(lib().or_walk_pids(g.n, g.m, _p(rp), _p(col), _p(w), T, seed, int(start_all),
                              _p(p), p.shape[0], _p(out)), "walk_pids")
    return out


def stream_counts(g, T: int, R: int, seed: int, queries, start_all: bool = False):
    """List lengths |P_v| for every v and dense counts c(q, v) for each query,
    streamed over all R paths without storing them (small graphs only:
    one n-array per query).  Returns (list_len uint64[n], counts uint32[nq][n])."""
    rp = _c(g.row_ptr, np.int32)
    col = _c(g.col, np.int32)
    w = _c(g.w, np.uint32)
    q = _c(queries, np.int32)
    ln = np.zeros(g.n, np.uint64)
    cnt = np.zeros((max(q.shape[0], 1), g.n), np.uint32)
    _check(lib().or_stream_counts(g.n, g.m, _p(rp), _p(col), _p(w), T, R, seed, int(start_all),
                                  _p(q), q.shape[0], _p(ln), _p(cnt)), "stream_counts")
    return ln, cnt[:q.shape[0]]


def topk_from_counts(counts, q: int, k: int):
    """Top-k of one query from its dense counts: the vertices v != q with
    c > 0, ordered by (c descending, id ascending), padded with (-1, 0)."""
    c = np.asarray(counts).astype(np.int64).copy()
    c[q] = 0
    cand = np.nonzero(c)[0]
    order = np.lexsort((cand, -c[cand]))[:k]
    ids = np.full(k, -1, np.int32)
    cnt = np.zeros(k, np.uint32)
    ids[:order.size] = cand[order]
    cnt[:order.size] = c[cand[order]]
    return ids, cnt, int(order.size)


def index(n: int, paths: np.ndarray):
    paths = _c(paths, np.int32)
    R, T1 = paths.shape
    inv_ptr = np.zeros(n + 1, np.int64)
    nnz = int(lib().or_index_ptr(n, T1 - 1, R, _p(paths), _p(inv_ptr)))
    inv_pid = np.zeros(max(nnz, 1), np.uint32)
    _check(lib().or_index_fill(n, T1 - 1, R, _p(paths), _p(inv_ptr), _p(inv_pid)), "index")
    return inv_ptr, inv_pid[:nnz]


def counts_dense(n: int, paths, inv_ptr, inv_pid, q: int) -> np.ndarray:
    paths = _c(paths, np.int32)
    out = np.zeros(n, np.uint32)
    ip = _c(inv_pid, np.uint32) if len(inv_pid) else np.zeros(1, np.uint32)
    _check(lib().or_counts_dense(n, paths.shape[1] - 1, _p(paths), _p(_c(inv_ptr, np.int64)),
                                 _p(ip), q, _p(out)), "counts")
    return out


def topk(n: int, paths, inv_ptr, inv_pid, queries, k: int):
    paths = _c(paths, np.int32)
    q = _c(queries, np.int32)
    nq = q.shape[0]
    ids = np.zeros((nq, k), np.int32)
    cnt = np.zeros((nq, k), np.uint32)
    ln = np.zeros(nq, np.int32)
    ip = _c(inv_pid, np.uint32) if len(inv_pid) else np.zeros(1, np.uint32)
    _check(lib().or_topk(n, paths.shape[1] - 1, _p(paths), _p(_c(inv_ptr, np.int64)),
                         _p(ip), _p(q), nq, k, _p(ids), _p(cnt), _p(ln)), "topk")
    return ids, cnt, ln


def features(n: int, paths, inv_ptr, inv_pid, D: int) -> np.ndarray:
    paths = _c(paths, np.int32)
    R = paths.shape[0]
    theta = np.zeros((n, D), np.float32)
    ip = _c(inv_pid, np.uint32) if len(inv_pid) else np.zeros(1, np.uint32)
    _check(lib().or_features(n, paths.shape[1] - 1, R, _p(paths), _p(_c(inv_ptr, np.int64)),
                             _p(ip), D, _p(theta)), "features")
    return theta


def dist2(a, b) -> float:
    a = _c(a, np.float32)
    b = _c(b, np.float32)
    return float(lib().or_dist2(_p(a), _p(b), a.shape[0]))


def knn(theta, queries, k: int):
    theta = _c(theta, np.float32)
    n, D = theta.shape
    q = _c(queries, np.int32)
    ids = np.zeros((q.shape[0], k), np.int32)
    dist = np.zeros((q.shape[0], k), np.float64)
    _check(lib().or_knn(n, D, _p(theta), _p(q), q.shape[0], k, _p(ids), _p(dist)), "knn")
    return ids, dist


def knn_cross(theta_q, theta_db, k: int):
    """Cross-graph kNN: row i of theta_q (a query's features in its own
    graph) against every row of theta_db (the other graph); no row is
    excluded."""
    tq = _c(theta_q, np.float32)
    tdb = _c(theta_db, np.float32)
    nq, D = tq.shape
    assert tdb.shape[1] == D
    ids = np.zeros((nq, k), np.int32)
    dist = np.zeros((nq, k), np.float64)
    _check(lib().or_knn_cross(D, nq, _p(tq), tdb.shape[0], _p(tdb), k, _p(ids), _p(dist)),
           "knn_cross")
    return ids, dist


def set_threads(n: int) -> None:
    """Thread count of the oracle's OpenMP loops (timing only)."""
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def sample_size(eps: float, c: float, delta: float, T: int) -> int:
    return int(lib().or_sample_size(eps, c, delta, T))
