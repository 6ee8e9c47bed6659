"""ctypes binding of libpanther.so (the C ABI of include/panther.h).

Only argument marshalling lives here: every step of the hot path runs in
the HIP kernels of the library.  The functions keep the C names; the
``Panther`` class bundles a context with numpy/torch conveniences.  Host
buffers are numpy arrays; device buffers are torch CUDA tensors (their
``data_ptr()`` is passed with PANTHER_MEM_DEVICE).

Importing this module does not load the library; the first call does, and
raises if ``libpanther.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpanther.so")

PANTHER_OK = 0
PANTHER_EINVAL = -1
PANTHER_ESTATE = -2
PANTHER_ENOMEM = -3
PANTHER_ERANGE = -4
PANTHER_EDEVICE = -5
PANTHER_MEM_HOST = 0
PANTHER_MEM_DEVICE = 1
PANTHER_START_ALL_VERTICES = 1
PANTHER_CHECK_SYMMETRIC = 2
PANTHER_FORM_PLAIN = 0
PANTHER_FORM_BATCHED = 1
PANTHER_PP_FP64 = 0
PANTHER_PP_BF16 = 1

EXPORTS = [
    "panther_create", "panther_destroy", "panther_last_error", "panther_load_graph",
    "panther_sample_paths", "panther_topk_similar", "panther_topk_similar_noalloc",
    "panther_topk_all", "panther_pp_topk",
    "panther_pp_topk_cross", "panther_pp_certified", "panther_pp_scanned",
    "panther_sample_size", "panther_set_option", "panther_get_paths", "panther_index_nnz",
    "panther_get_index", "panther_get_features", "panther_pp_stats", "panther_synchronize",
    "panther_stage_times", "panther_server_start", "panther_server_submit",
    "panther_server_poll", "panther_server_stats", "panther_server_memory",
    "panther_server_stop",
]

PANTHER_SERVER_KMAX = 256


class PantherResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("kind", ctypes.c_int32), ("query", ctypes.c_int32),
                ("k", ctypes.c_int32), ("len", ctypes.c_int32), ("status", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("latency_ms", ctypes.c_double),
                ("ids", ctypes.c_int32 * PANTHER_SERVER_KMAX),
                ("scores", ctypes.c_double * PANTHER_SERVER_KMAX)]

_lib = None


class PantherError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch bundles its own HIP runtime under the same soname as /opt/rocm's;
    # loading torch first makes both libraries share that single runtime
    # (device pointers and streams from torch are then valid here).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double)
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "panther_create": (ctypes.c_int, [ctypes.c_int, PP]),
        "panther_destroy": (None, [P]),
        "panther_last_error": (ctypes.c_char_p, [P]),
        "panther_load_graph": (ctypes.c_int, [P, i32, i64, P, P, P, ctypes.c_int, u32]),
        "panther_sample_paths": (ctypes.c_int, [P, i32, i64, u64]),
        "panther_topk_similar": (ctypes.c_int, [P, P, i64, i32, P, P, P, ctypes.c_int, P]),
        "panther_topk_similar_noalloc": (ctypes.c_int, [P, P, i64, i32, P, P, P, P]),
        "panther_pp_topk": (ctypes.c_int, [P, P, i64, i32, i32, P, P, ctypes.c_int, P]),
        "panther_topk_all": (ctypes.c_int, [P, i32, P, P, P, ctypes.c_int, P]),
        "panther_pp_topk_cross": (ctypes.c_int, [P, P, P, i64, i32, i32, P, P, ctypes.c_int, P]),
        "panther_sample_size": (i64, [dbl, dbl, dbl, i32]),
        "panther_set_option": (ctypes.c_int, [P, ctypes.c_char_p, i64]),
        "panther_get_paths": (ctypes.c_int, [P, P, ctypes.c_int]),
        "panther_index_nnz": (i64, [P]),
        "panther_get_index": (ctypes.c_int, [P, P, P, ctypes.c_int]),
        "panther_get_features": (ctypes.c_int, [P, i32, P, ctypes.c_int]),
        "panther_pp_stats": (ctypes.c_int, [P, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
        "panther_pp_certified": (ctypes.c_int, [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "panther_pp_scanned": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_double)]),
        "panther_synchronize": (ctypes.c_int, [P]),
        "panther_stage_times": (ctypes.c_int, [P, ctypes.POINTER(dbl)]),
        "panther_server_start": (ctypes.c_int, [P, i64, i32, i32, i32, PP]),
        "panther_server_submit": (ctypes.c_int, [P, i32, i32, i32, u64]),
        "panther_server_poll": (ctypes.c_int, [P, ctypes.POINTER(PantherResult), i32, i32]),
        "panther_server_stats": (ctypes.c_int, [P, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                                ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
        "panther_server_memory": (ctypes.c_int, [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "panther_server_stop": (ctypes.c_int, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


# ---------------------------------------------------------------------------
# C names
# ---------------------------------------------------------------------------
def panther_create(device_ordinal=0):
    h = ctypes.c_void_p()
    st = lib().panther_create(device_ordinal, ctypes.byref(h))
    if st != PANTHER_OK:
        raise PantherError(st, f"panther_create({device_ordinal}) failed")
    return h


def panther_destroy(ctx):
    lib().panther_destroy(ctx)


def panther_last_error(ctx):
    return lib().panther_last_error(ctx).decode()


def panther_load_graph(ctx, n, m, row_ptr, col, w, mem, flags=0):
    return lib().panther_load_graph(ctx, n, m, row_ptr, col, w, mem, flags)


def panther_sample_paths(ctx, T, R, seed):
    return lib().panther_sample_paths(ctx, T, R, seed)


def panther_topk_similar(ctx, queries, nq, k, out_ids, out_counts, out_len, mem, stream=None):
    return lib().panther_topk_similar(ctx, queries, nq, k, out_ids, out_counts, out_len, mem,
                                      stream)


def panther_topk_similar_noalloc(ctx, queries, nq, k, out_ids, out_counts, out_len,
                                 stream=None):
    return lib().panther_topk_similar_noalloc(ctx, queries, nq, k, out_ids, out_counts, out_len,
                                              stream)


def panther_pp_topk_cross(qctx, dbctx, queries, nq, D, k, out_ids, out_dist, mem, stream=None):
    return lib().panther_pp_topk_cross(qctx, dbctx, queries, nq, D, k, out_ids, out_dist, mem,
                                       stream)


def panther_topk_all(ctx, k, out_ids, out_counts, out_len, mem, stream=None):
    return lib().panther_topk_all(ctx, k, out_ids, out_counts, out_len, mem, stream)


def panther_pp_topk(ctx, queries, nq, D, k, out_ids, out_dist, mem, stream=None):
    return lib().panther_pp_topk(ctx, queries, nq, D, k, out_ids, out_dist, mem, stream)


def panther_sample_size(eps, c, delta, T):
    return lib().panther_sample_size(eps, c, delta, T)


def panther_set_option(ctx, key, value):
    return lib().panther_set_option(ctx, key.encode(), value)


def panther_get_paths(ctx, out, mem):
    return lib().panther_get_paths(ctx, out, mem)


def panther_index_nnz(ctx):
    return lib().panther_index_nnz(ctx)


def panther_get_index(ctx, inv_ptr, inv_pid, mem):
    return lib().panther_get_index(ctx, inv_ptr, inv_pid, mem)


def panther_get_features(ctx, D, out, mem):
    return lib().panther_get_features(ctx, D, out, mem)


def panther_pp_stats(ctx):
    a, b = ctypes.c_double(), ctypes.c_double()
    st = lib().panther_pp_stats(ctx, ctypes.byref(a), ctypes.byref(b))
    return st, a.value, b.value


def panther_synchronize(ctx):
    return lib().panther_synchronize(ctx)


def panther_stage_times(ctx):
    out = (ctypes.c_double * 5)()
    st = lib().panther_stage_times(ctx, out)
    return st, list(out)


def panther_server_start(ctx, mem_budget_bytes, max_batch, lanes, D):
    h = ctypes.c_void_p()
    st = lib().panther_server_start(ctx, mem_budget_bytes, max_batch, lanes, D, ctypes.byref(h))
    return st, h


def panther_server_submit(srv, kind, q, k, tag):
    return lib().panther_server_submit(srv, kind, q, k, tag)


def panther_server_poll(srv, results, max_results, timeout_us):
    return lib().panther_server_poll(srv, results, max_results, timeout_us)


def panther_server_stats(srv):
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n = ctypes.c_int64()
    st = lib().panther_server_stats(srv, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                    ctypes.byref(n))
    return st, a.value, b.value, c.value, n.value


def panther_server_memory(srv):
    share, peak = ctypes.c_int64(), ctypes.c_int64()
    st = lib().panther_server_memory(srv, ctypes.byref(share), ctypes.byref(peak))
    return st, share.value, peak.value


def panther_server_stop(srv):
    return lib().panther_server_stop(srv)


class Server:
    """Continuous-batching server over a context's resident state."""

    def __init__(self, panther, mem_budget_bytes, max_batch=256, lanes=3, D=50):
        self.P = panther
        st, self.h = panther_server_start(panther.h, mem_budget_bytes, max_batch, lanes, D)
        if st != PANTHER_OK:
            raise PantherError(st, panther_last_error(panther.h))
        self._buf = (PantherResult * 1024)()

    def submit(self, kind, q, k, tag):
        return panther_server_submit(self.h, kind, q, k, tag)

    def poll(self, timeout_us=1000):
        n = panther_server_poll(self.h, self._buf, 1024, timeout_us)
        if n < 0:
            raise PantherError(n, "poll failed")
        out = []
        for i in range(n):
            r = self._buf[i]
            out.append(dict(tag=r.tag, kind=r.kind, query=r.query, k=r.k, len=r.len,
                            status=r.status, latency_ms=r.latency_ms,
                            ids=np.ctypeslib.as_array(r.ids)[:r.k].copy(),
                            scores=np.ctypeslib.as_array(r.scores)[:r.k].copy()))
        return out

    def stats(self):
        st, p50, p99, qps, done = panther_server_stats(self.h)
        return dict(status=st, p50_ms=p50, p99_ms=p99, qps=qps, completed=done)

    def memory(self):
        st, share, peak = panther_server_memory(self.h)
        return dict(status=st, lane_share_bytes=share, peak_lane_bytes=peak)

    def stop(self):
        if self.h:
            st = panther_server_stop(self.h)
            self.h = None
            return st
        return PANTHER_OK


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------
def _buf(x, dtype):
    """(pointer, mem, keepalive) for a numpy array or a torch CUDA tensor."""
    if isinstance(x, np.ndarray):
        a = np.ascontiguousarray(x, dtype=dtype)
        return a.ctypes.data_as(ctypes.c_void_p), PANTHER_MEM_HOST, a
    import torch

    if isinstance(x, torch.Tensor):
        want = {np.int32: torch.int32, np.uint32: torch.uint32, np.int64: torch.int64,
                np.float32: torch.float32, np.float64: torch.float64}[dtype]
        if x.dtype != want or not x.is_contiguous():
            raise TypeError(f"expected a contiguous {want} tensor")
        mem = PANTHER_MEM_DEVICE if x.is_cuda else PANTHER_MEM_HOST
        return ctypes.c_void_p(x.data_ptr()), mem, x
    raise TypeError(type(x))


class Panther:
    """One context on one GPU."""

    def __init__(self, device=0):
        self.h = panther_create(device)

    def close(self):
        if self.h:
            panther_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != PANTHER_OK:
            raise PantherError(st, panther_last_error(self.h))
        return st

    def set_option(self, key, value):
        return self._check(panther_set_option(self.h, key, int(value)))

    def load_graph(self, g=None, *, n=None, row_ptr=None, col=None, w=None, flags=0):
        if g is not None:
            n, row_ptr, col, w = g.n, g.row_ptr, g.col, g.w
        rp, mem, k1 = _buf(row_ptr, np.int32)
        cp, mem2, k2 = _buf(col, np.int32)
        wp, mem3, k3 = _buf(w, np.uint32)
        if not (mem == mem2 == mem3):
            raise ValueError("row_ptr, col and w must live in the same memory")
        m = int(col.shape[0])
        return self._check(panther_load_graph(self.h, n, m, rp, cp, wp, mem, flags))

    def sample_paths(self, T, R, seed):
        self._check(panther_sample_paths(self.h, T, R, seed))
        self._TR = (T, R)

    def topk(self, queries, k, out=None, stream=None):
        """Host queries -> host numpy (ids, counts, len); device tensors -> in place."""
        if isinstance(queries, np.ndarray):
            q = np.ascontiguousarray(queries, np.int32)
            nq = q.shape[0]
            ids = np.empty((nq, k), np.int32)
            cnt = np.empty((nq, k), np.uint32)
            ln = np.empty(nq, np.int32)
            self._check(panther_topk_similar(
                self.h, q.ctypes.data_as(ctypes.c_void_p), nq, k,
                ids.ctypes.data_as(ctypes.c_void_p), cnt.ctypes.data_as(ctypes.c_void_p),
                ln.ctypes.data_as(ctypes.c_void_p), PANTHER_MEM_HOST, stream))
            return ids, cnt, ln
        ids, cnt, ln = out
        qp, _, _ = _buf(queries, np.int32)
        self._check(panther_topk_similar(
            self.h, qp, int(queries.shape[0]), k, _buf(ids, np.int32)[0],
            _buf(cnt, np.uint32)[0], _buf(ln, np.int32)[0], PANTHER_MEM_DEVICE, stream))
        return out

    def pp_topk_cross(self, db, queries, D, k):
        """Panther++ of this context's vertices `queries` against every vertex
        of the context `db` (another graph); host numpy (ids, dist)."""
        q = np.ascontiguousarray(queries, np.int32)
        nq = q.shape[0]
        ids = np.empty((nq, k), np.int32)
        dist = np.empty((nq, k), np.float64)
        st = panther_pp_topk_cross(self.h, db.h, q.ctypes.data_as(ctypes.c_void_p), nq, D, k,
                                   ids.ctypes.data_as(ctypes.c_void_p),
                                   dist.ctypes.data_as(ctypes.c_void_p), PANTHER_MEM_HOST, None)
        db._check(st)
        return ids, dist

    def topk_all(self, n, k, out=None, stream=None):
        """Top-k of every vertex 0..n-1: host numpy (ids, counts, len), or into
        the device tensors of `out`."""
        if out is None:
            ids = np.empty((n, k), np.int32)
            cnt = np.empty((n, k), np.uint32)
            ln = np.empty(n, np.int32)
            self._check(panther_topk_all(
                self.h, k, ids.ctypes.data_as(ctypes.c_void_p), cnt.ctypes.data_as(ctypes.c_void_p),
                ln.ctypes.data_as(ctypes.c_void_p), PANTHER_MEM_HOST, stream))
            return ids, cnt, ln
        ids, cnt, ln = out
        self._check(panther_topk_all(self.h, k, _buf(ids, np.int32)[0], _buf(cnt, np.uint32)[0],
                                     _buf(ln, np.int32)[0], PANTHER_MEM_DEVICE, stream))
        return out

    def pp_topk(self, queries, D, k, out=None, stream=None):
        if isinstance(queries, np.ndarray):
            q = np.ascontiguousarray(queries, np.int32)
            nq = q.shape[0]
            ids = np.empty((nq, k), np.int32)
            dist = np.empty((nq, k), np.float64)
            self._check(panther_pp_topk(
                self.h, q.ctypes.data_as(ctypes.c_void_p), nq, D, k,
                ids.ctypes.data_as(ctypes.c_void_p), dist.ctypes.data_as(ctypes.c_void_p),
                PANTHER_MEM_HOST, stream))
            return ids, dist
        ids, dist = out
        qp, _, _ = _buf(queries, np.int32)
        self._check(panther_pp_topk(self.h, qp, int(queries.shape[0]), D, k,
                                    _buf(ids, np.int32)[0], _buf(dist, np.float64)[0],
                                    PANTHER_MEM_DEVICE, stream))
        return out

    def paths(self):
        nnz = self.nnz()  # raises ESTATE without paths
        del nnz
        T, R = self._TR
        out = np.empty((R, T + 1), np.int32)
        self._check(panther_get_paths(self.h, out.ctypes.data_as(ctypes.c_void_p),
                                      PANTHER_MEM_HOST))
        return out

    def paths_device(self):
        """The paths as a device tensor int32[R][T+1]."""
        import torch

        T, R = self._TR
        out = torch.empty((R, T + 1), dtype=torch.int32, device="cuda")
        self._check(panther_get_paths(self.h, ctypes.c_void_p(out.data_ptr()), PANTHER_MEM_DEVICE))
        return out

    def index_device(self, n):
        """The inverted index as device tensors (int64[n+1], int32 view of
        uint32[nnz])."""
        import torch

        nnz = self.nnz()
        ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        pid = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
        self._check(panther_get_index(self.h, ctypes.c_void_p(ptr.data_ptr()),
                                      ctypes.c_void_p(pid.data_ptr()), PANTHER_MEM_DEVICE))
        return ptr, pid[:nnz]

    def nnz(self):
        v = panther_index_nnz(self.h)
        if v < 0:
            raise PantherError(v, "no index")
        return v

    def index(self, n):
        nnz = self.nnz()
        ptr = np.empty(n + 1, np.int64)
        pid = np.empty(max(nnz, 1), np.uint32)
        self._check(panther_get_index(self.h, ptr.ctypes.data_as(ctypes.c_void_p),
                                      pid.ctypes.data_as(ctypes.c_void_p), PANTHER_MEM_HOST))
        return ptr, pid[:nnz]

    def features(self, n, D):
        out = np.empty((n, D), np.float32)
        self._check(panther_get_features(self.h, D, out.ctypes.data_as(ctypes.c_void_p),
                                         PANTHER_MEM_HOST))
        return out

    def pp_stats(self):
        st, err, rec = panther_pp_stats(self.h)
        self._check(st)
        return err, rec

    def pp_certified(self):
        """(queries, recomputed) of the last BF16-form Panther++ call."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().panther_pp_certified(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value


    def pp_scanned(self):
        """Fraction of the (query, row) products the last BF16-form pool pass
        computed (norm-band pruning)."""
        f = ctypes.c_double()
        self._check(lib().panther_pp_scanned(self.h, ctypes.byref(f)))
        return f.value

    def stage_times(self):
        """dict of stage -> device milliseconds (option "timing" must be on)."""
        st, v = panther_stage_times(self.h)
        self._check(st)
        return dict(zip(("walk", "index", "topk", "features", "pp"), v))

    def synchronize(self):
        return self._check(panther_synchronize(self.h))
