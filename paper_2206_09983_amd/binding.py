"""Thin ctypes binding of the C ABI in include/mnemonic.h.

Argument marshalling only: every step of the matcher runs in the HIP library
``libmnemonic.so`` built next to this file. There is no fallback: if the
library is missing, loading fails with an error that says how to build it.
Function names are the ABI's; ``Matcher`` is a small convenience wrapper.
Device inputs may be torch tensors (their data pointers are passed as is).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmnemonic.so")

ISO = 0
HOMO = 1
F_EMIT = 1
F_TIMING = 2
F_AUTOTUNE = 4
F_INDEX_ONLY = 8
F_SORT = 16
F_TREE_FILTER = 32
SCHED_STATIC = 0
SCHED_LEARNED = 1
SCHED_FIXED = 2
MLP_IN = 24
MLP_HIDDEN = 64
MLP_WEIGHTS = 5825
MAX_ORDERS = 4

ERRORS = {
    -1: "MNEMONIC_E_ARG", -2: "MNEMONIC_E_QUERY", -3: "MNEMONIC_E_VERTEX", -4: "MNEMONIC_E_LABEL",
    -5: "MNEMONIC_E_TS_ORDER", -6: "MNEMONIC_E_BAD_DELETE", -7: "MNEMONIC_E_OOM",
    -8: "MNEMONIC_E_CAPACITY", -9: "MNEMONIC_E_HIP", -10: "MNEMONIC_E_LIMIT",
}
EXPORTS = ["mnemonic_create", "mnemonic_apply_batch", "mnemonic_get_result", "mnemonic_copy_keys",
           "mnemonic_get_stats", "mnemonic_last_error", "mnemonic_destroy", "mnemonic_set_scheduler",
           "mnemonic_query_orders", "mnemonic_set_trace", "mnemonic_get_trace", "mnemonic_mlp_predict",
           "mnemonic_mlp_grad", "mnemonic_mlp_adam", "mnemonic_set_queries", "mnemonic_fail_alloc_after",
           "mnemonic_apply_batch_noalloc"]

_u8p = C.POINTER(C.c_uint8)
_u32p = C.POINTER(C.c_uint32)
_u64p = C.POINTER(C.c_uint64)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)


class mnemonic_graph(C.Structure):
    _fields_ = [("n_vertices", C.c_uint32), ("n_elabels", C.c_uint32), ("vlabel_mask", _u64p),
                ("n_edges", C.c_uint64), ("src", _u32p), ("dst", _u32p), ("elabel", _u8p), ("ts", _i64p)]


class mnemonic_query(C.Structure):
    _fields_ = [("n_qv", C.c_uint32), ("qv_require", _u64p), ("n_qe", C.c_uint32), ("qsrc", _u32p),
                ("qdst", _u32p), ("qelabel", _i32p), ("sem", C.c_int), ("qtorder", _i32p)]


class mnemonic_edges(C.Structure):
    _fields_ = [("n", C.c_uint64), ("src", _u32p), ("dst", _u32p), ("elabel", _u8p), ("ts", _i64p),
                ("on_device", C.c_uint32)]


class mnemonic_options(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("out_capacity", C.c_uint64), ("rows_per_level", C.c_uint64)]


class mnemonic_result(C.Structure):
    _fields_ = [("n_new", C.c_uint64), ("n_expired", C.c_uint64), ("dig_new", C.c_uint64 * 2),
                ("dig_expired", C.c_uint64 * 2), ("new_keys", _u64p), ("expired_keys", _u64p),
                ("n_qe", C.c_uint32)]


class mnemonic_stats(C.Structure):
    _fields_ = [("n_live_edges", C.c_uint64), ("slot_high_water", C.c_uint64), ("seeds", C.c_uint64 * 2),
                ("entries_scanned", C.c_uint64 * 2), ("probe_words", C.c_uint64 * 2),
                ("range_probe_words", C.c_uint64 * 2), ("key_reads", C.c_uint64 * 2),
                ("tuples", C.c_uint64 * 2), ("tuple_words", C.c_uint64 * 2), ("vf_reads", C.c_uint64 * 2),
                ("frontier_rows", C.c_uint64 * 2), ("expand_launches", C.c_uint64 * 2),
                ("expand_tile", C.c_uint64), ("ms_expand", C.c_double * 2), ("ms_enumerate", C.c_double * 2),
                ("ms_batch", C.c_double), ("reruns", C.c_uint64 * 2), ("rerun_causes", C.c_uint64 * 2),
                ("vf_rejects", C.c_uint64 * 2), ("key_capacity", C.c_uint64), ("key_lo", C.c_uint64),
                ("allocations", C.c_uint64), ("ms_alloc", C.c_double), ("tree_cleared", C.c_uint64)]


class MnemonicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code
        self.name = ERRORS.get(code, "?")


_LIB = None


def load():
    """Loads libmnemonic.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmnemonic.so not found at %s; build it with "
                           "`python -m paper_2206_09983_amd.build`" % LIB_PATH)
    # torch ships its own HIP runtime whose soname equals the system one's.
    # Loading torch first makes the library bind to that already-loaded
    # runtime; the other order leaves two HIP runtimes in one process and
    # torch then finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.mnemonic_create.restype = C.c_int
    L.mnemonic_create.argtypes = [C.POINTER(mnemonic_graph), C.POINTER(mnemonic_query), C.c_uint32,
                                  C.POINTER(mnemonic_options), vp, C.POINTER(vp)]
    L.mnemonic_apply_batch.restype = C.c_int
    L.mnemonic_apply_batch.argtypes = [vp, C.POINTER(mnemonic_edges), _u64p, C.c_uint64, _u64p]
    L.mnemonic_apply_batch_noalloc.restype = C.c_int
    L.mnemonic_apply_batch_noalloc.argtypes = [vp, C.POINTER(mnemonic_edges), _u64p, C.c_uint64, _u64p]
    L.mnemonic_get_result.restype = C.c_int
    L.mnemonic_get_result.argtypes = [vp, C.c_uint32, C.POINTER(mnemonic_result)]
    L.mnemonic_copy_keys.restype = C.c_int
    L.mnemonic_copy_keys.argtypes = [vp, C.c_uint32, C.c_int, _u64p, C.c_uint64, _u64p]
    L.mnemonic_get_stats.restype = C.c_int
    L.mnemonic_get_stats.argtypes = [vp, C.POINTER(mnemonic_stats)]
    L.mnemonic_last_error.restype = C.c_char_p
    L.mnemonic_last_error.argtypes = [vp]
    L.mnemonic_destroy.restype = None
    L.mnemonic_destroy.argtypes = [vp]
    L.mnemonic_set_queries.restype = C.c_int
    L.mnemonic_set_queries.argtypes = [vp, C.POINTER(mnemonic_query), C.c_uint32]
    fp = C.POINTER(C.c_float)
    L.mnemonic_set_scheduler.restype = C.c_int
    L.mnemonic_set_scheduler.argtypes = [vp, C.c_int, fp]
    L.mnemonic_query_orders.restype = C.c_int
    L.mnemonic_query_orders.argtypes = [vp, C.c_uint32, C.c_uint32, _u32p]
    L.mnemonic_set_trace.restype = C.c_int
    L.mnemonic_set_trace.argtypes = [vp, C.c_uint64]
    L.mnemonic_get_trace.restype = C.c_int
    L.mnemonic_get_trace.argtypes = [vp, C.c_int, _u64p, _u64p, fp, _u64p, C.c_uint64]
    L.mnemonic_mlp_predict.restype = C.c_int
    L.mnemonic_mlp_predict.argtypes = [vp, vp, C.c_uint64, C.c_int, vp, vp]
    L.mnemonic_mlp_grad.restype = C.c_int
    L.mnemonic_mlp_grad.argtypes = [vp, vp, vp, vp, C.c_uint64, C.c_uint64, vp, vp, vp]
    L.mnemonic_mlp_adam.restype = C.c_int
    L.mnemonic_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_float, C.c_uint32, vp]
    L.mnemonic_fail_alloc_after.restype = None
    L.mnemonic_fail_alloc_after.argtypes = [C.c_uint64]
    _LIB = L
    return L


def _ptr(a, ct):
    """Pointer to a numpy array's data, or a torch tensor's device data."""
    if a is None:
        return C.cast(None, C.POINTER(ct))
    if hasattr(a, "data_ptr"):
        return C.cast(C.c_void_p(a.data_ptr()), C.POINTER(ct))
    return a.ctypes.data_as(C.POINTER(ct))


def _check(rc, ctx):
    if rc != 0:
        raise MnemonicError(rc, mnemonic_last_error(ctx))


def _queries(queries, arr):
    """mnemonic_query array of query dicts (arr keeps the arrays alive)."""
    qs = (mnemonic_query * len(queries))()
    for i, q in enumerate(queries):
        qs[i].n_qv = int(q["n_qv"])
        qs[i].qv_require = _ptr(arr(q["vreq"], np.uint64), C.c_uint64)
        qs[i].n_qe = len(q["qsrc"])
        qs[i].qsrc = _ptr(arr(q["qsrc"], np.uint32), C.c_uint32)
        qs[i].qdst = _ptr(arr(q["qdst"], np.uint32), C.c_uint32)
        qs[i].qelabel = _ptr(arr(q["qlabel"], np.int32), C.c_int32)
        qs[i].sem = int(q["sem"])
        qs[i].qtorder = _ptr(None if q.get("rank") is None else arr(q["rank"], np.int32), C.c_int32)
    return qs


# ------------------------------------------------------------------- ABI calls
def mnemonic_create(graph, queries, flags=F_EMIT, out_capacity=0, stream=None, n_elabels=0, rows_per_level=0):
    """graph/queries: dicts as produced by paper_2206_09983_amd.synth. Returns the context."""
    L = load()
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return a

    g = mnemonic_graph()
    g.n_vertices = int(graph["n_vertices"])
    g.n_elabels = int(n_elabels or graph.get("n_elabels", 0))
    g.vlabel_mask = _ptr(arr(graph["vlabel_mask"], np.uint64), C.c_uint64)
    g.n_edges = len(graph["src"])
    g.src = _ptr(arr(graph["src"], np.uint32), C.c_uint32)
    g.dst = _ptr(arr(graph["dst"], np.uint32), C.c_uint32)
    g.elabel = _ptr(arr(graph["elabel"], np.uint8), C.c_uint8)
    g.ts = _ptr(arr(graph["ts"], np.int64), C.c_int64)
    qs = _queries(queries, arr)
    opt = mnemonic_options(int(flags), int(out_capacity), int(rows_per_level))
    ctx = C.c_void_p()
    rc = L.mnemonic_create(C.byref(g), qs, len(queries), C.byref(opt),
                           C.c_void_p(stream) if stream else None, C.byref(ctx))
    if rc != 0:
        raise MnemonicError(rc, L.mnemonic_last_error(None).decode())
    return ctx


def mnemonic_apply_batch(ctx, batch, no_alloc=False):
    """batch: dict with src, dst, elabel, ts, del_keys as numpy arrays (host) or
    torch device tensors (int32/uint8/int64; read in place). Returns the first
    inserted key. no_alloc: call mnemonic_apply_batch_noalloc instead."""
    L = load()
    src = batch["src"]
    on_dev = hasattr(src, "data_ptr") and getattr(src, "is_cuda", False)
    if on_dev:
        s, d, l, t, k = src, batch["dst"], batch["elabel"], batch["ts"], batch.get("del_keys")
    else:
        s = np.ascontiguousarray(batch["src"], dtype=np.uint32)
        d = np.ascontiguousarray(batch["dst"], dtype=np.uint32)
        l = np.ascontiguousarray(batch["elabel"], dtype=np.uint8)
        t = np.ascontiguousarray(batch["ts"], dtype=np.int64)
        k = np.ascontiguousarray(batch.get("del_keys", np.zeros(0)), dtype=np.uint64)
    n = int(s.shape[0])
    nd = 0 if k is None else int(k.shape[0])
    e = mnemonic_edges(n, _ptr(s, C.c_uint32), _ptr(d, C.c_uint32), _ptr(l, C.c_uint8),
                       _ptr(t, C.c_int64), 1 if on_dev else 0)
    first = C.c_uint64(0)
    fn = L.mnemonic_apply_batch_noalloc if no_alloc else L.mnemonic_apply_batch
    rc = fn(ctx, C.byref(e), _ptr(k, C.c_uint64) if nd else None, nd, C.byref(first))
    _check(rc, ctx)
    return int(first.value)


def mnemonic_get_result(ctx, query):
    r = mnemonic_result()
    _check(load().mnemonic_get_result(ctx, int(query), C.byref(r)), ctx)
    return {"n_new": int(r.n_new), "n_expired": int(r.n_expired),
            "dig_new": (int(r.dig_new[0]), int(r.dig_new[1])),
            "dig_expired": (int(r.dig_expired[0]), int(r.dig_expired[1])),
            "new_keys": C.cast(r.new_keys, C.c_void_p).value,
            "expired_keys": C.cast(r.expired_keys, C.c_void_p).value, "n_qe": int(r.n_qe)}


def mnemonic_copy_keys(ctx, query, expired=False):
    """Copies one query's new (or expired) tuples to a (n, n_qe) uint64 array."""
    L = load()
    res = mnemonic_get_result(ctx, query)
    n = res["n_expired"] if expired else res["n_new"]
    out = np.zeros((n, res["n_qe"]), dtype=np.uint64)
    needed = C.c_uint64(0)
    rc = L.mnemonic_copy_keys(ctx, int(query), 1 if expired else 0, _ptr(out, C.c_uint64), n,
                              C.byref(needed))
    _check(rc, ctx)
    return out


def mnemonic_get_stats(ctx):
    st = mnemonic_stats()
    _check(load().mnemonic_get_stats(ctx, C.byref(st)), ctx)
    return {f: (list(getattr(st, f)) if not isinstance(getattr(st, f), (int, float)) else getattr(st, f))
            for f, _ in mnemonic_stats._fields_}


def mnemonic_last_error(ctx):
    return load().mnemonic_last_error(ctx).decode()


def mnemonic_destroy(ctx):
    if ctx:
        load().mnemonic_destroy(ctx)


def mnemonic_set_queries(ctx, queries):
    """Replaces the context's query set (between batches)."""
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return a

    qs = _queries(queries, arr)
    _check(load().mnemonic_set_queries(ctx, qs, len(queries)), ctx)


def mnemonic_set_scheduler(ctx, mode, weights=None):
    """mode: SCHED_STATIC, SCHED_LEARNED (weights: 5,825 floats) or SCHED_FIXED + v."""
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    if w is not None and w.size != MLP_WEIGHTS:
        raise ValueError("the network has %d weights" % MLP_WEIGHTS)
    _check(load().mnemonic_set_scheduler(ctx, int(mode), _ptr(w, C.c_float)), ctx)


def mnemonic_query_orders(ctx, query, j):
    n = C.c_uint32(0)
    _check(load().mnemonic_query_orders(ctx, int(query), int(j), C.byref(n)), ctx)
    return int(n.value)


def mnemonic_set_trace(ctx, capacity):
    _check(load().mnemonic_set_trace(ctx, int(capacity)), ctx)


def mnemonic_get_trace(ctx, phase, with_x=True):
    """Last batch's trace of one phase: codes (n,), x (n, 4, 24) float32 (None
    unless with_x), work (n,)."""
    L = load()
    n = C.c_uint64(0)
    _check(L.mnemonic_get_trace(ctx, int(phase), C.byref(n), None, None, None, 0), ctx)
    m = int(n.value)
    codes = np.zeros(m, dtype=np.uint64)
    x = np.zeros((m, MAX_ORDERS, MLP_IN), dtype=np.float32) if with_x else None
    work = np.zeros(m, dtype=np.uint64)
    _check(L.mnemonic_get_trace(ctx, int(phase), C.byref(n), _ptr(codes, C.c_uint64), _ptr(x, C.c_float),
                                _ptr(work, C.c_uint64), m), ctx)
    return {"codes": codes, "x": x, "work": work}


def mnemonic_fail_alloc_after(n):
    """Test hook: the n-th device allocation from now fails (0 disarms)."""
    load().mnemonic_fail_alloc_after(int(n))


def _dev(t):
    """Device address of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def _mlp_check(rc, what):
    if rc != 0:
        raise MnemonicError(rc, what + " launch failed")


def mnemonic_mlp_predict(w, x, y, bf16=False, stream=None):
    """Device tensors: w (5825,), x (n, 24), y (n,) float32."""
    _mlp_check(load().mnemonic_mlp_predict(_dev(w), _dev(x), int(x.shape[0]), 1 if bf16 else 0, _dev(y), stream),
               "mnemonic_mlp_predict")


def mnemonic_mlp_grad(w, x, target, grad, loss, idx=None, off=0, m=None, stream=None):
    """Adds the MSE gradient over samples idx[off:off+m] (or off:off+m) to grad and the loss to loss[0]."""
    m = int(x.shape[0] if m is None else m)
    _mlp_check(load().mnemonic_mlp_grad(_dev(w), _dev(x), _dev(target), _dev(idx), int(off), m, _dev(grad),
                                        _dev(loss), stream), "mnemonic_mlp_grad")


def mnemonic_mlp_adam(w, m1, m2, grad, lr, step, stream=None):
    _mlp_check(load().mnemonic_mlp_adam(_dev(w), _dev(m1), _dev(m2), _dev(grad), float(lr), int(step), stream),
               "mnemonic_mlp_adam")


class Matcher:
    """Owns one context: create on construction, destroy on close."""

    def __init__(self, graph, queries, flags=F_EMIT, out_capacity=0, stream=None, n_elabels=0, rows_per_level=0):
        self.n_q = len(queries)
        self.ctx = mnemonic_create(graph, queries, flags, out_capacity, stream, n_elabels, rows_per_level)

    def apply_batch(self, batch, no_alloc=False):
        return mnemonic_apply_batch(self.ctx, batch, no_alloc)

    def result(self, q):
        return mnemonic_get_result(self.ctx, q)

    def keys(self, q, expired=False):
        return mnemonic_copy_keys(self.ctx, q, expired)

    def stats(self):
        return mnemonic_get_stats(self.ctx)

    def set_queries(self, queries):
        mnemonic_set_queries(self.ctx, queries)
        self.n_q = len(queries)

    def set_scheduler(self, mode, weights=None):
        mnemonic_set_scheduler(self.ctx, mode, weights)

    def orders(self, q, j):
        return mnemonic_query_orders(self.ctx, q, j)

    def set_trace(self, capacity):
        mnemonic_set_trace(self.ctx, capacity)

    def trace(self, phase, with_x=True):
        return mnemonic_get_trace(self.ctx, phase, with_x)

    def close(self):
        if self.ctx:
            mnemonic_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
