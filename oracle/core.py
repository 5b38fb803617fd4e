"""ctypes wrapper of the C oracle (test infrastructure only).

``Oracle`` mirrors the batch phases of Algorithm 1: ``apply_batch`` runs the
insert phase, then the delete phase, and keeps per query the sorted lists of
new and expired embeddings (tuples of edge keys in query-edge index order).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None
SEED_A = 0x243F6A8885A308D3
SEED_B = 0x13198A2E03707344


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        vp, u64, u32, i64, i32 = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int64, C.c_int
        P = C.POINTER
        L.orc_create.restype = vp
        L.orc_create.argtypes = [u32, P(u64), u64, P(u32), P(u32), P(C.c_uint8), P(i64)]
        L.orc_destroy.argtypes = [vp]
        L.orc_set_limit.argtypes = [vp, u64]
        L.orc_add_query.restype = i32
        L.orc_add_query.argtypes = [vp, u32, P(u64), u32, P(u32), P(u32), P(C.c_int32), i32]
        L.orc_set_temporal.restype = i32
        L.orc_set_temporal.argtypes = [vp, u32, P(C.c_int32)]
        L.orc_insert.restype = i64
        L.orc_insert.argtypes = [vp, u64, P(u32), P(u32), P(C.c_uint8), P(i64), i32]
        L.orc_mark.restype = i32
        L.orc_mark.argtypes = [vp, u64, P(u64)]
        L.orc_unmark.argtypes = [vp, u64, P(u64)]
        L.orc_delete.restype = i32
        L.orc_delete.argtypes = [vp, u64, P(u64), i32]
        L.orc_apply_batch.restype = i32
        L.orc_apply_batch.argtypes = [vp, u64, P(u32), P(u32), P(C.c_uint8), P(i64), u64, P(u64)]
        L.orc_count.restype = u64
        L.orc_count.argtypes = [vp, u32, i32]
        L.orc_keys.restype = P(u64)
        L.orc_keys.argtypes = [vp, u32, i32]
        L.orc_overflow.restype = u64
        L.orc_overflow.argtypes = [vp, u32, i32]
        L.orc_digest.argtypes = [vp, u32, i32, P(u64)]
        L.orc_static.restype = u64
        L.orc_static.argtypes = [vp, u32]
        L.orc_seed.restype = u64
        L.orc_seed.argtypes = [vp, u32, u64, u32, i32]
        L.orc_aux_keys.restype = P(u64)
        L.orc_aux_keys.argtypes = [vp]
        L.orc_aux_overflow.restype = u64
        L.orc_aux_overflow.argtypes = [vp]
        L.orc_aux_digest.argtypes = [vp, u32, P(u64)]
        L.orc_mix64.restype = u64
        L.orc_mix64.argtypes = [u64]
        L.orc_tuple_hash.restype = u64
        L.orc_tuple_hash.argtypes = [u64, u32, P(u64), u32]
        L.orc_n_keys.restype = u64
        L.orc_n_keys.argtypes = [vp]
        L.orc_n_live.restype = u64
        L.orc_n_live.argtypes = [vp]
        _LIB = L
    return _LIB


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def mix64(x):
    return int(lib().orc_mix64(C.c_uint64(int(x) & 0xFFFFFFFFFFFFFFFF)))


def tuple_hash(seed, qidx, keys):
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    return int(lib().orc_tuple_hash(seed, qidx, _p(k, C.c_uint64), len(k)))


class Oracle:
    """Incremental matcher over one data graph and a set of queries."""

    def __init__(self, graph, queries, limit=0):
        L = lib()
        g = graph
        self._keep = [np.ascontiguousarray(g["vlabel_mask"], dtype=np.uint64),
                      np.ascontiguousarray(g["src"], dtype=np.uint32),
                      np.ascontiguousarray(g["dst"], dtype=np.uint32),
                      np.ascontiguousarray(g["elabel"], dtype=np.uint8),
                      np.ascontiguousarray(g["ts"], dtype=np.int64)]
        vm, s, d, l, t = self._keep
        self.h = L.orc_create(int(g["n_vertices"]), _p(vm, C.c_uint64), len(s), _p(s, C.c_uint32),
                              _p(d, C.c_uint32), _p(l, C.c_uint8), _p(t, C.c_int64))
        if not self.h:
            raise MemoryError("oracle create failed")
        self.n_qe = []
        for q in queries:
            vr = np.ascontiguousarray(q["vreq"], dtype=np.uint64)
            qs = np.ascontiguousarray(q["qsrc"], dtype=np.uint32)
            qd = np.ascontiguousarray(q["qdst"], dtype=np.uint32)
            ql = np.ascontiguousarray(q["qlabel"], dtype=np.int32)
            r = L.orc_add_query(self.h, int(q["n_qv"]), _p(vr, C.c_uint64), len(qs), _p(qs, C.c_uint32),
                                _p(qd, C.c_uint32), _p(ql, C.c_int32), int(q["sem"]))
            if r < 0:
                raise ValueError("query rejected by oracle: %r" % (q.get("name"),))
            if q.get("rank") is not None:  # temporal order on the query edges
                rk = np.ascontiguousarray(q["rank"], dtype=np.int32)
                if len(rk) != len(qs) or L.orc_set_temporal(self.h, r, _p(rk, C.c_int32)) < 0:
                    raise ValueError("bad temporal ranks")
                self._keep.append(rk)
            self.n_qe.append(len(qs))
        if limit:
            L.orc_set_limit(self.h, int(limit))

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- phases ---------------------------------------------------------
    def apply_batch(self, batch):
        s = np.ascontiguousarray(batch["src"], dtype=np.uint32)
        d = np.ascontiguousarray(batch["dst"], dtype=np.uint32)
        l = np.ascontiguousarray(batch["elabel"], dtype=np.uint8)
        t = np.ascontiguousarray(batch["ts"], dtype=np.int64)
        k = np.ascontiguousarray(batch.get("del_keys", np.zeros(0)), dtype=np.uint64)
        r = lib().orc_apply_batch(self.h, len(s), _p(s, C.c_uint32), _p(d, C.c_uint32), _p(l, C.c_uint8),
                                  _p(t, C.c_int64), len(k), _p(k, C.c_uint64))
        if r != 0:
            raise ValueError("oracle rejected the batch")

    def insert(self, batch, enumerate=True):
        s = np.ascontiguousarray(batch["src"], dtype=np.uint32)
        d = np.ascontiguousarray(batch["dst"], dtype=np.uint32)
        l = np.ascontiguousarray(batch["elabel"], dtype=np.uint8)
        t = np.ascontiguousarray(batch["ts"], dtype=np.int64)
        r = lib().orc_insert(self.h, len(s), _p(s, C.c_uint32), _p(d, C.c_uint32), _p(l, C.c_uint8),
                             _p(t, C.c_int64), int(bool(enumerate)))
        if r < 0:
            raise ValueError("oracle rejected the insertions")
        return int(r)

    def delete(self, keys, enumerate=True):
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        if lib().orc_delete(self.h, len(k), _p(k, C.c_uint64), int(bool(enumerate))) != 0:
            raise ValueError("oracle rejected the deletions")

    def mark(self, keys):
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        if lib().orc_mark(self.h, len(k), _p(k, C.c_uint64)) != 0:
            raise ValueError("bad deletion keys")

    def unmark(self, keys):
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        lib().orc_unmark(self.h, len(k), _p(k, C.c_uint64))

    # -- results --------------------------------------------------------
    def result(self, q, expired=False):
        """Sorted (n, n_qe) uint64 array of new (or expired) embeddings."""
        L = lib()
        ph = 1 if expired else 0
        n = int(L.orc_count(self.h, q, ph))
        m = self.n_qe[q]
        if n == 0:
            return np.zeros((0, m), dtype=np.uint64)
        ptr = L.orc_keys(self.h, q, ph)
        return np.ctypeslib.as_array(ptr, shape=(n * m,)).reshape(n, m).copy()

    def count(self, q, expired=False):
        return int(lib().orc_count(self.h, q, 1 if expired else 0))

    def overflow(self, q, expired=False):
        return int(lib().orc_overflow(self.h, q, 1 if expired else 0))

    def digest(self, q, expired=False):
        out = (C.c_uint64 * 2)()
        lib().orc_digest(self.h, q, 1 if expired else 0, out)
        return int(out[0]), int(out[1])

    def _aux(self, q, n):
        m = self.n_qe[q]
        if n == 0:
            return np.zeros((0, m), dtype=np.uint64)
        ptr = lib().orc_aux_keys(self.h)
        return np.ctypeslib.as_array(ptr, shape=(n * m,)).reshape(n, m).copy()

    def static(self, q):
        """S(G) of the current graph for query q, sorted."""
        n = int(lib().orc_static(self.h, q))
        return self._aux(q, n)

    def seed(self, q, key, j, mode):
        """Embeddings produced by one work unit (edge `key` at position j);
        mode 0 no mask, 1 last inserted batch masked, 2 marked keys masked."""
        n = int(lib().orc_seed(self.h, q, int(key), int(j), int(mode)))
        return self._aux(q, n), int(lib().orc_aux_overflow(self.h))

    @property
    def n_keys(self):
        return int(lib().orc_n_keys(self.h))

    @property
    def n_live(self):
        return int(lib().orc_n_live(self.h))


def digest_of(rows, qidx):
    """Digest of an (n, m) key array by the oracle's hash (for comparing lists)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    da = db = 0
    for r in rows:
        da = (da + tuple_hash(SEED_A, qidx, r)) & 0xFFFFFFFFFFFFFFFF
        db = (db + tuple_hash(SEED_B, qidx, r)) & 0xFFFFFFFFFFFFFFFF
    return da, db
