"""Closed-form homomorphism counts for tree-shaped queries (test infrastructure).

Under homomorphism (Section III: the injectivity check is dropped and one data
edge may serve several query edges) the number of embeddings (f, g) of a tree
query factorises over its edges:
    count = sum_v c_root(v),   c_u = D_u * prod_{child w via edge e} (A_e c_w)
where D_u is the 0/1 vector of data vertices whose label set contains u's
required set, and A_e is the edge-multiplicity matrix of the query edge's label
oriented from u towards w (parallel edges count separately). For a directed
path this is a chain of sparse matrix-vector products. Counts are exact integers
modulo 2^64 (the GPU's counter width); the float64 estimate flags overflow.
"""
import numpy as np
import scipy.sparse as sp


def _mult_matrix(n, src, dst, lab, label):
    if label >= 0:
        sel = lab == label
        s, d = src[sel], dst[sel]
    else:
        s, d = src, dst
    data = np.ones(len(s), dtype=np.int64)
    return sp.csr_matrix((data, (s.astype(np.int64), d.astype(np.int64))), shape=(n, n))


def hom_count_tree(n_vertices, vmask, src, dst, lab, query):
    """Homomorphism count of a tree query (n_qe == n_qv - 1, weakly connected)."""
    nqv = int(query["n_qv"])
    qs = [int(x) for x in query["qsrc"]]
    qd = [int(x) for x in query["qdst"]]
    ql = [int(x) for x in query["qlabel"]]
    if len(qs) != nqv - 1:
        raise ValueError("not a tree query")
    src = np.asarray(src)
    dst = np.asarray(dst)
    lab = np.asarray(lab).astype(np.int64)
    vmask = np.asarray(vmask, dtype=np.uint64)
    D = [((vmask & np.uint64(int(r))) == np.uint64(int(r))).astype(np.int64) for r in query["vreq"]]
    adj = [[] for _ in range(nqv)]
    for e, (a, b) in enumerate(zip(qs, qd)):
        adj[a].append((b, e, +1))  # from a to b along the edge direction
        adj[b].append((a, e, -1))  # from b to a against it
    mats = {}

    def M(e, direction):
        key = (e, direction)
        if key not in mats:
            A = _mult_matrix(n_vertices, src, dst, lab, ql[e])
            mats[key] = A if direction > 0 else A.T.tocsr()
        return mats[key]

    def solve(u, parent):
        c = D[u].copy()
        cf = D[u].astype(np.float64)
        for w, e, direction in adj[u]:
            if w == parent:
                continue
            cw, cwf = solve(w, u)
            A = M(e, direction)
            with np.errstate(over="ignore"):
                c = c * (A @ cw)
            cf = cf * (A.astype(np.float64) @ cwf)
        return c, cf

    c, cf = solve(0, -1)
    with np.errstate(over="ignore"):
        total = int(np.sum(c.astype(np.uint64), dtype=np.uint64))
    est = float(cf.sum())
    return total, est


def graph_arrays_after(graph, batches, upto, include_deletions=True, last_insert_only=False):
    """Live edge arrays after applying batches[:upto] (deletions of batch upto-1
    skipped when last_insert_only)."""
    s = [np.asarray(graph["src"])]
    d = [np.asarray(graph["dst"])]
    l = [np.asarray(graph["elabel"])]
    dead = []
    for i, b in enumerate(batches[:upto]):
        s.append(np.asarray(b["src"]))
        d.append(np.asarray(b["dst"]))
        l.append(np.asarray(b["elabel"]))
        if include_deletions and not (last_insert_only and i == upto - 1):
            dead.append(np.asarray(b["del_keys"], dtype=np.int64))
    s = np.concatenate(s)
    d = np.concatenate(d)
    l = np.concatenate(l)
    keep = np.ones(len(s), dtype=bool)
    if dead:
        keep[np.concatenate(dead)] = False
    return s[keep], d[keep], l[keep]
