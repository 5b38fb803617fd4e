"""Seeded synthetic inputs for the streaming subgraph matcher.

This module only draws graphs, edge streams and query graphs. It holds none of
the matching arithmetic, so both the oracle and the HIP path can be fed from it.
All randomness comes from numpy's PCG64 generator seeded explicitly.

Workloads (stand-ins for the paper's NetFlow / LSBench streams, Section VII):
  * ``chung_lu_case``  - power-law graph, 2,000 vertices, 20,000 initial edges,
    a 2,000-edge insert-only stream in batches of 256, one labelled 4-cycle.
  * ``rmat_case``      - R-MAT(a=.57,b=.19,c=.19,d=.05) graph with ~10% parallel
    edges, Zipf(1.2) vertex and edge labels, a stream of insert batches each
    followed by deletion of the oldest 10% live keys; queries triangle-with-tail,
    4-cycle and 5-path under isomorphism and homomorphism.  The full size is
    2^20 vertices, 2^24 initial edges and 2^23 stream edges in batches of 65,536.
  * ``multiquery_case`` - the R-MAT stream re-batched with log-uniform batch
    sizes in [1,000, 262,144] (10% oldest-key deletions each) and 64 random
    connected queries of 3-8 vertices (trees, cycles, a 4-clique core with
    tree attachments), labels from the data Zipfs, isomorphism.
  * ``tiny_case``      - small multigraphs with self-loops and parallel edges,
    for brute-force checks.

Conventions: edge keys are assigned in arrival order (initial edge i has key i),
timestamps equal keys, vertex labels are one-hot 64-bit masks, a query vertex
requirement of 0 is a wildcard and a query edge label of -1 matches any label.
"""
from __future__ import annotations

import numpy as np

ISO = 0
HOMO = 1


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
def make_graph(n_vertices, vlabel_mask, src, dst, elabel, ts=None):
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    elabel = np.ascontiguousarray(elabel, dtype=np.uint8)
    if ts is None:
        ts = np.arange(len(src), dtype=np.int64)
    return {
        "n_vertices": int(n_vertices),
        "vlabel_mask": np.ascontiguousarray(vlabel_mask, dtype=np.uint64),
        "src": src,
        "dst": dst,
        "elabel": elabel,
        "ts": np.ascontiguousarray(ts, dtype=np.int64),
    }


def make_batch(src, dst, elabel, ts, del_keys=()):
    return {
        "src": np.ascontiguousarray(src, dtype=np.uint32),
        "dst": np.ascontiguousarray(dst, dtype=np.uint32),
        "elabel": np.ascontiguousarray(elabel, dtype=np.uint8),
        "ts": np.ascontiguousarray(ts, dtype=np.int64),
        "del_keys": np.ascontiguousarray(del_keys, dtype=np.uint64),
    }


def make_query(n_qv, vreq, edges, sem, name="", rank=None):
    """edges: list of (src, dst, label) with label -1 meaning any label.
    rank: None, or a temporal rank per query edge (-1: unconstrained)."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    return {
        "name": name,
        "n_qv": int(n_qv),
        "vreq": np.ascontiguousarray(vreq, dtype=np.uint64),
        "qsrc": np.ascontiguousarray(e[:, 0], dtype=np.uint32),
        "qdst": np.ascontiguousarray(e[:, 1], dtype=np.uint32),
        "qlabel": np.ascontiguousarray(e[:, 2], dtype=np.int32),
        "sem": int(sem),
        "rank": None if rank is None else np.ascontiguousarray(rank, dtype=np.int32),
    }


def with_ranks(query, rank):
    """A copy of query with temporal ranks."""
    q = dict(query)
    q["rank"] = np.ascontiguousarray(rank, dtype=np.int32)
    return q


def split_stream(n_vertices, vmask, src, dst, elabel, n_init, batch_sizes,
                 del_per_batch=None, del_frac=0.0):
    """Cut one edge sequence into an initial graph and a list of batches.

    Keys and timestamps follow arrival order. Each batch first inserts its
    edges, then deletes the oldest still-live keys (``del_per_batch[b]`` of
    them, or ``floor(del_frac * batch size)``).
    """
    ts = np.arange(len(src), dtype=np.int64)
    graph = make_graph(n_vertices, vmask, src[:n_init], dst[:n_init],
                       elabel[:n_init], ts[:n_init])
    batches = []
    pos = n_init
    oldest = 0
    for b, bs in enumerate(batch_sizes):
        bs = int(bs)
        if del_per_batch is not None:
            nd = int(del_per_batch[b])
        else:
            nd = int(np.floor(del_frac * bs))
        sl = slice(pos, pos + bs)
        dk = np.arange(oldest, oldest + nd, dtype=np.uint64)
        oldest += nd
        pos += bs
        batches.append(make_batch(src[sl], dst[sl], elabel[sl], ts[sl], dk))
    return graph, batches


# --------------------------------------------------------------------------
# graph generators
# --------------------------------------------------------------------------
def zipf_pmf(k, s):
    w = np.arange(1, k + 1, dtype=np.float64) ** (-float(s))
    return w / w.sum()


def zipf_draw(rng, k, s, n):
    """Rank r (1-based) drawn with probability proportional to r^-s; returns r-1."""
    return rng.choice(k, size=n, p=zipf_pmf(k, s)).astype(np.int64)


def chung_lu_pairs(rng, n, m, beta):
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (beta - 1.0))
    p = w / w.sum()
    src = rng.choice(n, size=m, p=p)
    dst = rng.choice(n, size=m, p=p)
    bad = np.nonzero(src == dst)[0]
    while len(bad):
        src[bad] = rng.choice(n, size=len(bad), p=p)
        dst[bad] = rng.choice(n, size=len(bad), p=p)
        bad = bad[src[bad] == dst[bad]]
    return src.astype(np.uint32), dst.astype(np.uint32)


def _rmat_raw(rng, scale, m, a, b, c):
    src = np.zeros(m, dtype=np.uint32)
    dst = np.zeros(m, dtype=np.uint32)
    chunk = 1 << 22
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        s = np.zeros(hi - lo, dtype=np.uint32)
        d = np.zeros(hi - lo, dtype=np.uint32)
        for lvl in range(scale):
            u = rng.random(hi - lo)
            sbit = u >= (a + b)                       # quadrants c, d
            dbit = ((u >= a) & (u < a + b)) | (u >= a + b + c)   # quadrants b, d
            s = (s << 1) | sbit.astype(np.uint32)
            d = (d << 1) | dbit.astype(np.uint32)
        src[lo:hi] = s
        dst[lo:hi] = d
    return src, dst


def rmat_pairs(rng, scale, m, a=0.57, b=0.19, c=0.19, multi_p=0.10):
    """R-MAT pairs, vertex ids permuted, self-loops redrawn, and a fraction
    ``multi_p`` of edges that copy the endpoints of a uniformly chosen earlier
    edge (explicit parallel multi-edges)."""
    n = 1 << scale
    src, dst = _rmat_raw(rng, scale, m, a, b, c)
    bad = np.nonzero(src == dst)[0]
    while len(bad):
        s2, d2 = _rmat_raw(rng, scale, len(bad), a, b, c)
        src[bad] = s2
        dst[bad] = d2
        bad = bad[src[bad] == dst[bad]]
    perm = rng.permutation(n).astype(np.uint32)
    src = perm[src]
    dst = perm[dst]
    if multi_p > 0 and m > 1:
        copy = rng.random(m) < multi_p
        copy[0] = False
        idx = np.arange(m, dtype=np.int64)
        parent = idx.copy()
        ci = np.nonzero(copy)[0]
        parent[ci] = (rng.random(len(ci)) * ci).astype(np.int64)  # uniform in [0, i)
        # resolve chains of copies (parents are always earlier)
        while True:
            pp = parent[parent]
            if np.array_equal(pp, parent):
                break
            parent = pp
        src = src[parent]
        dst = dst[parent]
    return src, dst


# --------------------------------------------------------------------------
# query graphs
# --------------------------------------------------------------------------
def triangle_with_tail_edges():
    return [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4)], 5


def cycle_edges(k):
    return [(i, (i + 1) % k) for i in range(k)], k


def path_edges(k):
    return [(i, i + 1) for i in range(k - 1)], k


def labelled_query(rng, shape, n_vlabels, n_elabels, s, sem, name):
    edges, nv = shape
    vl = zipf_draw(rng, n_vlabels, s, nv)
    el = zipf_draw(rng, n_elabels, s, len(edges))
    vreq = (np.uint64(1) << vl.astype(np.uint64)).astype(np.uint64)
    return make_query(nv, vreq, [(a, b, int(l)) for (a, b), l in zip(edges, el)], sem, name)


def rmat_queries(seed=7, n_vlabels=16, n_elabels=32, s=1.2, sems=(ISO, HOMO)):
    """Triangle-with-tail, 4-cycle and 5-path, labels drawn i.i.d. from the data
    Zipf distributions; each shape is returned once per semantics."""
    rng = _rng(seed)
    shapes = [("tt", triangle_with_tail_edges()), ("c4", cycle_edges(4)), ("p5", path_edges(5))]
    base = [labelled_query(rng, sh, n_vlabels, n_elabels, s, ISO, nm) for nm, sh in shapes]
    out = []
    for q in base:
        for sem in sems:
            qq = dict(q)
            qq["sem"] = int(sem)
            qq["name"] = q["name"] + ("_iso" if sem == ISO else "_homo")
            out.append(qq)
    return out


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def chung_lu_case(seed=1, n=2000, n_init=20000, n_stream=2000, batch=256, beta=2.1,
                  n_vlabels=4, n_elabels=8, sems=(ISO, HOMO)):
    rng = _rng(seed)
    m = n_init + n_stream
    src, dst = chung_lu_pairs(rng, n, m, beta)
    vl = rng.integers(0, n_vlabels, size=n)
    el = rng.integers(0, n_elabels, size=m).astype(np.uint8)
    vmask = (np.uint64(1) << vl.astype(np.uint64)).astype(np.uint64)
    sizes = [batch] * (n_stream // batch) + ([n_stream % batch] if n_stream % batch else [])
    graph, batches = split_stream(n, vmask, src, dst, el, n_init, sizes, del_frac=0.0)
    c4, _ = cycle_edges(4)
    vreq = np.array([1 << 0, 1 << 1, 1 << 0, 1 << 1], dtype=np.uint64)
    queries = []
    for sem in sems:
        queries.append(make_query(4, vreq, [(a, b, l) for (a, b), l in zip(c4, range(4))], sem,
                                  "c4_" + ("iso" if sem == ISO else "homo")))
    return {"name": "chung_lu_n%d_m%d" % (n, n_init), "graph": graph,
            "batches": batches, "queries": queries}


def rmat_case(scale=20, n_init=1 << 24, n_stream=1 << 23, batch=65536, del_frac=0.10,
              seed=7, query_seed=7, n_vlabels=16, n_elabels=32, s=1.2, multi_p=0.10,
              n_batches=None, sems=(ISO, HOMO)):
    """R-MAT stream; ``n_batches`` limits how many stream batches are drawn."""
    rng = _rng(seed)
    nb = n_stream // batch
    if n_batches is not None:
        nb = min(nb, int(n_batches))
    m = n_init + nb * batch
    src, dst = rmat_pairs(rng, scale, m, multi_p=multi_p)
    n = 1 << scale
    vl = zipf_draw(rng, n_vlabels, s, n)
    el = zipf_draw(rng, n_elabels, s, m).astype(np.uint8)
    vmask = (np.uint64(1) << vl.astype(np.uint64)).astype(np.uint64)
    graph, batches = split_stream(n, vmask, src, dst, el, n_init, [batch] * nb,
                                  del_frac=del_frac)
    queries = rmat_queries(query_seed, n_vlabels, n_elabels, s, sems)
    return {"name": "rmat_s%d_m%d_b%d" % (scale, n_init, batch), "graph": graph,
            "batches": batches, "queries": queries}


def serving_edges(scale=22, n_window=1 << 26, n_arrivals=1 << 25, seed=7, n_vlabels=16, n_elabels=32, s=1.2,
                  multi_p=0.10):
    """The edges of the serving workload: R-MAT (same parameters and label
    Zipfs as rmat_case) with n_window edges for the initial window followed by
    n_arrivals streamed edges. Timestamps come from serving_times."""
    rng = _rng(seed)
    m = n_window + n_arrivals
    src, dst = rmat_pairs(rng, scale, m, multi_p=multi_p)
    n = 1 << scale
    vl = zipf_draw(rng, n_vlabels, s, n)
    el = zipf_draw(rng, n_elabels, s, m).astype(np.uint8)
    vmask = (np.uint64(1) << vl.astype(np.uint64)).astype(np.uint64)
    return {"n_vertices": n, "vlabel_mask": vmask, "src": src.astype(np.uint32), "dst": dst.astype(np.uint32),
            "elabel": el, "n_window": n_window}


def serving_times(edges, window_ticks=1 << 24, rate=1e6, tick_s=1e-6, seed=7):
    """Initial window: its edges spread evenly over window_ticks (ts = key *
    window / n_window). Arrivals: a Poisson process at `rate` edges per second
    (exponential gaps, ticks of tick_s seconds, ts rounded down), starting at
    the end of the window. Returns (graph, (src, dst, elabel, ts))."""
    nw = edges["n_window"]
    rng = _rng(seed + 3000 + int(rate))
    ts0 = (np.arange(nw, dtype=np.float64) * (window_ticks / nw)).astype(np.int64)
    graph = make_graph(edges["n_vertices"], edges["vlabel_mask"], edges["src"][:nw], edges["dst"][:nw],
                       edges["elabel"][:nw], ts=ts0)
    n = len(edges["src"]) - nw
    gaps = rng.exponential(1.0 / (rate * tick_s), n)
    ts = (window_ticks + np.floor(np.cumsum(gaps))).astype(np.int64)
    return graph, (edges["src"][nw:], edges["dst"][nw:], edges["elabel"][nw:], ts)


def serving_case(queries, scale=22, n_window=1 << 26, rate=2e7, batch=65536, n_batches=2,
                 window_ticks=1 << 24, seed=7):
    """A fixed slice of the serving stream: the initial window of
    serving_times at ``rate``, then ``n_batches`` batches of ``batch``
    consecutive arrivals. Each batch deletes the live keys whose timestamp is
    at most (the batch's last arrival timestamp - window_ticks), as a server
    flushing full batches would. ``queries`` are used as given."""
    edges = serving_edges(scale=scale, n_window=n_window, n_arrivals=batch * n_batches, seed=seed)
    graph, (s, d, l, ts) = serving_times(edges, window_ticks=window_ticks, rate=rate, seed=seed)
    all_ts = np.concatenate([graph["ts"], ts])
    batches, oldest = [], 0
    for i in range(n_batches):
        a, b = i * batch, (i + 1) * batch
        now = int(ts[b - 1])
        cut = max(oldest, int(np.searchsorted(all_ts, now - window_ticks, side="right")))
        batches.append(make_batch(s[a:b], d[a:b], l[a:b], ts[a:b], np.arange(oldest, cut, dtype=np.uint64)))
        oldest = cut
    return {"name": "serving_rmat_s%d_window%d_ticks%d_rate%.0e_b%d" % (scale, n_window, window_ticks, rate, batch),
            "graph": graph, "batches": batches, "queries": list(queries)}


def random_connected_query(rng, nv, n_extra, n_vlabels, n_elabels, wild_p, sem):
    """Random weakly connected simple digraph query (no self-loops, at most one
    edge per ordered pair)."""
    pairs = set()
    edges = []
    for v in range(1, nv):
        u = int(rng.integers(0, v))
        a, b = (u, v) if rng.random() < 0.5 else (v, u)
        pairs.add((a, b))
        edges.append((a, b))
    tries = 0
    while n_extra > 0 and tries < 50:
        tries += 1
        a, b = (int(x) for x in rng.integers(0, nv, size=2))
        if a == b or (a, b) in pairs:
            continue
        pairs.add((a, b))
        edges.append((a, b))
        n_extra -= 1
    order = rng.permutation(len(edges))
    edges = [edges[i] for i in order]
    vreq = []
    for _ in range(nv):
        if rng.random() < wild_p:
            vreq.append(0)
        else:
            m = 1 << int(rng.integers(0, n_vlabels))
            if rng.random() < 0.15:
                m |= 1 << int(rng.integers(0, n_vlabels))
            vreq.append(m)
    labs = [(-1 if rng.random() < wild_p else int(rng.integers(0, n_elabels))) for _ in edges]
    return make_query(nv, np.array(vreq, dtype=np.uint64),
                      [(a, b, l) for (a, b), l in zip(edges, labs)], sem, "rand")


def temporal_tiny_case(seed, ts_ties=False, **kw):
    """tiny_case with random temporal ranks on its queries (ranks in
    -1..m-1, ties allowed); with ts_ties, timestamps are key // 2, so that
    pairs of edges share a timestamp."""
    case = tiny_case(seed, **kw)
    rng = _rng(seed + 7000)
    m = len(case["queries"][0]["qsrc"])
    rank = rng.integers(-1, m, size=m)
    case["queries"] = [with_ranks(q, rank) for q in case["queries"]]
    if ts_ties:
        g = dict(case["graph"])
        g["ts"] = np.arange(len(g["src"]), dtype=np.int64) // 2
        case["graph"] = g
        case["batches"] = [dict(b, ts=np.ascontiguousarray(b["ts"] // 2)) for b in case["batches"]]
    case["name"] = "temporal_" + case["name"] + ("_ties" if ts_ties else "")
    return case


def tiny_case(seed, max_v=6, max_init=10, n_batches=3, max_ins=4, max_del=3,
              n_vlabels=2, n_elabels=2, max_qv=4, wild_p=0.3, self_loops=True):
    """A tiny multigraph stream (self-loops and parallel edges allowed) with a
    random query under both semantics; sized for brute force."""
    rng = _rng(seed)
    n = int(rng.integers(2, max_v + 1))
    vmask = np.zeros(n, dtype=np.uint64)
    for v in range(n):
        m = 1 << int(rng.integers(0, n_vlabels))
        if rng.random() < 0.2:
            m |= 1 << int(rng.integers(0, n_vlabels))
        vmask[v] = m

    def draw_edges(k):
        s = rng.integers(0, n, size=k)
        d = rng.integers(0, n, size=k)
        if not self_loops:
            d = np.where(s == d, (d + 1) % n, d)
        # repeat some earlier pairs to create parallel edges
        for i in range(1, k):
            if rng.random() < 0.25:
                j = int(rng.integers(0, i))
                s[i], d[i] = s[j], d[j]
        lab = rng.integers(0, n_elabels, size=k)
        return s, d, lab

    n_init = int(rng.integers(0, max_init + 1))
    s0, d0, l0 = draw_edges(n_init)
    graph = make_graph(n, vmask, s0, d0, l0)
    batches = []
    next_key = n_init
    live = list(range(n_init))
    for _ in range(n_batches):
        ni = int(rng.integers(0, max_ins + 1))
        s, d, lab = draw_edges(ni)
        ts = np.arange(next_key, next_key + ni, dtype=np.int64)
        live_after = live + list(range(next_key, next_key + ni))
        nd = int(rng.integers(0, min(max_del, len(live_after)) + 1))
        dk = sorted(int(x) for x in rng.choice(live_after, size=nd, replace=False)) if nd else []
        batches.append(make_batch(s, d, lab, ts, dk))
        next_key += ni
        live = [k for k in live_after if k not in set(dk)]
    nqv = int(rng.integers(2, max_qv + 1))
    q = random_connected_query(rng, nqv, int(rng.integers(0, 3)), n_vlabels, n_elabels, wild_p, ISO)
    qh = dict(q)
    qh["sem"] = HOMO
    return {"name": "tiny%d" % seed, "graph": graph, "batches": batches, "queries": [q, qh]}


# --------------------------------------------------------------------------
# many queries over one stream
# --------------------------------------------------------------------------
def random_shape_query(rng, n_vlabels, n_elabels, s, sem, min_v=3, max_v=8):
    """One query: shape uniform over {tree, cycle, 4-clique core + tree
    attachments}, 3..8 vertices (>= 4 with the clique), edge directions
    uniform, vertex and edge labels drawn from the data Zipfs."""
    kind = int(rng.integers(0, 3))
    lo = 4 if kind == 2 else min_v
    nv = int(rng.integers(lo, max_v + 1))
    pairs = []
    if kind == 1:  # cycle
        pairs = [(i, (i + 1) % nv) for i in range(nv)]
        start = nv
    elif kind == 2:  # 4-clique core
        pairs = [(a, b) for a in range(4) for b in range(a + 1, 4)]
        start = 4
    else:  # tree
        start = 1
    for v in range(start, nv):
        pairs.append((int(rng.integers(0, v)), v))
    edges = [(a, b) if rng.random() < 0.5 else (b, a) for a, b in pairs]
    order = rng.permutation(len(edges))
    edges = [edges[i] for i in order]
    vl = zipf_draw(rng, n_vlabels, s, nv)
    el = zipf_draw(rng, n_elabels, s, len(edges))
    vreq = (np.uint64(1) << vl.astype(np.uint64)).astype(np.uint64)
    name = ("tree", "cycle", "k4")[kind] + str(nv)
    return make_query(nv, vreq, [(a, b, int(l)) for (a, b), l in zip(edges, el)], sem, name)


def random_queries(n, seed=7, n_vlabels=16, n_elabels=32, s=1.2, sem=ISO):
    rng = _rng(seed + 1000)
    return [random_shape_query(rng, n_vlabels, n_elabels, s, sem) for _ in range(n)]


def log_uniform_sizes(rng, total, lo=1000, hi=262144):
    """Batch sizes floor(exp U(ln lo, ln hi)) until `total` edges are used."""
    sizes = []
    used = 0
    while used < total:
        b = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        b = min(b, total - used)
        sizes.append(b)
        used += b
    return sizes


def queries_from_json(entries, sem=ISO):
    """Query dicts from a list of {"name", "n_qv", "vreq", "edges": [[src, dst, label], ...]}."""
    return [make_query(e["n_qv"], e["vreq"], e["edges"], sem, e.get("name", "")) for e in entries]


def multiquery_case(scale=20, n_init=1 << 24, n_stream=1 << 23, n_queries=64, del_frac=0.10, seed=7,
                    n_vlabels=16, n_elabels=32, s=1.2, multi_p=0.10, lo=1000, hi=262144, max_batches=None,
                    queries=None):
    """The R-MAT stream of ``rmat_case`` (same seed, same edges) cut into
    log-uniform batches, with ``n_queries`` random queries (or the given
    ``queries``)."""
    base = rmat_case(scale=scale, n_init=n_init, n_stream=n_stream, batch=min(65536, n_stream),
                     del_frac=0.0, seed=seed, n_vlabels=n_vlabels, n_elabels=n_elabels, s=s,
                     multi_p=multi_p, sems=(ISO,))
    g = base["graph"]
    src = np.concatenate([g["src"]] + [b["src"] for b in base["batches"]])
    dst = np.concatenate([g["dst"]] + [b["dst"] for b in base["batches"]])
    lab = np.concatenate([g["elabel"]] + [b["elabel"] for b in base["batches"]])
    rng = _rng(seed + 2000)
    sizes = log_uniform_sizes(rng, len(src) - n_init, lo, hi)
    if max_batches is not None:
        sizes = sizes[:max_batches]
    graph, batches = split_stream(g["n_vertices"], g["vlabel_mask"], src, dst, lab, n_init, sizes,
                                  del_frac=del_frac)
    if queries is None:
        queries = random_queries(n_queries, seed, n_vlabels, n_elabels, s, ISO)
    return {"name": "rmat_s%d_m%d_logbatch_%dq" % (scale, n_init, len(queries)), "graph": graph,
            "batches": batches, "queries": queries}

