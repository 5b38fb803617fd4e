"""Brute-force embedding sets for tiny graphs (test infrastructure only).

S(G) is listed straight from the definition of Section II-B: every vertex map
f: V_Q -> V (injective for isomorphism, any for homomorphism), kept when every
query vertex's required label set is a subset of its image's label set, times
every choice of one live edge instance per query edge with matching direction
and label (an empty query label matches any label). Parallel edges are distinct
instances. New and expired sets of a snapshot are then plain set differences:
    new     = S(G u I) - S(G)
    expired = S(G u I) - S(G u I - D)
Nothing here is incremental, ordered or masked, so it pins the oracle's
incremental matcher independently.
"""
import itertools

import numpy as np


def static_set(n_vertices, vmask, live, query, ts=None):
    """live: dict key -> (src, dst, label). Returns a set of key tuples.
    With query["rank"] (temporal order) and ts (key -> timestamp), a tuple is
    kept only when ts strictly increases from every ranked edge to every edge
    of a higher rank (rank -1: unconstrained)."""
    nqv = int(query["n_qv"])
    vreq = [int(x) for x in query["vreq"]]
    qs = [int(x) for x in query["qsrc"]]
    qd = [int(x) for x in query["qdst"]]
    ql = [int(x) for x in query["qlabel"]]
    iso = int(query["sem"]) == 0
    vm = [int(x) for x in vmask]
    by_pair = {}
    for k, (s, d, l) in live.items():
        by_pair.setdefault((s, d), []).append((k, l))
    out = set()
    # Every vertex map f, built one query vertex at a time in index order. A
    # partial map is dropped as soon as a fixed vertex breaks its label
    # requirement or injectivity, or a query edge with both endpoints fixed
    # has no instance: every full map extending it would fail the same test.
    edges_at = [[k for k in range(len(qs)) if max(qs[k], qd[k]) == u] for u in range(nqv)]
    rank = query.get("rank")

    def in_time_order(combo):
        for a, ka in enumerate(combo):
            for b, kb in enumerate(combo):
                if rank[a] >= 0 and rank[b] >= 0 and rank[a] < rank[b] and not ts[ka] < ts[kb]:
                    return False
        return True

    def inst(k, f):
        return [key for key, el in by_pair.get((f[qs[k]], f[qd[k]]), []) if ql[k] < 0 or ql[k] == el]

    def rec(f):
        u = len(f)
        if u == nqv:
            choices = [inst(k, f) for k in range(len(qs))]
            for combo in itertools.product(*choices):
                if rank is not None and not in_time_order(combo):
                    continue
                out.add(tuple(combo))
            return
        for v in range(n_vertices):
            if vreq[u] & ~vm[v]:
                continue
            if iso and v in f:
                continue
            f2 = f + [v]
            if all(inst(k, f2) for k in edges_at[u]):
                rec(f2)

    rec([])
    return out


def run_stream(graph, batches, query):
    """Per batch: (sorted new tuples, sorted expired tuples), by set differences."""
    n = int(graph["n_vertices"])
    vmask = graph["vlabel_mask"]
    live, ts = {}, {}
    for k, (s, d, l, t) in enumerate(zip(graph["src"], graph["dst"], graph["elabel"], graph["ts"])):
        live[k] = (int(s), int(d), int(l))
        ts[k] = int(t)
    next_key = len(live)
    results = []
    for b in batches:
        before = static_set(n, vmask, live, query, ts)
        for s, d, l, t in zip(b["src"], b["dst"], b["elabel"], b["ts"]):
            live[next_key] = (int(s), int(d), int(l))
            ts[next_key] = int(t)
            next_key += 1
        mid = static_set(n, vmask, live, query, ts)
        for k in b["del_keys"]:
            del live[int(k)]
        after = static_set(n, vmask, live, query, ts)
        results.append((sorted(mid - before), sorted(mid - after)))
    return results


def as_array(tuples, m):
    if not tuples:
        return np.zeros((0, m), dtype=np.uint64)
    return np.array(sorted(tuples), dtype=np.uint64).reshape(-1, m)
