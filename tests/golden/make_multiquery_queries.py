"""Writes multiquery_queries.json: the 64 queries of the multi-query workload.

Queries are drawn in order from the seeded shape generator (trees, cycles,
4-clique cores with tree attachments, 3..8 vertices, labels from the data
Zipfs). A draw is kept when the homomorphism count of its spanning tree on
the initial R-MAT graph (2^20 vertices, 2^24 edges, seed 7) is at most
BOUND. Removing edges from a query can only add homomorphisms, and every
isomorphism is a homomorphism, so this bounds the query's embeddings; at
BOUND = 1e8 one batch of the stream creates at most a few million
embeddings per query. Without the bound some random trees have 1e12..1e14
embeddings on this graph, far beyond any per-batch budget (the paper, too,
reports queries over its time limit separately).

Test infrastructure: run once, offline (`python tests/golden/make_multiquery_queries.py`);
the JSON it writes is the workload definition that bench.py and the tests read.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import closed_form  # noqa: E402
from oracle.closed_form import hom_count_tree  # noqa: E402
from paper_2206_09983_amd import synth  # noqa: E402

# The graph never changes between draws: build each label's multiplicity
# matrix once.
_matrix = closed_form._mult_matrix
_cache = {}


def _cached_matrix(n, src, dst, lab, label):
    if label not in _cache:
        _cache[label] = _matrix(n, src, dst, lab, label)
    return _cache[label]


closed_form._mult_matrix = _cached_matrix

BOUND = 1e8
N = 64
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "multiquery_queries.json")


def spanning_tree(q):
    """The query with edges that close cycles (in index order, union-find) removed."""
    parent = list(range(int(q["n_qv"])))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    keep = []
    for k, (a, b) in enumerate(zip(q["qsrc"], q["qdst"])):
        ra, rb = find(int(a)), find(int(b))
        if ra != rb:
            parent[ra] = rb
            keep.append(k)
    t = dict(q)
    for f in ("qsrc", "qdst", "qlabel"):
        t[f] = np.asarray(q[f])[keep]
    return t


def main():
    case = synth.rmat_case()  # the initial graph of the full stream (the draw depends on the stream length)
    g = case["graph"]
    rng = synth._rng(7 + 1000)
    kept, drawn = [], 0
    while len(kept) < N:
        q = synth.random_shape_query(rng, 16, 32, 1.2, synth.ISO)
        drawn += 1
        _, est = hom_count_tree(g["n_vertices"], g["vlabel_mask"], g["src"], g["dst"], g["elabel"], spanning_tree(q))
        print("draw %d %-7s bound %.3g %s" % (drawn, q["name"], est, "kept" if est <= BOUND else ""), flush=True)
        if est <= BOUND:
            kept.append({"name": q["name"], "n_qv": int(q["n_qv"]), "vreq": [int(x) for x in q["vreq"]],
                         "edges": [[int(a), int(b), int(l)] for a, b, l in zip(q["qsrc"], q["qdst"], q["qlabel"])],
                         "spanning_tree_hom_bound": float(est)})
    doc = {"description": __doc__.strip().split("\n\n")[1], "bound": BOUND, "draws": drawn,
           "generator": "paper_2206_09983_amd.synth.random_shape_query, rng PCG64 seed 1007, 16 vertex / 32 edge "
                        "labels, Zipf s=1.2, isomorphism",
           "queries": kept}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("kept %d of %d draws -> %s" % (len(kept), drawn, OUT))


if __name__ == "__main__":
    main()
