"""GPU parity at the benchmark's full size, in the configuration bench.py times.

The R-MAT stream (2^20 vertices, 2^24 initial edges, batches of 65,536
insertions + 6,553 oldest-key deletions, six queries):

  * counts and both digests of every query and phase of the first six
    batches (the benchmark's first timed batch is the sixth) equal the
    oracle's, stored in tests/golden/fullsize_rmat_s20.json by a script that
    runs only the oracle; the first snapshot's full lists, sorted on the
    device, equal the oracle's lists computed here;

and, where the oracle cannot recompute whole lists per batch within a test,
what holds at any size plus outputs the oracle can compute one by one:

  * every emitted tuple is an embedding of the post-insert graph (live edges,
    consistent vertex map, labels, injectivity under isomorphism), tuples are
    distinct, and each uses a batch edge (insertions: new; deletions: expired);
  * work units (batch edge at start position j, Section VI) are recovered
    from the tuples (the smallest position holding a batch edge) and sampled
    units, including the heaviest the oracle handles quickly, are compared
    bit-exact with the oracle's per-unit enumeration;
  * the homomorphic 5-path counts equal the closed form (chains of sparse
    matrix-vector products) on the graphs before and after each phase.

The 64-query stream (the same edges in log-uniform batches, 64 random
queries): counts and both digests of every query and phase of its first four
batches equal the oracle's, stored in tests/golden/fullsize_multiquery_s20.json
by the same oracle-only script. The serving stream's window (2^22 vertices,
2^26 edges, 16 temporally ordered queries): counts and digests of two
batches of 65,536 arrivals with the deletions of the keys that left the
window, likewise from the oracle (tests/golden/fullsize_serving_s22.json).
"""
import json
import os
import sys
import time

import numpy as np
import pytest

from oracle.closed_form import hom_count_tree
from oracle.core import Oracle
from paper_2206_09983_amd import synth

pytestmark = pytest.mark.gpu

N_BATCHES = 2
SAMPLE_UNITS = 6       # random units per (query, phase), plus the heaviest manageable one
HEAVY_LIMIT = 20000    # largest unit (in tuples) handed to the oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def canon(rows):
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    if len(rows) == 0:
        return rows
    return rows[np.lexsort(rows.T[::-1])]


class LiveGraph:
    """Key-indexed edge arrays of the stream, with a live mask."""

    def __init__(self, graph, batches):
        self.nv = graph["n_vertices"]
        self.vmask = graph["vlabel_mask"]
        src = [graph["src"]] + [b["src"] for b in batches]
        dst = [graph["dst"]] + [b["dst"] for b in batches]
        lab = [graph["elabel"]] + [b["elabel"] for b in batches]
        self.src = np.concatenate(src).astype(np.int64)
        self.dst = np.concatenate(dst).astype(np.int64)
        self.lab = np.concatenate(lab).astype(np.int64)
        self.live = np.zeros(len(self.src), dtype=bool)
        self.live[:len(graph["src"])] = True

    def hom_count(self, q):
        k = np.nonzero(self.live)[0]
        exact, estimate = hom_count_tree(self.nv, self.vmask, self.src[k], self.dst[k], self.lab[k], q)
        return exact


def distinct_rows(rows):
    """True when no two rows are equal: rows with distinct 64-bit hashes are
    distinct; rows whose hashes collide are compared exactly."""
    h = np.zeros(len(rows), dtype=np.uint64)
    with np.errstate(over="ignore"):
        for k in range(rows.shape[1]):
            h = (h ^ rows[:, k].astype(np.uint64)) * np.uint64(0x9E3779B97F4A7C15)
            h ^= h >> np.uint64(29)
    order = np.argsort(h, kind="stable")
    hs = h[order]
    dup = np.nonzero(hs[1:] == hs[:-1])[0]
    if len(dup) == 0:
        return True
    idx = np.unique(np.concatenate([order[dup], order[dup + 1]]))
    sub = rows[idx]
    return len(np.unique(sub, axis=0)) == len(sub)


def check_embeddings(G, q, rows, in_batch):
    """Every row is an embedding of the live graph using >= 1 batch edge."""
    if len(rows) == 0:
        return
    rows = rows.astype(np.int64)
    assert G.live[rows].all(), "tuple uses a dead edge"
    qs, qd, ql = q["qsrc"], q["qdst"], q["qlabel"]
    nqv = int(q["n_qv"])
    f = np.full((len(rows), nqv), -1, dtype=np.int64)
    for k in range(len(qs)):
        s, d = G.src[rows[:, k]], G.dst[rows[:, k]]
        for u, img in ((int(qs[k]), s), (int(qd[k]), d)):
            seen = f[:, u] >= 0
            assert (f[seen, u] == img[seen]).all(), "inconsistent vertex map"
            f[:, u] = img
        if ql[k] >= 0:
            assert (G.lab[rows[:, k]] == ql[k]).all(), "edge label"
    for u in range(nqv):
        req = np.uint64(int(q["vreq"][u]))
        assert ((G.vmask[f[:, u]] & req) == req).all(), "vertex labels"
    if int(q["sem"]) == synth.ISO:
        fs = np.sort(f, axis=1)
        assert (fs[:, 1:] != fs[:, :-1]).all(), "isomorphism needs an injective vertex map"
    assert in_batch.any(axis=1).all(), "tuple uses no batch edge"
    assert distinct_rows(rows), "duplicate tuples"


def units_of(rows, in_batch):
    """(key, position) of the unit producing each tuple: smallest batch position."""
    j = np.argmax(in_batch, axis=1)
    return rows[np.arange(len(rows)), j], j


def compare_units(o, qi, q, rows, in_batch, mode, batch_keys, rng):
    keys, js = units_of(rows, in_batch)
    code = keys.astype(np.uint64) * np.uint64(64) + js.astype(np.uint64)
    uniq, counts = np.unique(code, return_counts=True)
    picks = []
    ok = np.nonzero(counts <= HEAVY_LIMIT)[0]
    if len(ok):
        picks.append(int(uniq[ok[np.argmax(counts[ok])]]))
    if len(uniq):
        picks += [int(x) for x in rng.choice(uniq, size=min(SAMPLE_UNITS, len(uniq)), replace=False)]
    # units the GPU produced nothing for: batch edges at random positions
    for _ in range(3):
        picks.append(int(rng.choice(batch_keys)) * 64 + int(rng.integers(0, len(q["qsrc"]))))
    checked = 0
    for c in sorted(set(picks)):
        key, j = c // 64, c % 64
        ref, ovf = o.seed(qi, key, j, mode)
        assert ovf == 0
        sel = (keys == key) & (js == j)
        got = canon(rows[sel])
        np.testing.assert_array_equal(got, ref, err_msg="unit key %d position %d" % (key, j))
        checked += len(ref)
    return checked


def test_full_size_rmat_stream(request):
    torch = pytest.importorskip("torch")
    from paper_2206_09983_amd import binding as B
    B.load()
    t0 = time.time()
    case = synth.rmat_case()  # the whole stream, as bench.py draws it
    batches = case["batches"][:N_BATCHES]
    qs = case["queries"]
    say("full-size case %s: %d initial edges, %d batches checked (%.1f s)" % (
        case["name"], len(case["graph"]["src"]), N_BATCHES, time.time() - t0))
    G = LiveGraph(case["graph"], batches)
    o = Oracle(case["graph"], qs)
    stream = torch.cuda.current_stream()
    m = B.Matcher(case["graph"], qs, flags=B.F_EMIT | B.F_TIMING, out_capacity=1 << 22,
                  stream=stream.cuda_stream, n_elabels=32)
    rng = np.random.default_rng(11)
    p5h = [i for i, q in enumerate(qs) if q["name"] == "p5_homo"][0]
    try:
        for bi, b in enumerate(batches):
            db = {"src": torch.from_numpy(b["src"].view(np.int32)).cuda(),
                  "dst": torch.from_numpy(b["dst"].view(np.int32)).cuda(),
                  "elabel": torch.from_numpy(b["elabel"]).cuda(),
                  "ts": torch.from_numpy(b["ts"]).cuda(),
                  "del_keys": torch.from_numpy(b["del_keys"].view(np.int64)).cuda()}
            torch.cuda.synchronize()
            hom_before = G.hom_count(qs[p5h])
            first = m.apply_batch(db)
            ins_keys = np.arange(first, first + len(b["src"]), dtype=np.int64)
            del_keys = b["del_keys"].astype(np.int64)
            G.live[ins_keys] = True
            o.insert(b, enumerate=False)
            hom_mid = G.hom_count(qs[p5h])
            total = 0
            for qi, q in enumerate(qs):
                rows = m.keys(qi).astype(np.int64)
                inb = rows >= first
                check_embeddings(G, q, rows, inb)
                total += compare_units(o, qi, q, rows, inb, 1, ins_keys, rng)
            assert m.result(p5h)["n_new"] == (hom_mid - hom_before) % (1 << 64)
            o.mark(del_keys)
            for qi, q in enumerate(qs):
                rows = m.keys(qi, expired=True).astype(np.int64)
                inb = np.isin(rows, del_keys)
                check_embeddings(G, q, rows, inb)
                total += compare_units(o, qi, q, rows, inb, 2, del_keys, rng)
            o.unmark(del_keys)
            o.delete(del_keys, enumerate=False)
            G.live[del_keys] = False
            hom_after = G.hom_count(qs[p5h])
            assert m.result(p5h)["n_expired"] == (hom_mid - hom_after) % (1 << 64)
            say("batch %d: %s new, %s expired; %d tuples of sampled units matched the oracle (%.1f s)" % (
                bi, [m.result(i)["n_new"] for i in range(len(qs))],
                [m.result(i)["n_expired"] for i in range(len(qs))], total, time.time() - t0))
    finally:
        m.close()
        o.close()


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fullsize_rmat_s20.json")


def device_batch(torch, b):
    return {"src": torch.from_numpy(b["src"].view(np.int32)).cuda(),
            "dst": torch.from_numpy(b["dst"].view(np.int32)).cuda(),
            "elabel": torch.from_numpy(b["elabel"]).cuda(),
            "ts": torch.from_numpy(b["ts"]).cuda(),
            "del_keys": torch.from_numpy(b["del_keys"].view(np.int64)).cuda()}


def test_full_size_stream_equals_the_oracle_golden_and_lists():
    torch = pytest.importorskip("torch")
    from paper_2206_09983_amd import binding as B
    B.load()
    with open(GOLDEN) as f:
        gold = json.load(f)
    t0 = time.time()
    case = synth.rmat_case(**{k: v for k, v in gold["params"].items()})
    qs = case["queries"]
    assert [q["name"] for q in qs] == gold["queries"]
    say("full-size golden: %s, %d batches (%.1f s)" % (case["name"], len(gold["batches"]), time.time() - t0))
    stream = torch.cuda.current_stream()
    # counts and digests of every batch, in the benchmark's configuration
    m = B.Matcher(case["graph"], qs, flags=B.F_EMIT | B.F_TIMING, out_capacity=1 << 22,
                  stream=stream.cuda_stream, n_elabels=32)
    try:
        for rec in gold["batches"]:
            b = case["batches"][rec["index"]]
            assert (len(b["src"]), len(b["del_keys"])) == (rec["n_ins"], rec["n_del"])
            m.apply_batch(device_batch(torch, b))
            for qi, rq in enumerate(rec["queries"]):
                r = m.result(qi)
                assert [r["n_new"], *r["dig_new"]] == rq["new"], (rec["index"], rq["name"], "new")
                assert [r["n_expired"], *r["dig_expired"]] == rq["expired"], (rec["index"], rq["name"], "expired")
            say("batch %d: counts and digests equal the oracle's (%.1f s)" % (rec["index"], time.time() - t0))
    finally:
        m.close()
    # the first snapshot's lists, element by element
    o = Oracle(case["graph"], qs)
    m = B.Matcher(case["graph"], qs, flags=B.F_EMIT | B.F_SORT, out_capacity=1 << 22, stream=stream.cuda_stream,
                  n_elabels=32)
    try:
        b = case["batches"][0]
        m.apply_batch(device_batch(torch, b))
        o.apply_batch(b)
        n = 0
        for qi in range(len(qs)):
            for ph in (False, True):
                got = m.keys(qi, ph)
                ref = o.result(qi, ph)
                assert got.shape == ref.shape, (qi, ph)
                assert np.array_equal(got, ref), (qs[qi]["name"], ph)
                n += len(ref)
        say("snapshot 0: %d embeddings in lists equal to the oracle's (%.1f s)" % (n, time.time() - t0))
    finally:
        m.close()
        o.close()


MULTI_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fullsize_multiquery_s20.json")


def test_full_size_multiquery_stream_equals_the_oracle_golden():
    # The 64-query stream: the same 2^24 initial edges, log-uniform batches,
    # the 64 queries of multiquery_queries.json, in the benchmark's
    # configuration for that workload (emitting, output buffers grown on
    # demand from 2^16 tuples per query).
    torch = pytest.importorskip("torch")
    from paper_2206_09983_amd import binding as B
    B.load()
    with open(MULTI_GOLDEN) as f:
        gold = json.load(f)
    with open(os.path.join(os.path.dirname(__file__), "golden", "multiquery_queries.json")) as f:
        qdoc = json.load(f)
    t0 = time.time()
    case = synth.multiquery_case(queries=synth.queries_from_json(qdoc["queries"]), **gold["params"])
    qs = case["queries"]
    assert [q["name"] for q in qs] == gold["queries"]
    say("full-size golden: %s, %d batches (%.1f s)" % (case["name"], len(gold["batches"]), time.time() - t0))
    stream = torch.cuda.current_stream()
    m = B.Matcher(case["graph"], qs, flags=B.F_EMIT | B.F_TIMING, out_capacity=1 << 16,
                  stream=stream.cuda_stream, n_elabels=32)
    try:
        for rec in gold["batches"]:
            b = case["batches"][rec["index"]]
            assert (len(b["src"]), len(b["del_keys"])) == (rec["n_ins"], rec["n_del"])
            m.apply_batch(device_batch(torch, b))
            for qi, rq in enumerate(rec["queries"]):
                r = m.result(qi)
                assert [r["n_new"], *r["dig_new"]] == rq["new"], (rec["index"], rq["name"], "new")
                assert [r["n_expired"], *r["dig_expired"]] == rq["expired"], (rec["index"], rq["name"], "expired")
            say("batch %d (%d insertions, %d deletions): 64 queries' counts and digests equal the oracle's (%.1f s)"
                % (rec["index"], rec["n_ins"], rec["n_del"], time.time() - t0))
    finally:
        m.close()


SERVING_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fullsize_serving_s22.json")


def test_full_size_serving_window_equals_the_oracle_golden():
    # A slice of the serving stream: 2^22 vertices, a 2^26-edge window over
    # 2^24 ticks, arrivals at 2e7 edges/s in batches of 65,536, each deleting
    # the keys that left the window, and the serving workload's 16 queries,
    # each ordered in time along its edges.
    torch = pytest.importorskip("torch")
    from paper_2206_09983_amd import binding as B
    B.load()
    with open(SERVING_GOLDEN) as f:
        gold = json.load(f)
    with open(os.path.join(os.path.dirname(__file__), "golden", "multiquery_queries.json")) as f:
        qdoc = json.load(f)
    t0 = time.time()
    qs = [synth.with_ranks(q, np.arange(len(q["qsrc"]))) for q in synth.queries_from_json(qdoc["queries"][:16])]
    case = synth.serving_case(qs, **gold["params"])
    assert [q["name"] for q in qs] == gold["queries"]
    say("full-size golden: %s, %d batches (%.1f s)" % (case["name"], len(gold["batches"]), time.time() - t0))
    stream = torch.cuda.current_stream()
    m = B.Matcher(case["graph"], qs, flags=B.F_EMIT | B.F_TIMING, out_capacity=1 << 16, stream=stream.cuda_stream,
                  n_elabels=32)
    try:
        for rec in gold["batches"]:
            b = case["batches"][rec["index"]]
            assert (len(b["src"]), len(b["del_keys"])) == (rec["n_ins"], rec["n_del"])
            m.apply_batch(device_batch(torch, b))
            for qi, rq in enumerate(rec["queries"]):
                r = m.result(qi)
                assert [r["n_new"], *r["dig_new"]] == rq["new"], (rec["index"], rq["name"], "new")
                assert [r["n_expired"], *r["dig_expired"]] == rq["expired"], (rec["index"], rq["name"], "expired")
            say("batch %d (%d insertions, %d deletions): 16 temporal queries equal the oracle (%.1f s)"
                % (rec["index"], rec["n_ins"], rec["n_del"], time.time() - t0))
    finally:
        m.close()


MULTI_TIMED_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fullsize_multiquery_timed_s20.json")


@pytest.mark.skipif(not os.path.exists(MULTI_TIMED_GOLDEN), reason="the timed batches' golden file is not written")
def test_full_size_multiquery_timed_batches_equal_the_oracle_golden():
    # The 64-query stream's batches that bench.py times (5 warm-up, then 20
    # at a stride): the whole stream is replayed up to the last of them in
    # the benchmark's configuration, and each timed batch's counts and
    # digests are compared with the oracle's.
    torch = pytest.importorskip("torch")
    from paper_2206_09983_amd import binding as B
    import bench
    B.load()
    with open(MULTI_TIMED_GOLDEN) as f:
        gold = json.load(f)
    with open(os.path.join(os.path.dirname(__file__), "golden", "multiquery_queries.json")) as f:
        qdoc = json.load(f)
    t0 = time.time()
    case = synth.multiquery_case(queries=synth.queries_from_json(qdoc["queries"]), **gold["params"])
    qs = case["queries"]
    assert [q["name"] for q in qs] == gold["queries"]
    idx = [rec["index"] for rec in gold["batches"]]
    assert idx == bench.timed_batches(len(case["batches"]), gold["timed"]["warmup"], gold["timed"]["steps"])
    by_index = {rec["index"]: rec for rec in gold["batches"]}
    say("full-size golden: %s, timed batches %s (%.1f s)" % (case["name"], idx, time.time() - t0))
    stream = torch.cuda.current_stream()
    m = B.Matcher(case["graph"], qs, flags=B.F_EMIT | B.F_TIMING, out_capacity=1 << 16,
                  stream=stream.cuda_stream, n_elabels=32)
    try:
        for i in range(idx[-1] + 1):
            b = case["batches"][i]
            m.apply_batch(device_batch(torch, b))
            rec = by_index.get(i)
            if rec is None:
                continue
            assert (len(b["src"]), len(b["del_keys"])) == (rec["n_ins"], rec["n_del"])
            for qi, rq in enumerate(rec["queries"]):
                r = m.result(qi)
                assert [r["n_new"], *r["dig_new"]] == rq["new"], (i, rq["name"], "new")
                assert [r["n_expired"], *r["dig_expired"]] == rq["expired"], (i, rq["name"], "expired")
            say("batch %d (%d insertions): 64 queries' counts and digests equal the oracle's (%.1f s)"
                % (i, rec["n_ins"], time.time() - t0))
    finally:
        m.close()
