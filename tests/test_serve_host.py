"""Host logic of the serving loop (paper_2206_09983_amd/serve.py) on the CPU:
batch cuts by size and deadline, sliding-window expiry, admission under a
memory budget and query lifetimes. The matcher is replaced by a recorder;
the GPU tests run the same loop on the HIP library."""
import numpy as np

from paper_2206_09983_amd import serve, synth


class Recorder:
    """Stands in for the matcher: records what the server hands it."""

    def __init__(self, graph, queries):
        self.next_key = len(graph["src"])
        self.sets = [list(queries)]
        self.calls = []

    def apply_batch(self, b):
        first = self.next_key
        self.calls.append({k: np.array(v) for k, v in b.items()})
        self.next_key += len(b["src"])
        return first

    def result(self, pos):
        return {"n_new": pos, "dig_new": (0, 0), "n_expired": 0, "dig_expired": (0, 0)}

    def set_queries(self, qs):
        self.sets.append(list(qs))

    def close(self):
        pass


def stream(n0=50, n=400, seed=1, gap=7):
    rng = np.random.default_rng(seed)
    g = synth.make_graph(16, np.ones(16, dtype=np.uint64), rng.integers(0, 16, n0), rng.integers(0, 16, n0),
                         np.zeros(n0, dtype=np.uint8), ts=np.arange(n0, dtype=np.int64) * gap)
    ts = np.cumsum(rng.integers(0, 2 * gap, n)) + n0 * gap
    return g, rng.integers(0, 16, n), rng.integers(0, 16, n), np.zeros(n, dtype=np.uint8), ts.astype(np.int64)


def q(name, n_qv=3):
    return synth.make_query(n_qv, [0] * n_qv, [(i, i + 1, -1) for i in range(n_qv - 1)], synth.ISO, name)


def test_batches_cut_by_size_and_deadline_and_window_expiry_is_exact():
    g, s, d, l, ts = stream()
    srv = serve.Server(g, [q("a")], window=300, flush_edges=32, deadline=60, backend=Recorder)
    serve.run_simulated(srv, s, d, l, ts)
    rec = srv.m.calls
    # every arrival lands in exactly one batch, in order
    assert np.array_equal(np.concatenate([c["ts"] for c in rec]), ts)
    all_ts = np.concatenate([g["ts"], ts])
    expired = set()
    for b, c in zip(srv.batches, rec):
        assert 1 <= len(c["ts"]) <= 32
        # a batch is cut when full, or once its first edge has waited the deadline
        assert len(c["ts"]) == 32 or b["now"] - c["ts"][0] >= 60 or b is srv.batches[-1]
        # deletions: exactly the keys inserted before this batch with ts <= now - window
        want = [k for k in range(b["first_key"]) if all_ts[k] <= b["now"] - 300 and k not in expired]
        assert list(c["del_keys"]) == want
        expired.update(want)
    assert len(expired) > 50


def test_admission_fifo_under_budget_and_lifetimes():
    g, s, d, l, ts = stream(n=600)
    qs = [q("q%d" % i, 3 + i % 3) for i in range(6)]
    est = [serve.query_bytes(x, 16, 64) for x in qs]
    budget = est[0] + est[1] + 1  # room for two of the first queries
    first = [(qs[0], 3), (qs[1], 5)]
    srv = serve.Server(g, first, window=10 ** 9, flush_edges=40, deadline=10 ** 9, mem_budget=budget,
                       out_capacity=64, backend=Recorder)
    later = [srv.submit(x, 4) for x in qs[2:]]
    serve.run_simulated(srv, s, d, l, ts)
    info = srv.info
    # never above the budget (the first admission aside: one query always runs)
    for b in srv.batches:
        assert sum(info[x]["bytes"] for x in b["active"]) <= max(budget, max(est))
    # lifetimes: each admitted query ran exactly its lifetime unless it was the last one left
    for qid, inf in info.items():
        if inf["retired"] is not None:
            assert inf["batches"] == inf["lifetime"]
    # first come, first served
    adm = [info[x]["admitted"] for x in [0, 1] + later]
    assert all(a is not None for a in adm)
    assert adm == sorted(adm)
    # the matcher saw one set per change, in the server's order
    assert srv.m.sets[0] == [qs[0], qs[1]]
    assert len(srv.m.sets) > 2


def test_last_query_stays_until_replaced():
    g, s, d, l, ts = stream(n=200)
    srv = serve.Server(g, [(q("only"), 1)], window=10 ** 9, flush_edges=20, deadline=10 ** 9, backend=Recorder)
    serve.run_simulated(srv, s, d, l, ts)
    assert all(b["active"] == [0] for b in srv.batches)
    assert srv.info[0]["retired"] is None
