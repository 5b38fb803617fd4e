"""Serving loop: continuous batching of arriving edges over a sliding window.

Edges arrive one by one with timestamps (ticks, non-decreasing); standing
queries are submitted with a lifetime. The server

  * batches arrivals by size or deadline: a batch is cut when `flush_edges`
    edges wait, or when the oldest waiting edge has waited `deadline` ticks;
  * keeps a sliding window (Section VII-A, sliding-window stream: edges drop
    from the tail of the window): each batch also deletes every edge with
    ts <= now - window. Timestamps never decrease with keys, so the expired
    edges are always the oldest keys, a contiguous key range;
  * admits queries at batch boundaries, first come first served, while their
    estimated device memory fits the budget; a query retires after its
    lifetime in batches (the last active query stays until another one is
    admitted) and frees its share for the next ones. The library swaps the
    query set in place (mnemonic_set_queries), keeping the graph resident;
  * hands each batch to the matcher and records, per batch, which queries were
    active and their counts and digests (and tuple lists when asked), and the
    latency from the arrival of the batch's first edge to its results.

The matching itself is exact, so a query's per-batch results do not depend on
which other queries share the batches: only the batch cut does, and that is a
function of the arrivals alone.

Time is the caller's: `step(now)` runs a due batch at time `now` (ticks), so a
simulated clock gives deterministic batches and a wall clock gives a real-time
server. `run_realtime` replays an arrival stream against the wall clock: an
intake thread accepts arriving edges (and so forms the next batch) while the
previous batch is on the GPU, so batches follow each other back to back under
load and latency includes the time an edge waits for the GPU.
"""
import collections
import threading
import time

import numpy as np

from . import binding as B


def query_bytes(query, n_vertices, out_capacity, emit=True):
    """Device memory one query adds (the admission estimate): its two result
    buffers (new and expired tuples of n_qe 8-byte keys) when emitting, its
    vertex-filter bits (one per query vertex per data vertex) and its plans."""
    n_qe = len(query["qsrc"])
    out = 2 * out_capacity * n_qe * 8 if emit else 0
    return out + n_vertices * int(query["n_qv"]) // 8 + 4 * 1024 * n_qe


class Server:
    """graph: the initial window (dict as from synth); queries: the first
    submissions as (query, lifetime) pairs or plain queries (lifetime None:
    forever). backend: a factory (graph, queries) -> matcher object with
    apply_batch / result / keys / set_queries / close (default: the HIP
    library through binding.Matcher)."""

    def __init__(self, graph, queries, window, flush_edges=65536, deadline=5000, mem_budget=1 << 34,
                 out_capacity=1 << 16, n_elabels=32, flags=B.F_EMIT, keep_lists=False, backend=None,
                 device_inputs=False, stream=None):
        self.window = int(window)
        self.flush = int(flush_edges)
        self.deadline = int(deadline)
        self.budget = int(mem_budget)
        self.out_capacity = int(out_capacity)
        self.keep_lists = keep_lists
        self.emit = bool(flags & B.F_EMIT)
        self.timing = bool(flags & B.F_TIMING) and backend is None
        self.n_vertices = int(graph["n_vertices"])
        self.device_inputs = device_inputs
        self.stream = stream
        # keys: the initial edges hold keys 0..n-1; ts by key of the live window
        ts0 = np.asarray(graph["ts"], dtype=np.int64)
        self.key_ts = collections.deque([ts0]) if len(ts0) else collections.deque()
        self.key_base = 0          # key of key_ts[0][0]
        self.oldest = 0            # oldest live key
        self.next_key = len(ts0)
        self.last_ts = int(ts0[-1]) if len(ts0) else np.iinfo(np.int64).min
        # waiting arrivals
        self.lock = threading.Lock()
        self.wait = collections.deque()  # chunks (src, dst, lab, ts, wall)
        self.n_wait = 0
        # queries
        self.queue = collections.deque()
        self.next_qid = 0
        self.info = {}      # qid -> dict(query, lifetime, bytes, admitted, batches, retired)
        self.active = []    # qids in the matcher's order
        self.used = 0
        first = []
        for q in queries:
            query, life = (q if isinstance(q, tuple) else (q, None))
            first.append(self.submit(query, life))
        self._admit()
        if not self.active:
            raise ValueError("no query fits the memory budget")
        act = [self.info[i]["query"] for i in self.active]
        if backend is None:
            self.m = B.Matcher(graph, act, flags=flags, out_capacity=out_capacity, n_elabels=n_elabels,
                               stream=stream)
        else:
            self.m = backend(graph, act)
        self.batches = []   # per batch: dict(now, n_ins, n_del, active, results, latency_ms)
        self.n_edges = 0
        # host time of the batch steps (ms, summed): forming batches, the
        # library call, reading results
        self.host_ms = {"form": 0.0, "apply": 0.0, "results": 0.0, "device": 0.0}

    # ------------------------------------------------------------ queries
    def submit(self, query, lifetime=None):
        qid = self.next_qid
        self.next_qid += 1
        self.info[qid] = {"query": query, "lifetime": lifetime, "admitted": None, "retired": None, "batches": 0,
                          "bytes": query_bytes(query, self.n_vertices, self.out_capacity, self.emit)}
        self.queue.append(qid)
        return qid

    def _admit(self):
        """Retires queries past their lifetime, then admits queued ones in
        order while they fit. Returns True when the active set changed."""
        changed = False
        done = [q for q in self.active
                if self.info[q]["lifetime"] is not None and self.info[q]["batches"] >= self.info[q]["lifetime"]]
        if len(done) == len(self.active) and not self.queue and done:
            done.pop()  # the matcher needs one query: the last one stays until another is admitted
        for qid in done:
            self.info[qid]["retired"] = len(getattr(self, "batches", []))
            self.used -= self.info[qid]["bytes"]
            changed = True
        self.active = [q for q in self.active if q not in done]
        while self.queue and len(self.active) < 255:
            qid = self.queue[0]
            if self.used + self.info[qid]["bytes"] > self.budget and self.active:
                break  # first come, first served: later ones wait too
            self.queue.popleft()
            self.info[qid]["admitted"] = len(getattr(self, "batches", []))
            self.used += self.info[qid]["bytes"]
            self.active.append(qid)
            changed = True
        return changed

    # ------------------------------------------------------------ arrivals
    def push(self, src, dst, lab, ts, wall=None):
        """Adds arrivals (host arrays; ts non-decreasing, in ticks). wall: the
        wall-clock time (seconds) of the first of them, for latency."""
        ts = np.asarray(ts, dtype=np.int64)
        if not len(ts):
            return
        with self.lock:
            self.wait.append((np.asarray(src, dtype=np.uint32), np.asarray(dst, dtype=np.uint32),
                              np.asarray(lab, dtype=np.uint8), ts, wall))
            self.n_wait += len(ts)

    def due(self, now):
        """A batch is due: enough edges wait, or the oldest waited long enough."""
        with self.lock:
            if not self.n_wait:
                return False
            return self.n_wait >= self.flush or now - int(self.wait[0][3][0]) >= self.deadline

    def _take(self, n):
        parts, wall0 = [], None
        with self.lock:
            while n and self.wait:
                s, d, l, t, w = self.wait[0]
                if wall0 is None:
                    wall0 = w
                k = min(n, len(t))
                parts.append((s[:k], d[:k], l[:k], t[:k]))
                if k == len(t):
                    self.wait.popleft()
                else:
                    self.wait[0] = (s[k:], d[k:], l[k:], t[k:], None)
                self.n_wait -= k
                n -= k
        cat = [np.concatenate([p[i] for p in parts]) for i in range(4)]
        return cat, wall0

    # ------------------------------------------------------------ window
    def _expired(self, now):
        """Live keys with ts <= now - window: [oldest, cut)."""
        lim = now - self.window
        cut = self.oldest
        while self.key_ts:
            chunk = self.key_ts[0]
            lo = cut - self.key_base
            j = lo + int(np.searchsorted(chunk[lo:], lim, side="right"))
            cut = self.key_base + j
            if j < len(chunk):
                break
            self.key_ts.popleft()
            self.key_base += len(chunk)
        return self.oldest, cut

    # ------------------------------------------------------------ batches
    def step(self, now):
        """Runs one batch if due at time `now` (ticks). Returns its record or None."""
        if not self.due(now):
            return None
        t_form = time.perf_counter()
        (src, dst, lab, ts), wall0 = self._take(self.flush)
        if int(ts[0]) < self.last_ts:
            raise ValueError("arrival timestamps must not decrease")
        self.last_ts = int(ts[-1])
        if self._admit():
            self.m.set_queries([self.info[i]["query"] for i in self.active])
        lo, cut = self._expired(now)
        del_keys = np.arange(lo, cut, dtype=np.uint64)
        batch = {"src": src, "dst": dst, "elabel": lab, "ts": ts, "del_keys": del_keys}
        if self.device_inputs:
            import torch
            batch = {"src": torch.from_numpy(src.view(np.int32)).cuda(),
                     "dst": torch.from_numpy(dst.view(np.int32)).cuda(),
                     "elabel": torch.from_numpy(lab).cuda(), "ts": torch.from_numpy(ts).cuda(),
                     "del_keys": torch.from_numpy(del_keys.view(np.int64)).cuda()}
            if self.stream is None:
                torch.cuda.current_stream().synchronize()
        t_apply = time.perf_counter()
        first = self.m.apply_batch(batch)
        done = time.perf_counter()
        assert first == self.next_key, (first, self.next_key)
        self.key_ts.append(ts)
        self.next_key += len(ts)
        self.oldest = cut
        res = {}
        for pos, qid in enumerate(self.active):
            r = self.m.result(pos)
            rec = {"n_new": r["n_new"], "dig_new": r["dig_new"], "n_expired": r["n_expired"],
                   "dig_expired": r["dig_expired"]}
            if self.keep_lists and self.emit:
                rec["new"] = self.m.keys(pos)
                rec["expired"] = self.m.keys(pos, expired=True)
            res[qid] = rec
            self.info[qid]["batches"] += 1
        if self.timing:
            self.host_ms["device"] += self.m.stats()["ms_batch"]
        t_end = time.perf_counter()
        self.host_ms["form"] += (t_apply - t_form) * 1e3
        self.host_ms["apply"] += (done - t_apply) * 1e3
        self.host_ms["results"] += (t_end - done) * 1e3
        rec = {"now": int(now), "n_ins": len(ts), "n_del": len(del_keys), "del_range": (lo, cut), "first_key": first,
               "active": list(self.active), "results": res,
               "latency_ms": (done - wall0) * 1e3 if wall0 is not None else None}
        self.batches.append(rec)
        self.n_edges += len(ts) + len(del_keys)
        return rec

    def drain(self, now):
        """Runs batches until nothing waits (the deadline no longer applies)."""
        while self.n_wait:
            keep = self.deadline
            self.deadline = -1 << 62
            try:
                self.step(now)
            finally:
                self.deadline = keep

    def latency(self):
        lat = sorted(b["latency_ms"] for b in self.batches if b["latency_ms"] is not None)
        if not lat:
            return None, None

        def pct(p):
            return lat[min(len(lat) - 1, int(np.ceil(p / 100.0 * len(lat))) - 1)]
        return pct(50), pct(99)

    def close(self):
        if self.m is not None:
            self.m.close()
            self.m = None


def run_simulated(server, src, dst, lab, ts, chunk=1):
    """Feeds arrivals on a simulated clock (now = each arrival's ts): pushes
    them, runs every due batch, and drains at the end. Deterministic."""
    i, n = 0, len(ts)
    while i < n:
        j = i + 1
        while j < n and j - i < chunk and ts[j] == ts[i]:
            j += 1
        now = int(ts[i])
        # a deadline may expire before this arrival
        if server.n_wait and now - int(server.wait[0][3][0]) >= server.deadline:
            server.step(int(server.wait[0][3][0]) + server.deadline)
        server.push(src[i:j], dst[i:j], lab[i:j], ts[i:j])
        while server.due(now):
            server.step(now)
        i = j
    server.drain(int(ts[-1]) if n else 0)


def run_realtime(server, src, dst, lab, ts, tick_s=1e-6, duration_s=None):
    """Replays arrivals against the wall clock (arrival i at t0 + ts[i] ticks).
    An intake thread pushes arrivals as their time comes; the calling thread
    runs batches as they fall due, so that arrivals keep being accepted (and
    batches formed) while the GPU works. Returns (edges/s, p50 ms, p99 ms)."""
    n = len(ts)
    base = int(ts[0])
    t0 = time.perf_counter() + 0.01
    stop = threading.Event()

    def intake():
        # arrivals are pushed in slices of at most `poll` seconds; the thread
        # sleeps between slices, as a network reader blocks on its socket,
        # so the batch loop gets the interpreter back as soon as its library
        # call returns
        poll = 0.0002
        i = 0
        while i < n and not stop.is_set():
            now = (time.perf_counter() - t0) / tick_s + base
            j = int(np.searchsorted(ts, now, side="right"))
            if j > i:
                server.push(src[i:j], dst[i:j], lab[i:j], ts[i:j], wall=t0 + (int(ts[i]) - base) * tick_s)
                i = j
                time.sleep(poll)
            else:
                time.sleep(min(poll, max(0.0, (int(ts[i]) - now) * tick_s)))
        stop.set()

    th = threading.Thread(target=intake, daemon=True)
    th.start()
    edges0 = server.n_edges
    t_start = time.perf_counter()
    while True:
        now = int((time.perf_counter() - t0) / tick_s + base)
        if server.step(now) is None:
            if stop.is_set() and not server.n_wait:
                break
            if duration_s is not None and time.perf_counter() - t_start > duration_s:
                stop.set()
                break
            time.sleep(0.0001)
    th.join()
    elapsed = time.perf_counter() - t_start
    p50, p99 = server.latency()
    return (server.n_edges - edges0) / elapsed, p50, p99
