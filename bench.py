#!/usr/bin/env python3
"""Throughput of the streaming matcher's hot path on one MI355X.

One step = one snapshot of the paper's batch loop (Algorithm 1 body,
Algorithm 2): validate and ingest a batch of insertions, merge them into the
sorted adjacency, edgeMatcher, vertex filter, enumerate the new embeddings,
then flag and enumerate the embeddings the batch's deletions expire, retire
the deleted edges and reduce counts and digests. Every step runs in the HIP
library through its C ABI; the batch arrays are resident in HBM before the
timed region starts.

Workload (stand-in for the paper's NetFlow/LSBench streams, Section VII):
R-MAT (a=.57, b=.19, c=.19, d=.05) with 2^20 vertices and 2^24 initial edges,
~10% parallel multi-edges, Zipf(1.2) vertex labels over 16 and edge labels
over 32, int64 timestamps; batches of 65,536 insertions, each followed by
deletion of the 6,553 oldest live edges; queries triangle-with-tail, 4-cycle
and 5-path, each under isomorphism and homomorphism (six query runs over the
same stream).

With --workload multiquery the same stream is cut into log-uniform batches
(1,000..262,144 insertions, 10% oldest-key deletions each) and matched
against 64 random trees, cycles and 4-clique cores (tests/golden/
multiquery_queries.json lists them and how they were drawn), all in the
same per-level launches; --autotune lets the library pick its expansion
tile on the warm-up batches.

Prints ONE JSON line. ``value`` = stream edges (insertions + deletions) fully
processed per second; embeddings/s and p50/p99 batch latency ride along.
With the committed order-cost network present, the same batches are also
timed under the learned scheduler (a fresh context; every start row takes
the matching order the network predicts cheapest) and ``learned_vs_plain``
is its throughput over the static order's, after checking that both give
identical counts and digests for every batch and query.
``roofline`` reports the expansion kernel's (k_expand, the enumerator's
dominant kernel) algorithmic bytes per launch divided by its average launch
time (HIP events the library records around each launch on its stream),
against the 8 TB/s HBM peak. ``cpu_baseline`` times the single-threaded CPU
oracle on a bounded prefix of the same stream.
"""
import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "matched data edges/sec + new embeddings/sec at 1 GPU; p99 batch latency; learned vs plain"
HBM_PEAK_GBS = 8000.0
ENUM_SRC = os.path.join(ROOT, "paper_2206_09983_amd", "csrc", "mn_enum.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_expand_traffic_rmat_s20.txt")

# Algorithmic bytes of the enumerator, per unit of work the library counts
# (the per-unit figures of the hot-path scope's measurement section):
#   work unit (seed): 8 B
#   candidate: its 8 B adjacency entry, plus the 4 B edge-index (edgeMatcher)
#     word and the 4 B vertex-filter word the method tests per candidate
#   closing-edge (intersection) lookup: 4 B per probe actually executed
#   emitted tuple: 8 B per query-edge key written
# Rows of partial embeddings passed between levels, and the keys gathered from
# them, are this implementation's choice, not the method's, and are not
# counted. Each term's total is printed inside the line's roofline object.
BYTES = {"seeds": 8, "entries_scanned": 8 + 4 + 4, "probe_words": 4, "tuple_words": 8}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--n-init", type=int, default=1 << 24)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--del-frac", type=float, default=0.10)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--count-only", action="store_true", help="counts and digests only, no tuples")
    ap.add_argument("--out-capacity", type=int, default=1 << 22, help="initial tuples per result buffer")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU-oracle sample")
    ap.add_argument("--workload", choices=("rmat", "multiquery", "serving"), default="rmat")
    ap.add_argument("--rates", default="1e6,2e6,5e6,1e7,2e7", help="serving: arrival rates (edges/s)")
    ap.add_argument("--seconds", type=float, default=1.5, help="serving: wall time replayed per rate")
    ap.add_argument("--serve-scale", type=int, default=22, help="serving: R-MAT scale")
    ap.add_argument("--serve-window", type=int, default=1 << 26, help="serving: edges in the initial window")
    ap.add_argument("--autotune", action="store_true", help="let the library choose its expansion tile")
    ap.add_argument("--tree-filter", action="store_true",
                    help="strengthen the vertex filter with the spanning-tree propagation before each batch")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration) and exit")
    ap.add_argument("--scheduler", choices=("both", "static", "learned"), default="both",
                    help="both: the line reports the static order and times the learned scheduler on the same "
                         "batches for learned_vs_plain; static or learned: time that one only")
    ap.add_argument("--weights", default=None, help="order-cost network (default: the committed weights)")
    ap.add_argument("--no-rates", action="store_true", help="skip the count-only and index-only runs")
    return ap.parse_args()


def timed_batches(n_total, warmup, steps):
    """Indices of the timed batches: `steps` batches spread at an equal stride
    over the stream after the `warmup` first ones (consecutive when the stream
    is no longer than warmup + steps), so the timing covers the graph as it
    grows and shrinks over the whole stream."""
    if steps < 1:
        raise SystemExit("--steps must be at least 1")
    if warmup + steps > n_total:
        raise SystemExit("the stream has %d batches: --warmup + --steps must not exceed it" % n_total)
    stride = max(1, (n_total - warmup) // steps)
    return [warmup + i * stride for i in range(steps)]


def describe_batches(idx):
    if len(idx) > 1:
        return "%d..%d step %d (%d batches)" % (idx[0], idx[-1], idx[1] - idx[0], len(idx))
    return "%d (1 batch)" % idx[0]


def enum_source_hash():
    with open(ENUM_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(workload, steps, warmup):
    """Per-launch HBM bytes of the enumerator from the committed counter
    summary, or None when absent, taken on a different kernel source, on
    other timed steps, or on another workload (the counters cover the default
    R-MAT stream)."""
    if workload != "rmat" or not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != enum_source_hash():
        return None
    if kv.get("bench_steps_warmup") != "%d %d" % (steps, warmup):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    import torch
    n = 1 << 30
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    torch.cuda.synchronize()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}), flush=True)


def copy_gbps(reps=5):
    """Achievable HBM rate on this device: the best of `reps` timed 1 GiB
    device-to-device copies (read + write bytes per second), in GB/s."""
    import torch
    n = 1 << 30
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * n / (best * 1e-3) / 1e9


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(case, budget_s):
    """Times the CPU oracle (single thread, pinned to one core where the OS
    allows) on a prefix of the first stream batch, applied as consecutive
    sub-batches of doubling size, until the budget is spent. Returns edges/s
    over the sample, its description and the core it ran on."""
    import numpy as np

    from oracle.core import Oracle
    from paper_2206_09983_amd import synth

    core, saved = None, None
    if hasattr(os, "sched_setaffinity"):
        saved = os.sched_getaffinity(0)
        core = min(saved)
        os.sched_setaffinity(0, {core})
    try:
        return _cpu_baseline(case, budget_s, np, Oracle, synth) + (core,)
    finally:
        if saved is not None:
            os.sched_setaffinity(0, saved)


def _cpu_baseline(case, budget_s, np, Oracle, synth):
    b = case["batches"][0]
    n_ins, n_del = len(b["src"]), len(b["del_keys"])
    t0 = time.perf_counter()
    o = Oracle(case["graph"], case["queries"], limit=1 << 22)
    t_load = time.perf_counter() - t0
    done_i = done_d = 0
    spent = 0.0
    size = 64
    while done_i < n_ins and spent < budget_s:
        s = min(size, n_ins - done_i)
        d = min(n_del - done_d, int(round((done_i + s) * n_del / n_ins)) - done_d)
        sl = slice(done_i, done_i + s)
        sub = synth.make_batch(b["src"][sl], b["dst"][sl], b["elabel"][sl], b["ts"][sl],
                               b["del_keys"][done_d:done_d + d])
        t1 = time.perf_counter()
        o.apply_batch(sub)
        spent += time.perf_counter() - t1
        done_i += s
        done_d += d
        size *= 2
    emb = 0
    o.close()
    rate = (done_i + done_d) / spent if spent > 0 else 0.0
    desc = ("oracle, 1 thread: first %d insertions + %d oldest-key deletions of stream batch 0, in "
            "doubling sub-batches from 64; %.1f s timed (graph load %.1f s not timed)"
            % (done_i, done_d, spent, t_load))
    return rate, desc, np


def serving_bench(args):
    """Serving workload: Poisson arrivals at each rate over a sliding window
    of 2^24 ticks (1 us) on an R-MAT graph whose initial window holds 2^26
    edges (4 per tick), 16 queries (the first 16 of the multi-query set) with
    a temporal order along their edges, batches cut at 65,536 edges or a 5 ms
    deadline, replayed against the wall clock."""
    import numpy as np
    import torch

    from paper_2206_09983_amd import binding, serve, synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    binding.load()
    rates = [float(r) for r in args.rates.split(",")]
    t0 = time.perf_counter()
    n_arr = int(max(rates) * args.seconds * 1.2) + 65536
    edges = synth.serving_edges(scale=args.serve_scale, n_window=args.serve_window, n_arrivals=n_arr, seed=args.seed)
    with open(os.path.join(ROOT, "tests", "golden", "multiquery_queries.json")) as f:
        qdoc = json.load(f)
    queries = [synth.with_ranks(q, np.arange(len(q["qsrc"])))
               for q in synth.queries_from_json(qdoc["queries"][:16])]
    log("generated %d + %d edges in %.1f s" % (args.serve_window, n_arr, time.perf_counter() - t0))
    out = []
    for rate in rates:
        graph, (s, d, l, ts) = synth.serving_times(edges, window_ticks=1 << 24, rate=rate)
        n = min(len(ts), int(rate * args.seconds))
        t1 = time.perf_counter()
        srv = serve.Server(graph, queries, window=1 << 24, flush_edges=65536, deadline=5000,
                           out_capacity=1 << 16, flags=binding.F_EMIT | binding.F_TIMING)
        log("rate %.0f: server up (%d edges, %d queries) in %.1f s" % (rate, len(graph["src"]), len(queries),
                                                                     time.perf_counter() - t1))
        eps, p50, p99 = serve.run_realtime(srv, s[:n], d[:n], l[:n], ts[:n])
        nb = len(srv.batches)
        ins = sum(b["n_ins"] for b in srv.batches)
        st = srv.m.stats()
        host = {k: v / max(1, nb) for k, v in srv.host_ms.items()}
        out.append({"rate": rate, "edges_per_s": eps, "insertions": ins, "batches": nb,
                    "mean_batch": ins / max(1, nb), "p50_ms": p50, "p99_ms": p99,
                    "slot_high_water": st["slot_high_water"], "host_ms_per_batch": host})
        log("rate %.0f: %.3gM edges/s processed, %d batches (mean %d insertions), p50 %.2f ms p99 %.2f ms; "
            "host ms per batch: form %.2f, apply %.2f (device %.2f), results %.2f" % (
                rate, eps / 1e6, nb, ins / max(1, nb), p50 or 0, p99 or 0, host["form"], host["apply"],
                host["device"], host["results"]))
        srv.close()
    top = out[-1]
    line = {"metric": METRIC, "value": top["edges_per_s"], "unit": "matched data edges/s", "n_gpus": 1,
            "steps": sum(o["batches"] for o in out), "warmup": 0,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
            "data": "synthetic (seeded R-MAT, Poisson arrivals; stand-in for the paper's sliding-window streams)",
            "config": {"workload": "serving_rmat_s%d_window%d_ticks%d_16q_temporal" % (
                args.serve_scale, args.serve_window, 1 << 24), "flush_edges": 65536, "deadline_us": 5000,
                "seconds_per_rate": args.seconds},
            "p50_batch_ms": top["p50_ms"], "p99_batch_ms": top["p99_ms"], "serving": out}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the matcher runs on a single MI355X; "
              "--gpus %d is not supported (how the path would shard is documented, not built)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        copy_calibration()
        return
    if args.workload == "serving":
        serving_bench(args)
        return

    import numpy as np
    import torch

    from paper_2206_09983_amd import binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    binding.load()  # raises if the HIP library is missing: there is no other path
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    # the whole 2^23-insertion stream is always drawn, so the graph and every
    # batch are the same whatever --steps and --warmup say
    if args.workload == "multiquery":
        with open(os.path.join(ROOT, "tests", "golden", "multiquery_queries.json")) as f:
            qdoc = json.load(f)
        case = synth.multiquery_case(scale=args.scale, n_init=args.n_init, del_frac=args.del_frac, seed=args.seed,
                                     queries=synth.queries_from_json(qdoc["queries"]))
    else:
        case = synth.rmat_case(scale=args.scale, n_init=args.n_init,
                               n_stream=max(1 << 23, (args.warmup + args.steps) * args.batch),
                               batch=args.batch, del_frac=args.del_frac, seed=args.seed, query_seed=7)
    log("generated %s: %d initial edges, %d batches in %.1f s" % (case["name"], len(case["graph"]["src"]),
                                                                   len(case["batches"]), time.perf_counter() - t0))
    timed = timed_batches(len(case["batches"]), args.warmup, args.steps)
    n_batches = timed[-1] + 1
    log("timed batches: %s" % describe_batches(timed))
    stream = torch.cuda.current_stream()
    dev_batches = []
    for b in case["batches"][:n_batches]:
        dev_batches.append({"src": torch.from_numpy(b["src"].view(np.int32)).cuda(),
                            "dst": torch.from_numpy(b["dst"].view(np.int32)).cuda(),
                            "elabel": torch.from_numpy(b["elabel"]).cuda(),
                            "ts": torch.from_numpy(b["ts"]).cuda(),
                            "del_keys": torch.from_numpy(b["del_keys"].view(np.int64)).cuda()})
    torch.cuda.synchronize()
    flags = binding.F_TIMING | (0 if args.count_only else binding.F_EMIT) | (binding.F_AUTOTUNE if args.autotune else 0)
    if args.tree_filter:
        flags |= binding.F_TREE_FILTER
    if args.workload == "multiquery":
        args.out_capacity = min(args.out_capacity, 1 << 16)  # 64 queries: buffers grow on demand
    weights = None
    if args.scheduler != "static":
        from paper_2206_09983_amd import sched
        try:
            weights = sched.load_weights(args.weights)
        except FileNotFoundError:
            if args.scheduler == "learned":
                raise
            log("no order-cost network weights found: timing the static order only")
            args.scheduler = "static"

    def run(mode, tag, fl=None):
        """Warm-up, then the timed steps, under one scheduler mode (and flags)."""
        t0 = time.perf_counter()
        m = binding.Matcher(case["graph"], case["queries"], flags=flags if fl is None else fl,
                            out_capacity=args.out_capacity,
                            stream=stream.cuda_stream, n_elabels=32)
        m.set_scheduler(mode, weights if mode == binding.SCHED_LEARNED else None)
        torch.cuda.synchronize()
        log("[%s] create (upload + sort + index of %d edges): %.2f s" % (
            tag, len(case["graph"]["src"]), time.perf_counter() - t0))
        for i in range(args.warmup):
            m.apply_batch(dev_batches[i])
            st = m.stats()
            log("[%s] warmup %d: %d insertions, %.2f ms, tuples %s, tile %d" % (
                tag, i, len(case["batches"][i]["src"]), st["ms_batch"], st["tuples"], st["expand_tile"]))
        r = {"lat": [], "tot": {k: 0 for k in BYTES}, "expand_ms": 0.0, "launches": 0, "rows": 0, "tuples": 0,
             "edges": 0, "results": []}
        steps = []
        want = set(timed)
        gc.collect()
        gc.disable()  # no collector pass inside the timed region
        for i in range(args.warmup, n_batches):
            if i not in want:  # between timed steps the stream goes on, untimed
                m.apply_batch(dev_batches[i])
                continue
            torch.cuda.synchronize()
            tb = time.perf_counter()
            m.apply_batch(dev_batches[i])  # returns once the batch's counts and digests are on the host
            torch.cuda.synchronize()
            r["lat"].append((time.perf_counter() - tb) * 1e3)
            st = m.stats()
            for p in range(2):
                r["launches"] += st["expand_launches"][p]
                r["expand_ms"] += st["ms_expand"][p]
                r["rows"] += st["frontier_rows"][p]
                for k in BYTES:
                    r["tot"][k] += st[k][p]
            r["tuples"] += st["tuples"][0] + st["tuples"][1]
            r["edges"] += len(case["batches"][i]["src"]) + len(case["batches"][i]["del_keys"])
            res = [m.result(q) for q in range(len(case["queries"]))]
            r["results"].append([(x["n_new"], x["dig_new"], x["n_expired"], x["dig_expired"]) for x in res])
            steps.append((i, r["lat"][-1], st))
        gc.enable()
        r["elapsed"] = sum(r["lat"]) * 1e-3
        for i, lat, st in steps:  # logged after the timed region
            log("[%s] step %d: %.2f ms (enumerate %.2f + %.2f ms, of which k_expand %.2f + %.2f ms in %s launches), "
                "seeds %s, rows %s, candidates %s, tuples %s%s" % (
                    tag, i, lat, st["ms_enumerate"][0], st["ms_enumerate"][1], st["ms_expand"][0],
                    st["ms_expand"][1], st["expand_launches"], st["seeds"], st["frontier_rows"],
                    st["entries_scanned"], st["tuples"],
                    (", re-runs %s (causes %s)" % (st["reruns"], st["rerun_causes"]) if any(st["reruns"]) else "") +
                    (", %d allocations in %.2f ms" % (st["allocations"], st["ms_alloc"]) if st["allocations"] else "")))
        r["tile"] = m.stats()["expand_tile"]
        m.close()
        return r

    main_mode = binding.SCHED_LEARNED if args.scheduler == "learned" else binding.SCHED_STATIC
    R = run(main_mode, args.scheduler if args.scheduler != "both" else "static")
    lat, tot, expand_ms, launches = R["lat"], R["tot"], R["expand_ms"], R["launches"]
    rows, tuples, edges, elapsed, m_tile = R["rows"], R["tuples"], R["edges"], R["elapsed"], R["tile"]
    learned = None
    if args.scheduler == "both":
        L = run(binding.SCHED_LEARNED, "learned")
        learned = {"value": L["edges"] / L["elapsed"], "ms_per_step": L["elapsed"] * 1e3 / args.steps,
                   "ratio": (L["edges"] / L["elapsed"]) / (edges / elapsed),
                   "identical_results": L["results"] == R["results"],
                   "candidates": L["tot"]["entries_scanned"], "candidates_static": tot["entries_scanned"],
                   "p99_batch_ms": sorted(L["lat"])[min(len(L["lat"]) - 1, int(np.ceil(0.99 * len(L["lat"]))) - 1)]}
        log("learned scheduler: %.3f ms per step vs %.3f (x%.3f), identical results: %s" % (
            learned["ms_per_step"], elapsed * 1e3 / args.steps, learned["ratio"], learned["identical_results"]))
        if not learned["identical_results"]:
            raise SystemExit("the learned scheduler changed the results")
    # the same batches without writing tuples (counts and digests only), and
    # with the index maintained but nothing enumerated
    rates = None
    if args.scheduler == "both" and not args.count_only and not args.no_rates:
        C = run(binding.SCHED_STATIC, "count-only", binding.F_TIMING)
        I = run(binding.SCHED_STATIC, "index-only", binding.F_TIMING | binding.F_INDEX_ONLY)
        if C["results"] != R["results"]:
            raise SystemExit("count-only mode changed the counts or digests")
        rates = {"count_only": C["edges"] / C["elapsed"], "index_only": I["edges"] / I["elapsed"],
                 "count_only_ms_per_step": C["elapsed"] * 1e3 / args.steps,
                 "index_only_ms_per_step": I["elapsed"] * 1e3 / args.steps,
                 "count_only_median_batch_ms": float(np.median(C["lat"])),
                 "index_only_median_batch_ms": float(np.median(I["lat"]))}
        log("count-only %.3f ms per step, index-only %.3f ms per step" % (
            rates["count_only_ms_per_step"], rates["index_only_ms_per_step"]))

    if args.count_only:
        tot["tuple_words"] = 0
    alg_bytes = sum(BYTES[k] * tot[k] for k in BYTES)
    per_launch = alg_bytes / max(launches, 1)
    avg_ms = expand_ms / max(launches, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = read_traffic(args.workload, args.steps, args.warmup)
    lat_s = sorted(lat)

    def pct(p):
        return lat_s[min(len(lat_s) - 1, int(np.ceil(p / 100.0 * len(lat_s))) - 1)]

    out = {
        "metric": METRIC,
        "value": edges / elapsed,
        "unit": "matched data edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded R-MAT stream, stand-in for the paper's NetFlow/LSBench streams)",
        "config": ({
            "workload": "rmat_s%d_init%d_batch%d_del%d%%_tt_c4_p5_iso_homo" % (
                args.scale, args.n_init, args.batch, int(round(args.del_frac * 100))),
            "vertices": 1 << args.scale, "initial_edges": args.n_init, "batch_insertions": args.batch,
            "batch_deletions": int(args.del_frac * args.batch), "queries": [q["name"] for q in case["queries"]],
            "emit_tuples": not args.count_only, "seed": args.seed,
            "stream_batches": len(case["batches"]), "timed_batches": describe_batches(timed),
        } if args.workload == "rmat" else {
            "workload": "rmat_s%d_init%d_logbatch1000-262144_del%d%%_64q" % (
                args.scale, args.n_init, int(round(args.del_frac * 100))),
            "vertices": 1 << args.scale, "initial_edges": args.n_init,
            "batch_insertions": [len(case["batches"][i]["src"]) for i in timed],
            "queries": len(case["queries"]), "emit_tuples": not args.count_only, "seed": args.seed,
            "stream_batches": len(case["batches"]), "timed_batches": describe_batches(timed),
            "autotune": bool(args.autotune), "expand_tile": m_tile, "tree_filter": bool(args.tree_filter),
        }),
        "embeddings_per_s": tuples / elapsed,
        "p50_batch_ms": pct(50),
        "p99_batch_ms": pct(99),
        "scheduler": args.scheduler if args.scheduler != "both" else "static",
        "learned_vs_plain": learned["ratio"] if learned else None,
        "learned": learned,
        "rates": rates,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_expand", "alg_bytes_per_launch": per_launch, "avg_launch_ms": avg_ms,
            "launches": launches, "sum_launch_ms": expand_ms, "frontier_rows_per_launch": rows / max(launches, 1),
            # each term of the byte model over the timed steps: units counted and bytes per unit
            "terms": {k: {"units": tot[k], "bytes_per_unit": BYTES[k], "bytes": BYTES[k] * tot[k]} for k in BYTES},
        },
    }
    # the achievable HBM rate on this device (a plain copy), beside the published peak
    cg = copy_gbps()
    out["roofline"]["copy_gbps"] = cg
    out["roofline"]["frac_of_copy"] = achieved / cg if cg else None
    if not args.no_cpu_baseline:
        rate, desc, _, core = cpu_baseline(case, args.cpu_seconds)
        out["cpu_baseline"] = {"value": rate, "unit": "matched data edges/s", "cores": 1, "kind": "oracle",
                               "sample": desc, "pinned_core": core, "cpu_model": cpu_model(),
                               "host_threads": os.cpu_count()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
