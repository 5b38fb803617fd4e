"""Writes the full-size golden results: counts and both digests per batch,
query and phase, computed by the CPU oracle alone.

Test infrastructure, run once offline (it takes minutes of CPU time):
    python tests/golden/make_fullsize_golden.py rmat [W]    # fullsize_rmat_s20.json (W worker processes)
    python tests/golden/make_fullsize_golden.py multiquery  # fullsize_multiquery_s20.json
    python tests/golden/make_fullsize_golden.py serving     # fullsize_serving_s22.json
    python tests/golden/make_fullsize_golden.py multiquery_timed W  # fullsize_multiquery_timed_s20.json
Each file records the workload's parameters and the oracle's results for the
first batches of its stream: the R-MAT benchmark stream (2^20 vertices, 2^24
initial edges, batches of 65,536 insertions and 6,553 oldest-key deletions,
six queries), the 64-query stream (the same edges in log-uniform batches)
and a slice of the serving stream (2^22 vertices, a 2^26-edge window over
2^24 ticks, arrivals at 2e7 edges/s in batches of 65,536, each deleting what
left the window, 16 temporally ordered queries). Only oracle/ and the seeded
generators are used: no result here comes from the HIP library.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.core import Oracle  # noqa: E402
from paper_2206_09983_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

RMAT = dict(scale=20, n_init=1 << 24, n_stream=1 << 23, batch=65536, del_frac=0.10, seed=7, query_seed=7)
RMAT_BATCHES = 120  # through the benchmark's last timed batch (5 warm-up, then every 6th up to 119)
MULTI = dict(scale=20, n_init=1 << 24, del_frac=0.10, seed=7)
MULTI_BATCHES = 4
SERVING = dict(scale=22, n_window=1 << 26, rate=2e7, batch=65536, n_batches=2, window_ticks=1 << 24, seed=7)


def multiquery_queries():
    with open(os.path.join(HERE, "multiquery_queries.json")) as f:
        return synth.queries_from_json(json.load(f)["queries"])


def rmat_case():
    return synth.rmat_case(**RMAT)


def multiquery_case():
    return synth.multiquery_case(queries=multiquery_queries(), **MULTI)


def serving_case():
    # the serving workload's 16 queries, each ordered in time along its edges
    qs = [synth.with_ranks(q, np.arange(len(q["qsrc"]))) for q in multiquery_queries()[:16]]
    return synth.serving_case(qs, **SERVING)


def oracle_results(case, n_batches, first=0):
    """Results of batches [first, n_batches): the batches before `first` are
    applied without enumeration (the graph after them is the same)."""
    o = Oracle(case["graph"], case["queries"])
    out = []
    try:
        for i in range(first):
            b = case["batches"][i]
            o.insert(b, enumerate=False)
            o.delete(b["del_keys"], enumerate=False)
        for i in range(first, n_batches):
            b = case["batches"][i]
            t = time.perf_counter()
            o.apply_batch(b)
            rec = {"index": i, "n_ins": int(len(b["src"])), "n_del": int(len(b["del_keys"])), "queries": []}
            for qi, q in enumerate(case["queries"]):
                rq = {"name": q.get("name", "")}
                for ph, nm in ((False, "new"), (True, "expired")):
                    d = o.digest(qi, ph)
                    rq[nm] = [o.count(qi, ph), d[0], d[1]]
                rec["queries"].append(rq)
            out.append(rec)
            print("batch %d: %.1f s, %d new / %d expired embeddings" % (
                i, time.perf_counter() - t, sum(r["new"][0] for r in rec["queries"]),
                sum(r["expired"][0] for r in rec["queries"])), flush=True)
    finally:
        o.close()
    return out


def _chunk(args):
    which, lo, hi = args
    case = {"rmat": rmat_case, "multiquery": multiquery_case, "serving": serving_case}[which]()
    return oracle_results(case, hi, first=lo)


def _one(args):
    which, i = args
    case = {"rmat": rmat_case, "multiquery": multiquery_case, "serving": serving_case}[which]()
    return oracle_results(case, i + 1, first=i)[0]


def timed_indices(n_total, warmup, steps):
    """The batches the benchmark times: `steps` at an equal stride after the
    `warmup` first ones."""
    stride = max(1, (n_total - warmup) // steps)
    return [warmup + k * stride for k in range(steps)]


def parallel_results(which, n, workers):
    """Batches cut into `workers` consecutive ranges, each computed by its own
    oracle process that first replays the batches before its range."""
    import multiprocessing as mp
    bounds = [round(n * k / workers) for k in range(workers + 1)]
    jobs = [(which, bounds[k], bounds[k + 1]) for k in range(workers) if bounds[k] < bounds[k + 1]]
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        parts = pool.map(_chunk, jobs)
    return [rec for part in parts for rec in part]


def main_timed(workers):
    """The 64-query stream's 20 timed batches (5 warm-up, 20 steps), each by
    its own oracle process after replaying the batches before it."""
    import multiprocessing as mp
    t = time.perf_counter()
    case = multiquery_case()
    idx = timed_indices(len(case["batches"]), 5, 20)
    print("generated %s in %.1f s; batches %s" % (case["name"], time.perf_counter() - t, idx), flush=True)
    # the largest batches first, so that the pool's last jobs are short
    order = sorted(idx, key=lambda i: -len(case["batches"][i]["src"]))
    with mp.get_context("fork").Pool(workers) as pool:
        recs = pool.map(_one, [("multiquery", i) for i in order], chunksize=1)
    recs.sort(key=lambda r: r["index"])
    doc = {"workload": case["name"], "params": MULTI, "generator": "paper_2206_09983_amd.synth.multiquery_case",
           "command": "python tests/golden/make_fullsize_golden.py multiquery_timed %d" % workers,
           "queries": [q.get("name", "") for q in case["queries"]],
           "result_format": "per query and phase: [count, digest seed A, digest seed B] (digests mod 2^64)",
           "timed": {"warmup": 5, "steps": 20}, "batches": recs}
    with open(os.path.join(HERE, "fullsize_multiquery_timed_s20.json"), "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print("wrote fullsize_multiquery_timed_s20.json", flush=True)


def main(which, workers=1):
    if which == "multiquery_timed":
        return main_timed(workers)
    t = time.perf_counter()
    if which == "rmat":
        case, params, n, name = rmat_case(), RMAT, RMAT_BATCHES, "fullsize_rmat_s20.json"
    elif which == "multiquery":
        case, params, n, name = multiquery_case(), MULTI, MULTI_BATCHES, "fullsize_multiquery_s20.json"
    elif which == "serving":
        case, params, n, name = serving_case(), SERVING, SERVING["n_batches"], "fullsize_serving_s22.json"
    else:
        raise SystemExit("usage: make_fullsize_golden.py rmat|multiquery|serving")
    print("generated %s in %.1f s" % (case["name"], time.perf_counter() - t), flush=True)
    doc = {"workload": case["name"], "params": params, "generator": "paper_2206_09983_amd.synth." + which + "_case",
           "command": "python tests/golden/make_fullsize_golden.py " + which,
           "queries": [q.get("name", "") for q in case["queries"]],
           "result_format": "per query and phase: [count, digest seed A, digest seed B] (digests mod 2^64)",
           "batches": oracle_results(case, n) if workers <= 1 else parallel_results(which, n, workers)}
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print("wrote", name)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "rmat", int(sys.argv[2]) if len(sys.argv) > 2 else 1)
