"""Learned scheduler: traces, training and evaluation of the order-cost network.

The matcher keeps up to four matching orders per (query, start position); all
of them find the same embeddings, at different cost. The network predicts,
from 24 features of a start row under one order, log2 of the search work
below that row (1 + the candidates examined at every level). In
SCHED_LEARNED mode the seed kernel evaluates it (bf16) for every order of the
row's pair and takes the cheapest prediction.

This module drives the library only through its C ABI (binding.py): traces
come from the enumerator itself (mnemonic_set_trace / mnemonic_get_trace, one
pass per fixed order over the same batches), and training runs on the GPU
with the library's own forward/backward/Adam kernels (mnemonic_mlp_*).
Device memory and streams come from torch.

    python -m paper_2206_09983_amd.sched --out DIR [--entries N] [--batches B]

collects traces on streams drawn like the benchmark's (the six-query R-MAT
stream and the 64-query stream with log-uniform batches) with stream seed 9,
trains one network, and compares static, learned and per-row best orders on
held-out streams: seed 7, the benchmark's own, writing
DIR/sched_weights.json and DIR/sched_report.json.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import binding as B
from . import synth

MASK_VAR = ~np.uint64(0xFF << 56)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _device_batch(torch, b):
    return {"src": torch.from_numpy(np.ascontiguousarray(b["src"]).view(np.int32)).cuda(),
            "dst": torch.from_numpy(np.ascontiguousarray(b["dst"]).view(np.int32)).cuda(),
            "elabel": torch.from_numpy(np.ascontiguousarray(b["elabel"])).cuda(),
            "ts": torch.from_numpy(np.ascontiguousarray(b["ts"])).cuda(),
            "del_keys": torch.from_numpy(np.ascontiguousarray(b["del_keys"]).view(np.int64)).cuda()}


def collect(graph, queries, batches, max_entries=2_000_000, trace_cap=1 << 21, n_elabels=32, flags=0):
    """Start-row traces of `batches` under every fixed order.

    Returns x (n, 4, 24) float32 features of each order, work (n, 4) int64
    (-1 where the pair has no such order), n_orders (n,) and the static plan
    (n,) of every traced start row."""
    import torch
    stream = torch.cuda.current_stream()
    dev = [_device_batch(torch, b) for b in batches]
    per_run = []
    for v in range(B.MAX_ORDERS):
        m = B.Matcher(graph, queries, flags=flags, stream=stream.cuda_stream, n_elabels=n_elabels)
        try:
            m.set_scheduler(B.SCHED_FIXED + v)
            m.set_trace(trace_cap)
            recs = []
            got = 0
            for bi, db in enumerate(dev):
                torch.cuda.synchronize()
                m.apply_batch(db)
                for ph in (0, 1):
                    t = m.trace(ph, with_x=(v == 0))
                    recs.append((bi, t))
                    got += len(t["codes"])
                if v == 0 and got >= max_entries:
                    break
            per_run.append(recs)
        finally:
            m.close()
        if v == 0:
            dev = dev[:len(per_run[0]) // 2]
        say("traces under order %d: %d entries over %d batches" % (v, sum(len(t["codes"]) for _, t in per_run[v]),
                                                                   len(per_run[v]) // 2))
    xs, works, nvs, plans = [], [], [], []
    for i, (bi, t0) in enumerate(per_run[0]):
        codes0 = t0["codes"]
        key0 = codes0 & MASK_VAR
        order = np.argsort(key0, kind="stable")
        k0 = key0[order]
        n = len(k0)
        work = np.full((n, B.MAX_ORDERS), -1, dtype=np.int64)
        for v in range(B.MAX_ORDERS):
            tv = per_run[v][i][1]
            var = (tv["codes"] >> np.uint64(56)) & np.uint64(0xFF)
            sel = var == v
            kv = tv["codes"][sel] & MASK_VAR
            pos = np.searchsorted(k0, kv)
            ok = (pos < n) & (k0[np.minimum(pos, n - 1)] == kv)
            work[pos[ok], v] = tv["work"][sel][ok].astype(np.int64)
        x = t0["x"][order]
        nv = (work >= 0).sum(axis=1)
        keep = work[:, 0] >= 0
        xs.append(x[keep])
        works.append(work[keep])
        nvs.append(nv[keep])
        plans.append(((k0 >> np.uint64(32)) & np.uint64(0xFFFFFF)).astype(np.int64)[keep])
    return np.concatenate(xs), np.concatenate(works), np.concatenate(nvs), np.concatenate(plans)


def samples(x, work):
    """(features, log2 work) of every (entry, order) with a measured work."""
    e, v = np.nonzero(work >= 0)
    return np.ascontiguousarray(x[e, v]), np.log2(work[e, v].astype(np.float64)).astype(np.float32)


def train(X, Y, epochs=8, lr=1e-3, batch=4096, seed=7, init_scale=None, log_every=0):
    """Trains the network on the GPU with the library's kernels. Returns the
    fp32 weights (numpy) and the mean loss of each epoch."""
    import torch
    dev = torch.device("cuda")
    rng = np.random.default_rng(seed)
    fan = [(B.MLP_IN, B.MLP_HIDDEN), (B.MLP_HIDDEN, B.MLP_HIDDEN), (B.MLP_HIDDEN, 1)]
    parts = []
    for (fi, fo) in fan:  # He initialisation for ReLU layers, zero biases
        parts.append(rng.normal(0.0, np.sqrt(2.0 / fi) if init_scale is None else init_scale, fi * fo))
        parts.append(np.zeros(fo))
    w0 = np.concatenate(parts).astype(np.float32)
    w0[-1] = float(np.mean(Y))  # start at the mean target
    w = torch.from_numpy(w0).to(dev)
    m1 = torch.zeros_like(w)
    m2 = torch.zeros_like(w)
    grad = torch.zeros_like(w)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    Yd = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.float32)).to(dev)
    s = torch.cuda.current_stream().cuda_stream
    n = len(X)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n).astype(np.uint32)).to(dev)
        loss.zero_()
        nb = 0
        for off in range(0, n, batch):
            m = min(batch, n - off)
            step += 1
            B.mnemonic_mlp_grad(w, Xd, Yd, grad, loss, idx=perm, off=off, m=m, stream=s)
            B.mnemonic_mlp_adam(w, m1, m2, grad, lr, step, stream=s)
            nb += 1
        torch.cuda.synchronize()
        hist.append(float(loss.item()) / max(1, nb))
        if log_every and (ep + 1) % log_every == 0:
            say("epoch %d: mse %.4f" % (ep + 1, hist[-1]))
    return w.cpu().numpy(), hist


def predict(w, X, bf16=True):
    import torch
    dev = torch.device("cuda")
    wd = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).to(dev)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    y = torch.empty(len(X), dtype=torch.float32, device=dev)
    B.mnemonic_mlp_predict(wd, Xd, y, bf16=bf16, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def choice_work(w, x, work, plan=None, queries=None, bf16=True):
    """Total work of the static order, the network's choice and the best order
    per entry, on traced entries (and per query when plans are given)."""
    n = len(x)
    y = predict(w, x.reshape(-1, B.MLP_IN), bf16).reshape(n, B.MAX_ORDERS)
    y = np.where(work >= 0, y, np.inf)
    pick = np.argmin(y, axis=1)
    best = np.where(work >= 0, work, np.iinfo(np.int64).max).min(axis=1)
    chosen = work[np.arange(n), pick]
    # a plain rule for comparison: the order whose first level has the fewest candidates
    first = np.where(work >= 0, x[:, :, 4], np.inf)
    rule = work[np.arange(n), np.argmin(first, axis=1)]
    out = {"static": int(work[:, 0].sum()), "learned": int(chosen.sum()), "best": int(best.sum()),
           "smallest_first_level": int(rule.sum()), "entries": n, "picked_other": float(np.mean(pick != 0))}
    if plan is not None and queries is not None:
        base = np.cumsum([0] + [len(q["qsrc"]) for q in queries])
        qi = np.searchsorted(base, plan, side="right") - 1
        out["per_query"] = {q.get("name", str(i)): {"static": int(work[qi == i, 0].sum()),
                                                    "learned": int(chosen[qi == i].sum()),
                                                    "best": int(best[qi == i].sum())}
                            for i, q in enumerate(queries)}
    return out


def save_weights(w, path, meta):
    with open(path, "w") as f:
        json.dump({"n_weights": int(len(w)), "layout": "W1[24][64] b1[64] W2[64][64] b2[64] W3[64] b3",
                   "meta": meta, "weights": [float(v) for v in np.asarray(w, dtype=np.float32)]}, f)


def load_weights(path=None):
    path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), "sched_weights.json")
    with open(path) as f:
        d = json.load(f)
    w = np.asarray(d["weights"], dtype=np.float32)
    assert len(w) == B.MLP_WEIGHTS
    return w


def time_stream(graph, queries, batches, mode, weights=None, flags=B.F_EMIT, n_elabels=32, warmup=2,
                out_capacity=1 << 22):
    """Runs the stream under one scheduler mode; returns ms per batch (timed
    batches, wall clock), the expansion kernels' summed device time over the
    timed batches (expand_ms), per-batch (count, digest) results and
    enumeration work."""
    import torch
    stream = torch.cuda.current_stream()
    dev = [_device_batch(torch, b) for b in batches]
    m = B.Matcher(graph, queries, flags=flags | B.F_TIMING, stream=stream.cuda_stream, n_elabels=n_elabels,
                  out_capacity=out_capacity)
    res, ms, work, expand_ms = [], [], 0, 0.0
    try:
        m.set_scheduler(mode, weights)
        for bi, db in enumerate(dev):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m.apply_batch(db)
            dt = (time.perf_counter() - t0) * 1e3
            if bi >= warmup:
                ms.append(dt)
            st = m.stats()
            if bi >= warmup:
                expand_ms += sum(st["ms_expand"])
            work += sum(st["entries_scanned"]) + sum(st["seeds"])
            res.append([(r["n_new"], r["dig_new"], r["n_expired"], r["dig_expired"])
                        for r in (m.result(q) for q in range(len(queries)))])
    finally:
        m.close()
    return {"ms": float(np.mean(ms)) if ms else 0.0, "expand_ms": expand_ms, "results": res, "work": int(work)}


def workload(name, seed, scale=20):
    """The benchmark's streams: 'rmat' (six queries, batches of 65,536) or
    'multiquery' (64 queries, log-uniform batches), on stream seed `seed`."""
    kw = {} if scale == 20 else {"scale": scale, "n_init": 16 << scale, "n_stream": 8 << scale}
    if name == "rmat":
        return synth.rmat_case(seed=seed, query_seed=7, **kw)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "tests", "golden", "multiquery_queries.json")) as f:
        qdoc = json.load(f)
    return synth.multiquery_case(seed=seed, queries=synth.queries_from_json(qdoc["queries"]), **kw)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--entries", type=int, default=2_000_000, help="traced start rows per workload (at most)")
    ap.add_argument("--batches", type=int, default=128, help="most batches traced per workload")
    ap.add_argument("--epochs", type=int, default=48)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-batches", type=int, default=10)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--workloads", default="rmat,multiquery")
    ap.add_argument("--train-seed", type=int, default=9)
    ap.add_argument("--eval-seed", type=int, default=7)
    ap.add_argument("--eval-only", metavar="WEIGHTS", default=None,
                    help="evaluate these weights (a sched_weights.json) instead of training; the report's "
                         "validation uses the same held-back tenth of the training traces")
    a = ap.parse_args(argv)
    import torch
    os.makedirs(a.out, exist_ok=True)
    t0 = time.time()
    names = a.workloads.split(",")
    xs, ws, plans, queries = [], [], [], {}
    for name in names:
        case = workload(name, a.train_seed, a.scale)
        say("%s training stream: %d initial edges (%.0f s)" % (name, len(case["graph"]["src"]), time.time() - t0))
        x, work, nv, plan = collect(case["graph"], case["queries"], case["batches"][:a.batches], a.entries)
        say("%s: %d traced start rows, %.1f%% with more than one order (%.0f s)" % (
            name, len(x), 100.0 * np.mean(nv > 1), time.time() - t0))
        xs.append(x)
        ws.append(work)
        plans.append(plan)
        queries[name] = case["queries"]
        del case
    x, work = np.concatenate(xs), np.concatenate(ws)
    src = np.concatenate([np.full(len(v), i) for i, v in enumerate(xs)])
    plan = np.concatenate(plans)
    rng = np.random.default_rng(7)
    perm = rng.permutation(len(x))
    n_val = len(x) // 10
    val, tr = perm[:n_val], perm[n_val:]
    X, Y = samples(x[tr], work[tr])
    Xv, Yv = samples(x[val], work[val])
    if a.eval_only:
        w, hist = load_weights(a.eval_only), []
        with open(a.eval_only) as f:
            trained = json.load(f)["meta"]
        prev = os.path.join(os.path.dirname(os.path.abspath(a.eval_only)), "sched_report.json")
        if os.path.exists(prev):  # keep the loss curve of the run that trained these weights
            with open(prev) as f:
                hist = json.load(f)["train"].get("loss", [])
    else:
        w, hist = train(X, Y, epochs=a.epochs, lr=a.lr, log_every=1)
        trained = {"stream_seed": a.train_seed, "workloads": names, "entries": int(len(tr)), "epochs": a.epochs}
    yv = predict(w, Xv, bf16=True)
    val_mse = float(np.mean((yv - Yv) ** 2))
    base_mse = float(np.mean((Yv - np.mean(Y)) ** 2))
    report = {"train": dict(trained, samples=int(len(X)), loss=hist, evaluated_only=bool(a.eval_only)),
              "validation": {"mse": val_mse, "constant_mse": base_mse}, "held_out": {},
              "device": torch.cuda.get_device_name(0)}
    for i, name in enumerate(names):
        sel = val[src[val] == i]
        report["validation"][name] = choice_work(w, x[sel], work[sel], plan[sel], queries[name])
        say("validation %s: %s" % (name, json.dumps({k: v for k, v in report["validation"][name].items()
                                                      if k != "per_query"})))
    if not a.eval_only:
        save_weights(w, os.path.join(a.out, "sched_weights.json"), dict(trained, val_mse=val_mse))
    del x, work, xs, ws
    same_all = True
    for name in names:
        held = workload(name, a.eval_seed, a.scale)
        hb = held["batches"][:a.eval_batches]
        hx, hw, hnv, hplan = collect(held["graph"], held["queries"], hb, max_entries=1 << 40)
        cw = choice_work(w, hx, hw, hplan, held["queries"])
        runs = {}
        for tag, mode, wts in (("static", B.SCHED_STATIC, None), ("learned", B.SCHED_LEARNED, w)):
            runs[tag] = time_stream(held["graph"], held["queries"], hb, mode, wts,
                                    out_capacity=(1 << 16) if name == "multiquery" else (1 << 22))
            say("held-out %s %s: %.3f ms per batch, work %d" % (name, tag, runs[tag]["ms"], runs[tag]["work"]))
        same = runs["static"]["results"] == runs["learned"]["results"]
        same_all = same_all and same
        report["held_out"][name] = {
            "stream_seed": a.eval_seed, "batches": len(hb), "traced": cw,
            "ms_static": runs["static"]["ms"], "ms_learned": runs["learned"]["ms"],
            "work_static": runs["static"]["work"], "work_learned": runs["learned"]["work"],
            "speedup": runs["static"]["ms"] / max(1e-9, runs["learned"]["ms"]), "identical_results": bool(same)}
        say(json.dumps(report["held_out"][name]))
        del held
    with open(os.path.join(a.out, "sched_report.json"), "w") as f:
        json.dump(report, f, indent=1)
    if not same_all:
        say("ERROR: learned and static orders gave different results")
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
