"""GPU tests of query-set changes and of the serving loop.

* mnemonic_set_queries rebuilds the query-dependent index in place: after any
  sequence of set changes (with deletions pending across the change) every
  active query's results equal the oracle's, which holds all queries all along.
* The serving loop on the HIP library: each query's per-batch results are the
  same alone and in a mix with admissions and retirements, and equal the
  oracle's on the same batches (sliding-window deletions, temporal orders).
"""
import numpy as np
import pytest

from oracle.core import Oracle, digest_of
from paper_2206_09983_amd import serve, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2206_09983_amd import binding
    binding.load()
    return binding


def canon(rows):
    rows = np.asarray(rows, dtype=np.uint64)
    if len(rows) == 0:
        return rows.reshape(0, rows.shape[1] if rows.ndim == 2 else 0)
    return rows[np.lexsort(rows.T[::-1])]


def test_set_queries_rebuilds_the_index(B):
    case = synth.rmat_case(scale=11, n_init=20000, n_stream=8192, batch=1024, n_batches=8, n_vlabels=3)
    qs = list(case["queries"])
    rng = np.random.default_rng(5)
    qs += [synth.with_ranks(q, np.arange(len(q["qsrc"]))) for q in case["queries"][:3]]
    qs += [q for q in synth.random_queries(16, seed=11, n_vlabels=3) if q["n_qv"] <= 5][:4]
    assert len(qs) == 13
    o = Oracle(case["graph"], qs)
    sets = [[0, 1], [6, 2, 9], [3], [10, 11, 4, 0, 7], [5, 8], [12, 9, 10], [1, 2, 3, 4], [9]]
    m = B.Matcher(case["graph"], [qs[i] for i in sets[0]])
    try:
        for bi, b in enumerate(case["batches"]):
            if bi:
                m.set_queries([qs[i] for i in sets[bi]])
            o.apply_batch(b)
            m.apply_batch(b)
            for pos, qi in enumerate(sets[bi]):
                r = m.result(pos)
                for ph in (False, True):
                    assert (r["n_expired"] if ph else r["n_new"]) == o.count(qi, ph), (bi, qi, ph)
                    # digests fold in the query's index in the matcher's current set
                    assert (r["dig_expired"] if ph else r["dig_new"]) == digest_of(o.result(qi, ph), pos), (bi, qi, ph)
                    np.testing.assert_array_equal(canon(m.keys(pos, ph)), o.result(qi, ph))
        # a rejected set changes nothing
        bad = synth.make_query(3, [0, 0, 0], [(0, 1, -1)], synth.ISO)
        with pytest.raises(B.MnemonicError):
            m.set_queries([qs[0], bad])
    finally:
        m.close()
        o.close()


def window_stream(seed=3, scale=11, n0=16000, n=12000, gap=4, window=40000):
    """An R-MAT stream with ts in ticks (gap ticks per edge on average,
    Poisson arrivals) whose initial window spans `window` ticks."""
    rng = np.random.default_rng(seed)
    base = synth.rmat_case(scale=scale, n_init=n0, n_stream=n, batch=n, n_batches=1, seed=seed, del_frac=0.0)
    g = dict(base["graph"])
    g["ts"] = np.sort(rng.integers(0, window, n0)).astype(np.int64)
    b = base["batches"][0]
    ts = (window + np.cumsum(rng.exponential(gap, n))).astype(np.int64)
    return g, b["src"], b["dst"], b["elabel"], ts, base["queries"]


def test_serving_results_alone_equal_in_the_mix_and_match_the_oracle(B):
    g, s, d, l, ts, base_q = window_stream()
    extra = [q for q in synth.random_queries(16, seed=21) if q["n_qv"] <= 5][:4]
    queries = [synth.with_ranks(q, np.arange(len(q["qsrc"]))) if i % 2 == 0 else q
               for i, q in enumerate(base_q + extra)]
    assert len(queries) == 10
    life = [3, 5, None, 4, 2, 6, 3, 5, 4, 2]
    cap = 1 << 12
    est = [serve.query_bytes(q, g["n_vertices"], cap) for q in queries]
    budget = sum(sorted(est)[-3:])  # about three queries at a time
    kw = dict(window=40000, flush_edges=1500, deadline=3000, out_capacity=cap, keep_lists=True)
    mix = serve.Server(g, [(queries[0], life[0]), (queries[1], life[1])], mem_budget=budget, **kw)
    for q, lf in zip(queries[2:], life[2:]):
        mix.submit(q, lf)
    serve.run_simulated(mix, s, d, l, ts)
    mix.close()
    n_b = len(mix.batches)
    assert n_b > 6 and max(len(b["active"]) for b in mix.batches) >= 2
    assert len({tuple(b["active"]) for b in mix.batches}) > 3  # admissions and retirements happened
    # the oracle on the mix's batches, holding every query throughout
    o = Oracle(g, queries)
    for b in mix.batches:
        k0 = b["first_key"] - len(g["src"])
        lo, cut = b["del_range"]
        o.apply_batch(synth.make_batch(s[k0:k0 + b["n_ins"]], d[k0:k0 + b["n_ins"]], l[k0:k0 + b["n_ins"]],
                                       ts[k0:k0 + b["n_ins"]], np.arange(lo, cut)))
        for qid, r in b["results"].items():
            pos = b["active"].index(qid)  # digests fold in the position in the matcher's set
            assert r["n_new"] == o.count(qid) and r["n_expired"] == o.count(qid, True)
            assert r["dig_new"] == digest_of(o.result(qid), pos)
            assert r["dig_expired"] == digest_of(o.result(qid, True), pos)
            np.testing.assert_array_equal(canon(r["new"]), o.result(qid))
            np.testing.assert_array_equal(canon(r["expired"]), o.result(qid, True))
    o.close()
    # each query alone over the same stream: the same batches, the same results
    for qid in range(len(queries)):
        alone = serve.Server(g, [queries[qid]], mem_budget=1 << 40, **kw)
        serve.run_simulated(alone, s, d, l, ts)
        alone.close()
        assert len(alone.batches) == n_b
        seen = 0
        for bm, ba in zip(mix.batches, alone.batches):
            assert (bm["first_key"], bm["n_ins"], bm["del_range"]) == (ba["first_key"], ba["n_ins"], ba["del_range"])
            if qid in bm["results"]:
                rm, ra = bm["results"][qid], ba["results"][0]
                for k in ("n_new", "n_expired"):
                    assert rm[k] == ra[k], (qid, k)
                np.testing.assert_array_equal(canon(rm["new"]), canon(ra["new"]))
                np.testing.assert_array_equal(canon(rm["expired"]), canon(ra["expired"]))
                seen += 1
        assert seen >= 1
