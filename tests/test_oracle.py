"""Pins of the CPU oracle against things other than itself (no GPU needed).

Each test checks the oracle against what the paper or mathematics fixes:
published hash test vectors, brute force from the definition, the paper's
worked example, recompute invariants, closed forms and special cases.
"""
import json
import os

import numpy as np
import pytest

from oracle import brute, closed_form
from oracle.core import SEED_A, Oracle, digest_of, mix64, tuple_hash
from paper_2206_09983_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- hashing
def test_splitmix64_published_vectors():
    # SplitMix64 (Steele, Lea, Flood 2014) seeded with 1234567: the widely
    # published first five outputs. The generator adds the golden gamma to the
    # state, then applies the output finaliser the digests use.
    gamma = 0x9E3779B97F4A7C15
    out = [mix64((1234567 + i * gamma) % 2**64) for i in range(1, 6)]
    assert out == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]
    assert mix64(gamma) == 0xE220A8397B1DCDAF  # seed 0, first output


def test_tuple_hash_is_ordered_chain():
    # h(t) = mix(...mix(mix(s ^ q) + k0)... + k_last): order of keys matters,
    # and the query index enters the first step.
    assert tuple_hash(SEED_A, 0, [1, 2]) != tuple_hash(SEED_A, 0, [2, 1])
    assert tuple_hash(SEED_A, 0, [1, 2]) != tuple_hash(SEED_A, 1, [1, 2])
    h = mix64(SEED_A ^ 3)
    for k in (5, 9, 11):
        h = mix64((h + k) % 2**64)
    assert tuple_hash(SEED_A, 3, [5, 9, 11]) == h


# ---------------------------------------------------------------- brute force
def _check_against_brute(case):
    for q in case["queries"]:
        m = len(q["qsrc"])
        ref = brute.run_stream(case["graph"], case["batches"], q)
        o = Oracle(case["graph"], [q])
        n_seen = 0
        for bi, b in enumerate(case["batches"]):
            o.apply_batch(b)
            new, exp = o.result(0), o.result(0, True)
            np.testing.assert_array_equal(new, brute.as_array(ref[bi][0], m))
            np.testing.assert_array_equal(exp, brute.as_array(ref[bi][1], m))
            # no duplicates in the incremental lists
            assert len(np.unique(new, axis=0)) == len(new)
            assert len(np.unique(exp, axis=0)) == len(exp)
            n_seen += len(new) + len(exp)
        o.close()
    return n_seen


@pytest.mark.parametrize("block", range(6))
def test_oracle_equals_brute_force_random_multigraphs(block):
    total = 0
    for seed in range(block * 60, block * 60 + 60):
        total += _check_against_brute(synth.tiny_case(seed))
    assert total > 50  # the cases are not all empty


def test_oracle_equals_brute_force_denser_queries():
    total = 0
    for seed in range(1000, 1040):
        case = synth.tiny_case(seed, max_v=4, max_init=12, max_ins=5, n_vlabels=1, n_elabels=1,
                               max_qv=4, wild_p=0.6)
        total += _check_against_brute(case)
    assert total > 200


def test_self_loops_only_match_under_homomorphism():
    # A data self-loop v->v can serve a query edge a->b only when f(a)=f(b),
    # which isomorphism forbids.
    g = synth.make_graph(2, [1, 1], [0], [1], [0])
    b = synth.make_batch([0], [0], [0], [1], [])
    for sem, expect in ((synth.ISO, 0), (synth.HOMO, 1)):
        q = synth.make_query(2, [0, 0], [(0, 1, -1)], sem)
        o = Oracle(g, [q])
        o.apply_batch(b)
        assert o.count(0) == expect
        o.close()


def test_parallel_edges_are_distinct_instances():
    # Three parallel (0->1) edges and one (1->2): a 2-edge path has 3 embeddings.
    g = synth.make_graph(3, [1, 1, 1], [0, 0, 1], [1, 1, 2], [0, 0, 0])
    q = synth.make_query(3, [0, 0, 0], [(0, 1, -1), (1, 2, -1)], synth.ISO)
    o = Oracle(g, [q])
    o.apply_batch(synth.make_batch([0], [1], [0], [3], []))
    new = o.result(0)
    assert new.tolist() == [[3, 2]]
    assert len(o.static(0)) == 3
    o.close()


# ---------------------------------------------------------------- worked example
def _paper_example():
    with open(os.path.join(GOLDEN, "paper_example.json")) as f:
        fx = json.load(f)
    e = np.array(fx["initial_edges"], dtype=np.int64)
    g = synth.make_graph(fx["n_vertices"], fx["vlabel_mask"], e[:, 0], e[:, 1], e[:, 2])
    qd = fx["query"]
    batches = []
    nk = len(e)
    for b in fx["batches"]:
        ins = np.array(b["insert"], dtype=np.int64).reshape(-1, 3)
        ts = np.arange(nk, nk + len(ins))
        nk += len(ins)
        batches.append(synth.make_batch(ins[:, 0], ins[:, 1], ins[:, 2], ts, b["delete"]))
    return fx, g, qd, batches


def test_paper_example_printed_values():
    fx, g, qd, batches = _paper_example()
    q = synth.make_query(qd["n_qv"], qd["vreq"], qd["edges"], synth.ISO)
    o = Oracle(g, [q])
    # Section II-B: two isomorphic embeddings at time t, printed as vertex pairs.
    s_g = o.static(0)
    pairs = sorted([[[int(g["src"][k]), int(g["dst"][k])] for k in row] for row in s_g])
    assert pairs == sorted(fx["printed"]["iso_at_t_pairs"]["value"])
    # Section VI: exactly the two printed new embeddings at t1.
    o.apply_batch(batches[0])
    pr = fx["printed"]["iso_new_at_t1_ids_start_order"]
    order = pr["order"]
    got = sorted([[int(row[k]) for k in order] for row in o.result(0)])
    assert got == sorted(pr["value"])
    assert o.count(0, expired=True) == 0
    o.close()


def test_paper_example_all_snapshots_vs_brute_force():
    fx, g, qd, batches = _paper_example()
    for sem in (synth.ISO, synth.HOMO):
        q = synth.make_query(qd["n_qv"], qd["vreq"], qd["edges"], sem)
        ref = brute.run_stream(g, batches, q)
        o = Oracle(g, [q])
        for bi, b in enumerate(batches):
            o.apply_batch(b)
            np.testing.assert_array_equal(o.result(0), brute.as_array(ref[bi][0], 7))
            np.testing.assert_array_equal(o.result(0, True), brute.as_array(ref[bi][1], 7))
        o.close()


# ---------------------------------------------------------------- invariants
def _recompute_check(case, batches, qidx_list=None):
    qs = case["queries"]
    o_inc = Oracle(case["graph"], qs)
    o_st = Oracle(case["graph"], qs)
    nonzero = 0
    for b in batches:
        before = [o_st.static(i) for i in range(len(qs))]
        o_st.insert(b, enumerate=False)
        mid = [o_st.static(i) for i in range(len(qs))]
        o_st.delete(b["del_keys"], enumerate=False)
        after = [o_st.static(i) for i in range(len(qs))]
        o_inc.apply_batch(b)
        for i in range(len(qs)):
            sm, sb, sa = ({tuple(r) for r in x[i]} for x in (mid, before, after))
            new = {tuple(r) for r in o_inc.result(i)}
            exp = {tuple(r) for r in o_inc.result(i, True)}
            assert new == sm - sb
            assert exp == sm - sa
            assert len(new) == o_inc.count(i) and len(exp) == o_inc.count(i, True)
            nonzero += len(new) + len(exp)
    o_inc.close()
    o_st.close()
    return nonzero


def test_incremental_equals_recompute_chung_lu():
    case = synth.chung_lu_case()
    assert _recompute_check(case, case["batches"]) > 0


def test_incremental_equals_recompute_small_rmat_with_deletions():
    case = synth.rmat_case(scale=9, n_init=4000, n_stream=1024, batch=256, n_batches=4)
    assert sum(len(b["del_keys"]) for b in case["batches"]) > 0
    assert _recompute_check(case, case["batches"]) > 0


def test_batch_size_invariance_insert_only():
    # For an insert-only stream the union of new embeddings over batches is
    # S(G_final) - S(G_0), whatever the batch size; the lists never overlap.
    base = synth.chung_lu_case(n=300, n_init=1500, n_stream=300, batch=300, n_vlabels=2, n_elabels=2)
    g, all_ins = base["graph"], base["batches"][0]
    c4 = [(0, 1, 0), (1, 2, 1), (2, 3, 0), (3, 0, 1)]
    q = [synth.make_query(4, [1, 2, 1, 2], c4, synth.ISO), synth.make_query(4, [1, 2, 1, 2], c4, synth.HOMO),
         synth.make_query(3, [0, 0, 0], [(0, 1, 0), (1, 2, -1)], synth.ISO)]
    o_ref = Oracle(g, q)
    s0 = [{tuple(r) for r in o_ref.static(i)} for i in range(len(q))]
    o_ref.insert(all_ins, enumerate=False)
    s1 = [{tuple(r) for r in o_ref.static(i)} for i in range(len(q))]
    o_ref.close()
    n = len(all_ins["src"])
    for bs in (1, 7, 256, n):
        o = Oracle(g, q)
        acc = [[] for _ in q]
        for lo in range(0, n, bs):
            sl = slice(lo, lo + bs)
            o.apply_batch(synth.make_batch(all_ins["src"][sl], all_ins["dst"][sl], all_ins["elabel"][sl],
                                           all_ins["ts"][sl], []))
            for i in range(len(q)):
                acc[i].extend(tuple(r) for r in o.result(i))
        for i in range(len(q)):
            assert len(acc[i]) == len(set(acc[i]))
            assert set(acc[i]) == s1[i] - s0[i]
        o.close()
    assert any(len(s1[i] - s0[i]) for i in range(len(q)))


def test_iso_subset_of_homo_and_equal_when_labels_force_injectivity():
    case = synth.rmat_case(scale=8, n_init=3000, n_stream=512, batch=256, n_batches=2,
                           n_vlabels=4, n_elabels=2)
    g = case["graph"]
    # distinct single labels on every query vertex -> f is injective anyway
    forced = synth.make_query(3, [1, 2, 4], [(0, 1, 0), (1, 2, 1), (2, 0, 0)], synth.ISO)
    forced_h = dict(forced, sem=synth.HOMO)
    loose = synth.make_query(3, [1, 1, 1], [(0, 1, -1), (1, 2, -1)], synth.ISO)
    loose_h = dict(loose, sem=synth.HOMO)
    o = Oracle(g, [forced, forced_h, loose, loose_h])
    strict = 0
    for b in case["batches"]:
        o.apply_batch(b)
        for ph in (False, True):
            np.testing.assert_array_equal(o.result(0, ph), o.result(1, ph))
            iso = {tuple(r) for r in o.result(2, ph)}
            hom = {tuple(r) for r in o.result(3, ph)}
            assert iso <= hom
            strict += len(hom) - len(iso)
    assert strict > 0
    o.close()


def test_single_edge_query_is_the_predicate():
    # One query edge: the new embeddings are exactly the batch edges that
    # satisfy the edge and endpoint predicates.
    case = synth.rmat_case(scale=8, n_init=2000, n_stream=512, batch=256, n_batches=2, n_vlabels=3,
                           n_elabels=3)
    g = case["graph"]
    q = synth.make_query(2, [1, 2], [(0, 1, 1)], synth.ISO)
    o = Oracle(g, [q])
    nk = len(g["src"])
    for b in case["batches"]:
        o.apply_batch(b)
        vm = g["vlabel_mask"]
        ok = ((b["elabel"] == 1) & ((vm[b["src"]] & 1) != 0) & ((vm[b["dst"]] & 2) != 0)
              & (b["src"] != b["dst"]))
        keys = np.arange(nk, nk + len(b["src"]), dtype=np.uint64)[ok]
        np.testing.assert_array_equal(o.result(0)[:, 0], keys)
        nk += len(b["src"])
    o.close()


def test_homomorphic_path_counts_match_closed_form():
    case = synth.rmat_case(scale=9, n_init=5000, n_stream=1024, batch=512, n_batches=2)
    g, batches = case["graph"], case["batches"]
    qs = [q for q in case["queries"] if q["name"] == "p5_homo"]
    # widen the labels so the counts are non-trivial at this size
    q = dict(qs[0])
    q["vreq"] = np.zeros(5, dtype=np.uint64)
    q["qlabel"] = np.array([0, 1, 0, 1], dtype=np.int32)
    o = Oracle(g, [q])
    n = g["n_vertices"]
    vm = g["vlabel_mask"]
    prev = closed_form.hom_count_tree(n, vm, g["src"], g["dst"], g["elabel"], q)[0]
    nonzero = 0
    for i, b in enumerate(batches):
        o.apply_batch(b)
        s, d, l = closed_form.graph_arrays_after(g, batches, i + 1, last_insert_only=True)
        mid, est = closed_form.hom_count_tree(n, vm, s, d, l, q)
        s, d, l = closed_form.graph_arrays_after(g, batches, i + 1)
        after = closed_form.hom_count_tree(n, vm, s, d, l, q)[0]
        assert est < 2**63
        assert o.count(0) == mid - prev
        assert o.count(0, True) == mid - after
        nonzero += mid - prev
        prev = after
    assert nonzero > 0
    o.close()


def test_digest_matches_list():
    case = synth.chung_lu_case()
    o = Oracle(case["graph"], case["queries"])
    o.apply_batch(case["batches"][0])
    for i in range(len(case["queries"])):
        assert o.digest(i) == digest_of(o.result(i), i)
    o.close()


def test_rejects_bad_batches_and_unsupported_queries():
    g = synth.make_graph(3, [1, 1, 1], [0], [1], [0])
    q = synth.make_query(2, [0, 0], [(0, 1, -1)], synth.ISO)
    o = Oracle(g, [q])
    with pytest.raises(ValueError):
        o.apply_batch(synth.make_batch([0], [7], [0], [5], []))  # vertex out of range
    with pytest.raises(ValueError):
        o.apply_batch(synth.make_batch([], [], [], [], [0, 0]))  # repeated key
    with pytest.raises(ValueError):
        o.apply_batch(synth.make_batch([], [], [], [], [9]))  # unknown key
    o.apply_batch(synth.make_batch([1], [2], [0], [1], [1]))  # may delete its own insert
    assert o.n_live == 1
    with pytest.raises(ValueError):
        Oracle(g, [synth.make_query(2, [0, 0], [(0, 0, -1)], synth.ISO)])  # self-loop
    with pytest.raises(ValueError):
        Oracle(g, [synth.make_query(3, [0, 0, 0], [(0, 1, -1)], synth.ISO)])  # disconnected
    o.close()


# ------------------------------------------------------------ temporal order
@pytest.mark.parametrize("ties", [False, True])
def test_temporal_oracle_equals_brute_force(ties):
    # random ranks (ties and unranked edges included); with ties, pairs of
    # edges share a timestamp, so the strict order rejects them
    total = 0
    for seed in range(120):
        total += _check_against_brute(synth.temporal_tiny_case(seed, ts_ties=ties))
    assert total > 20


def test_temporal_rank_permutations_partition_the_embeddings():
    # with distinct timestamps, an isomorphic embedding maps its m query
    # edges to m distinct data edges (f is injective), which come in exactly
    # one time order: the m! strict rank orders split the unconstrained set.
    # (Under homomorphism two query edges may share a data edge, whose equal
    # timestamps no strict order accepts.)
    import itertools
    checked = 0
    for seed in range(200, 300):
        case = synth.tiny_case(seed, max_qv=3)
        q = case["queries"][0]
        m = len(q["qsrc"])
        if m > 4:
            continue
        perms = list(itertools.permutations(range(m)))
        qs = [q] + [synth.with_ranks(q, p) for p in perms]
        o = Oracle(case["graph"], qs)
        for b in case["batches"]:
            o.apply_batch(b)
            for ph in (False, True):
                whole = o.result(0, ph)
                parts = [o.result(1 + i, ph) for i in range(len(perms))]
                assert sum(len(p) for p in parts) == len(whole)
                if len(whole):
                    joined = np.concatenate([p for p in parts if len(p)])
                    joined = joined[np.lexsort(joined.T[::-1])]
                    np.testing.assert_array_equal(joined, whole)
                checked += len(whole)
        o.close()
    assert checked > 50


def test_equal_or_missing_ranks_change_nothing():
    for seed in range(300, 330):
        case = synth.tiny_case(seed)
        q = case["queries"][0]
        m = len(q["qsrc"])
        qs = [q, synth.with_ranks(q, [0] * m), synth.with_ranks(q, [-1] * m)]
        o = Oracle(case["graph"], qs)
        for b in case["batches"]:
            o.apply_batch(b)
            for ph in (False, True):
                np.testing.assert_array_equal(o.result(1, ph), o.result(0, ph))
                np.testing.assert_array_equal(o.result(2, ph), o.result(0, ph))
        o.close()


# ---------------------------------------------------------------- work units
def _units_of_phase(o, qi, keys, n_qe, mode):
    """Per work unit (edge key at position j) lists of one phase, by orc_seed."""
    out = []
    for k in keys:
        for j in range(n_qe):
            rows, ovf = o.seed(qi, int(k), j, mode)
            assert ovf == 0
            out.append((int(k), j, rows))
    return out


def _check_units(units, batch_keys, expect, n_qe):
    """Section VI's exactly-once argument, stated on the lists themselves:
    every tuple of unit (k, j) maps q_j to k and uses no batch edge at a
    position before j; the units' lists are disjoint, and their union is the
    phase's list `expect` (sorted)."""
    batch = {int(x) for x in batch_keys}
    seen = set()
    total = 0
    for k, j, rows in units:
        for r in rows.tolist():
            assert r[j] == k
            assert not any(r[i] in batch for i in range(j))
            t = tuple(r)
            assert t not in seen  # disjoint units
            seen.add(t)
            total += 1
    assert total == len(expect)
    assert sorted(seen) == [tuple(r) for r in expect.tolist()]


def _per_unit_stream(case, ref_lists):
    """Walks the stream with insert(enumerate=False) + per-unit seeds (mode
    1), then mark + per-unit seeds (mode 2); ref_lists[qi][bi] = (new,
    expired) sorted arrays to compare the unions with."""
    qs = case["queries"]
    o = Oracle(case["graph"], qs)
    checked = 0
    for bi, b in enumerate(case["batches"]):
        first = o.insert(b, enumerate=False)
        ins_keys = range(first, first + len(b["src"]))
        for qi, q in enumerate(qs):
            m = len(q["qsrc"])
            _check_units(_units_of_phase(o, qi, ins_keys, m, 1), ins_keys, ref_lists[qi][bi][0], m)
            checked += len(ref_lists[qi][bi][0])
        dk = [int(x) for x in b["del_keys"]]
        o.mark(dk)
        for qi, q in enumerate(qs):
            m = len(q["qsrc"])
            _check_units(_units_of_phase(o, qi, dk, m, 2), dk, ref_lists[qi][bi][1], m)
            checked += len(ref_lists[qi][bi][1])
        # unmarking takes the mask away: a deleted key seeded with mode 2 now
        # sees the same embeddings as with no mask at all
        o.unmark(dk)
        for qi, q in enumerate(qs):
            for k in dk:
                for j in range(len(q["qsrc"])):
                    np.testing.assert_array_equal(o.seed(qi, k, j, 2)[0], o.seed(qi, k, j, 0)[0])
        o.delete(dk, enumerate=False)
    o.close()
    return checked


def test_work_units_partition_the_phase_lists_tiny():
    # Reference: brute force over every vertex map (independent of the
    # oracle's phase code), on tiny multigraph streams, iso and homo.
    checked = 0
    for seed in range(40):
        case = synth.tiny_case(seed)
        refs = []
        for q in case["queries"]:
            m = len(q["qsrc"])
            refs.append([(brute.as_array(n, m), brute.as_array(e, m))
                         for n, e in brute.run_stream(case["graph"], case["batches"], q)])
        checked += _per_unit_stream(case, refs)
    assert checked > 20


def test_work_units_partition_the_phase_lists_small_rmat():
    # Reference: the phase lists of a second oracle, which the recompute
    # invariant pins on this same stream.
    case = synth.rmat_case(scale=9, n_init=3000, n_stream=256, batch=128, n_batches=2, n_vlabels=3, n_elabels=4)
    o = Oracle(case["graph"], case["queries"])
    refs = [[] for _ in case["queries"]]
    for b in case["batches"]:
        o.apply_batch(b)
        for qi in range(len(case["queries"])):
            refs[qi].append((o.result(qi), o.result(qi, True)))
    o.close()
    assert _per_unit_stream(case, refs) > 10000


def test_mark_rejects_bad_keys_and_changes_nothing():
    case = synth.tiny_case(3, max_init=8)
    g = case["graph"]
    o = Oracle(g, case["queries"])
    n0 = len(g["src"])
    assert n0 >= 2
    for bad in ([0, 0], [n0 + 5], [1, n0 + 5]):
        with pytest.raises(ValueError):
            o.mark(bad)
        # nothing stays marked: mode 2 masks nothing, so every unit sees the
        # same embeddings as without a mask
        for k in range(n0):
            for j in range(len(case["queries"][0]["qsrc"])):
                np.testing.assert_array_equal(o.seed(0, k, j, 2)[0], o.seed(0, k, j, 0)[0])
    o.delete([0], enumerate=False)
    with pytest.raises(ValueError):
        o.mark([0])  # no longer live
    o.close()


def test_replay_without_enumeration_leaves_the_same_graph():
    # The full-size golden script splits a stream over worker processes, each
    # first applying the batches before its range without enumerating. The
    # batches after that point must give the results of an oracle that
    # enumerated every batch (both phases, temporal queries included).
    case = synth.rmat_case(scale=10, n_init=8000, n_stream=3072, batch=512, n_batches=6, n_vlabels=3, n_elabels=4)
    qs = case["queries"] + [synth.with_ranks(q, np.arange(len(q["qsrc"]))) for q in case["queries"][:2]]
    ref = Oracle(case["graph"], qs)
    res = []
    for b in case["batches"]:
        ref.apply_batch(b)
        res.append([(ref.count(q, ph), ref.digest(q, ph)) for q in range(len(qs)) for ph in (False, True)])
    ref.close()
    assert sum(c for r in res for c, _ in r) > 0
    for start in (1, 3, 5):
        part = Oracle(case["graph"], qs)
        try:
            for i, b in enumerate(case["batches"]):
                if i < start:
                    part.insert(b, enumerate=False)
                    part.delete(b["del_keys"], enumerate=False)
                else:
                    part.apply_batch(b)
                    got = [(part.count(q, ph), part.digest(q, ph)) for q in range(len(qs)) for ph in (False, True)]
                    assert got == res[i], (start, i)
        finally:
            part.close()
