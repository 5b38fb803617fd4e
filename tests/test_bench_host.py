"""Host-side checks of bench.py that need no GPU: the one-GPU refusal and the
CPU baseline's timing of the oracle (single thread, pinned, affinity restored)."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line for an unsupported run


def test_cpu_baseline_times_the_oracle_pinned_and_restores_affinity():
    bench = load_bench()
    from paper_2206_09983_amd import synth
    case = synth.rmat_case(scale=10, n_init=12000, n_stream=2048, batch=1024, n_batches=1)
    before = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    rate, desc, _, core = bench.cpu_baseline(case, 0.5)
    assert rate > 0
    assert "oracle, 1 thread" in desc
    if before is not None:
        assert core in before
        assert os.sched_getaffinity(0) == before


@pytest.mark.skipif(not os.path.exists("/proc/cpuinfo"), reason="no /proc/cpuinfo")
def test_cpu_model_is_read():
    assert load_bench().cpu_model()


def test_timed_batches_spread_over_the_stream():
    bench = load_bench()
    t = bench.timed_batches(128, 5, 20)
    assert len(t) == 20 and t[0] == 5 and t == sorted(set(t)) and t[-1] < 128
    assert t[1] - t[0] == (128 - 5) // 20  # equal stride over what follows the warm-up
    assert bench.timed_batches(25, 5, 20) == list(range(5, 25))  # no room for a stride: consecutive
    assert bench.describe_batches(t) == "5..119 step 6 (20 batches)"
    with pytest.raises(SystemExit):
        bench.timed_batches(10, 5, 20)


def test_byte_model_terms_follow_the_scope():
    # per unit: 8 B per work unit, 8 B entry + 4 B edge-index word + 4 B
    # filter word per candidate, 4 B per closing-edge probe, 8 B per tuple key
    bench = load_bench()
    assert bench.BYTES == {"seeds": 8, "entries_scanned": 16, "probe_words": 4, "tuple_words": 8}
