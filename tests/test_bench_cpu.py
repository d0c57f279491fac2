"""CPU checks of bench.py's command-line contract (no GPU needed)."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_counter_record_requires_matching_source_and_split():
    sys.path.insert(0, ROOT)
    import bench

    with open(bench.COUNTERS_FILE) as f:
        rec = json.load(f)
    entry = rec["c3:kahan"]
    cfg = {"nsplit": entry["nsplit"], "rows": entry.get("rows", 1)}
    if entry["kernel_sha"] == bench.kernel_source_sha():
        assert bench.counter_record("c3", "kahan", cfg) == entry
    assert bench.counter_record("c3", "kahan", dict(cfg, nsplit=cfg["nsplit"] + 1)) is None
    assert bench.counter_record("c3", "kahan", dict(cfg, rows=3)) is None
    assert bench.counter_record("c3", "nonexistent-mode", cfg) is None


def test_served_sample_takes_one_request_per_size_decile():
    sys.path.insert(0, ROOT)
    import bench

    trace, desc = bench.serving_trace("full")
    assert len(trace) == 256 and "256 requests" in desc
    sample = bench.served_sample(trace)
    assert len(sample) == 10
    ns = [r.n for r in sample]
    assert ns == sorted(ns)
    all_n = sorted(r.n for r in trace)
    for d, r in enumerate(sample):  # each pick lies inside its own tenth of the sizes
        assert all_n[d * 256 // 10] <= r.n <= all_n[(d + 1) * 256 // 10 - 1]
    assert len({r.rid for r in sample}) == 10


def test_kernel_hash_ignores_comments_only():
    """The counter records are keyed by a hash of the kernels' code: comments and layout may
    change without invalidating them, any change of code may not."""
    sys.path.insert(0, ROOT)
    import bench

    src = "int f(int a) {\n    // add one\n    return a + 1; /* done */\n}\n"
    assert bench.code_text(src) == bench.code_text("int f(int a) { return a + 1; }")
    assert bench.code_text(src) != bench.code_text(src.replace("a + 1", "a + 2"))
    assert bench.code_text(src) != bench.code_text(src.replace("// add one", "a = 0;"))
