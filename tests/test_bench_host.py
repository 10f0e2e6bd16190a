"""Host logic of the benchmark: the roofline record, the source hash that
ties committed counter summaries to the kernels, and the rejection of stale
summaries.  No GPU."""
import json
import os

import pytest

import bench

INFO = {"n": 1_000_000, "m": 10_000_000, "v_gang": 400_000, "m_gang_internal": 4_000_000, "m_gang_between": 100_000}


def test_segment_roofline_bytes_and_rates():
    st = {"kt_count": [2, 0, 0, 0], "kt_ms": [4.0, 0.0, 0.0, 0.0]}
    r = bench.roofline(0, INFO, st, 0, False, 3_000_000)
    rows = INFO["n"] - INFO["v_gang"]
    edges = INFO["m"] - INFO["m_gang_internal"] - INFO["m_gang_between"]
    per_launch = (rows * bench.B_ONCE_ROW + edges * bench.B_ONCE_EDGE) / 2
    assert r["alg_bytes_per_launch"] == int(per_launch)
    assert r["avg_launch_us"] == pytest.approx(2000.0)
    assert r["achieved"] == pytest.approx(per_launch / 2e-3 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["traffic_gbs"] == pytest.approx(3_000_000 / 2e-3 / 1e9, rel=1e-3)


def test_plain_roofline_counts_every_term():
    st = {"kt_count": [0, 10, 0, 0], "kt_ms": [0.0, 1.0, 0.0, 0.0], "iters_max": 9}
    r = bench.roofline(1, INFO, st, 0, True, None)
    terms = st["iters_max"] + 1
    total = terms * (INFO["m"] * bench.B_TERM_EDGE[0] + INFO["n"] * bench.B_TERM_ROW[0]) + INFO["n"] * bench.B_ONCE_ROW
    assert r["alg_bytes_per_launch"] == int(total / 10)
    assert "traffic_gbs" not in r and r["traffic"] is None


def test_source_hash_ignores_comments_only():
    csrc = os.path.join(bench.ROOT, "paper_1609_09068_amd", "csrc")

    def read_with(edit):
        def read(name):
            with open(os.path.join(csrc, name)) as f:
                text = f.read()
            return edit(text) if name == "solve_dev.h" else text
        return read

    h = bench.source_hash()
    assert bench.source_hash(read_with(lambda t: t + "\n// a comment\n/* and\n another */\n")) == h
    assert bench.source_hash(read_with(lambda t: t.replace("kThreads = 256", "kThreads  =  256", 1))) == h
    assert bench.source_hash(read_with(lambda t: t + "\nstatic int unused_symbol;\n")) != h


def test_stale_counter_summary_is_ignored(tmp_path):
    good = {"source_hash": bench.source_hash(), "kernels": {"k_gang/plain": {"hbm_bytes_per_launch": 123}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(good))
    assert bench.load_traffic(str(p), "k_gang/plain") == 123
    assert bench.load_traffic(str(p), "k_segment/componentwise") is None
    p.write_text(json.dumps(dict(good, source_hash="0" * 16)))
    assert bench.load_traffic(str(p), "k_gang/plain") is None
    assert bench.load_traffic(str(tmp_path / "missing.json"), "k_gang/plain") is None
