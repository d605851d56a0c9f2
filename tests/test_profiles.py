"""The committed measurement summaries (host only): each names the command that produced it, and
the counter summary of the counting kernel was taken on the current sources of that kernel
and of the preprocessing that lays out its work, so that bench.py's roofline uses it."""
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def test_every_summary_names_its_command():
    names = sorted(os.listdir(PROFILES))
    assert names
    for name in names:
        assert name.endswith((".md", ".txt")), name
        text = open(os.path.join(PROFILES, name)).read()
        assert "rocprofv3" in text or "bench.py" in text, name
        assert len(text) < 64 * 1024, name  # short summaries, no raw traces
        assert not re.search(r"\bround\b", text, re.I), name


def test_counting_kernel_counters_match_sources():
    kv = bench.load_counters("k_count", "rmat23")
    assert kv is not None, "counter summary missing or taken on other sources"
    assert kv["sources_sha"] == bench.sources_sha()
    hbm = float(kv["hbm_bytes_per_launch"])
    ms = float(kv["kernel_ms_trace"])
    assert 0 < hbm and 0 < ms
    # the summary's own figures: scaled FETCH and WRITE sum to the bytes per launch (the
    # scales are printed to four decimals)
    f = float(kv["fetch_kib"]) * 1024 * float(kv["fetch_scale"])
    w = float(kv["write_kib"]) * 1024 * float(kv["write_scale"])
    assert abs(f + w - hbm) <= 1e-4 * hbm
    assert hbm / (ms * 1e-3) <= 8.0e12  # at most the HBM peak
