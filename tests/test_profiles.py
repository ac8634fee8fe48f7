"""The committed rocprofv3 summaries match the code they describe.

The benchmark reports HBM traffic of the connected-configuration forward from
the committed counter summary only while that summary was taken on the
current forward source; these checks fail as soon as the kernel source moves
on without new counters, instead of letting the benchmark print a null.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    import sys
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_forward_traffic_summary_is_current(bench):
    path = os.path.join(ROOT, "profiles", "fused_forward_c4_bf16w_traffic.md")
    text = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*`?([0-9a-f]{64})", text)
    assert m and m.group(1) == bench.kernel_source_hash(), "counter summary taken on another forward source"
    rows = int(re.search(r"rows_per_block:\s*`?(\d+)", text).group(1))
    for waves in (8, 16):
        t = bench.measured_traffic("c4", "bf16w", waves, rows)
        # at least the algorithmic 24 B per row (8 B configuration in, 16 B result out)
        assert t is not None and 24.0 <= t < 48.0


def test_summaries_name_their_commands():
    prof = os.path.join(ROOT, "profiles")
    names = sorted(f for f in os.listdir(prof) if f.endswith((".md", ".txt")))
    assert names
    for f in names:
        text = open(os.path.join(prof, f)).read()
        assert "rocprofv3" in text and "bench.py" in text, f
        assert len(text) < 64 * 1024, f
