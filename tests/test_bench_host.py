"""Host logic of bench.py (no GPU): the HBM traffic of the roofline is read from the committed
counter summary only for the level-0 tile variant the autotuner chose and only while the
kernel sources hash to the recorded value; the --gpus guard."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _summary():
    with open(os.path.join(ROOT, bench.COUNTER_SUMMARY)) as f:
        return f.read()


def test_traffic_read_per_profiled_variant():
    text = _summary()
    recorded = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text).group(1)
    if recorded != bench.kernel_source_hash():
        pytest.skip("kernel sources changed since the counters were taken (traffic is null then)")
    for cfg in bench.PROBE_CONFIGS:
        v = cfg["variant"][0]
        m = re.search(rf"level0_traffic_bytes_per_launch\[variant {v}\]:\s*([0-9.]+)", text)
        assert m, f"variant {v} missing from the summary"
        t = bench.measured_traffic(v)
        assert t == float(m.group(1))
        # no wasted bytes: within 5 % of 1024^2 x (2 x 1 + 16) B
        assert abs(t / (1024 * 1024 * 18) - 1) < 0.05
    assert bench.measured_traffic(7) is None   # a variant the probe does not profile


def test_traffic_null_when_sources_change(tmp_path, monkeypatch):
    text = _summary()
    stale = re.sub(r"kernel_source_sha256:\s*[0-9a-f]{64}", "kernel_source_sha256: " + "0" * 64, text)
    p = tmp_path / "counters.md"
    p.write_text(stale)
    monkeypatch.setattr(bench, "COUNTER_SUMMARY", str(p))   # absolute: os.path.join keeps it
    assert bench.measured_traffic(bench.PROBE_CONFIGS[0]["variant"][0]) is None


def test_kernel_hash_ignores_comments(tmp_path, monkeypatch):
    src = tmp_path / "k.h"
    src.write_text("int a = 1;  // one\n\nint b = 2;\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.h"])
    h1 = bench.kernel_source_hash()
    src.write_text("int a = 1;  // another comment\nint b = 2;\n")
    assert bench.kernel_source_hash() == h1
    src.write_text("int a = 1;\nint b = 3;\n")
    assert bench.kernel_source_hash() != h1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
