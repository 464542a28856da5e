"""Host-side logic of bench.py, on the CPU: the roofline arithmetic, the
per-order byte counts, the profile lookup keyed by the source hash, the
workload recipes and the single-GPU rule.  No GPU is touched."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bytes_per_edge_sweep_follows_the_order():
    # 8 bytes of edge ids plus 2h label reads of 4 bytes (Definition 3)
    assert bench.bytes_per_edge_sweep(1) == 16
    assert bench.bytes_per_edge_sweep(2) == 24
    assert bench.bytes_per_edge_sweep(3) == 32
    assert bench.bytes_per_edge_sweep(bench.order_value("full")) is None


def test_roofline_arithmetic():
    # 4 sweeps of 1,000,000 edges at order 2 in 2 ms: 96 MB / 2 ms = 48 GB/s
    r = {"stats": [(0, 4, 3, 0)] * 3, "kernel_ms": [2.0, 2.0, 2.0]}
    roof = bench.roofline(2, 1_000_000, r, None, n=500_000)
    assert roof["achieved"] == pytest.approx(48.0)
    assert roof["frac"] == pytest.approx(48.0 / bench.HBM_PEAK_GBPS, abs=1e-4)
    assert roof["edge_sweeps_per_launch"] == 4_000_000
    # compulsory: (8 m + 8 n) bytes per sweep
    assert roof["compulsory_GBps"] == pytest.approx(4 * (8e6 + 4e6) / 2e-3 / 1e9)
    assert roof["traffic"] is None
    roof = bench.roofline(2, 1_000_000, r, {"traffic": 50_000_000, "l2_hit_rate": 0.5})
    assert roof["traffic"] == 50_000_000
    assert roof["dram_GBps"] == pytest.approx(25.0)
    assert roof["l2_hit_rate"] == 0.5


def test_profile_figures_need_the_current_sources(tmp_path, monkeypatch):
    text = ("csrc_sha256: %s\n\ntraffic_bytes_per_launch: 1234\n\nl2_hit_rate: 0.75\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    h = bench.source_hash()
    (prof / "k_persistent_w.md").write_text(text % h)
    (prof / "k_persistent_stale.md").write_text(text % "0000000000000000")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: h)
    assert bench.profile_figures("w") == {"traffic": 1234, "l2_hit_rate": 0.75}
    assert bench.profile_figures("stale") is None
    assert bench.profile_figures("missing") is None


def test_source_hash_is_stable():
    assert bench.source_hash() == bench.source_hash()
    assert len(bench.source_hash()) == 16


def test_small_workload_recipe():
    src, dst, n = bench.make_workload("er65536_m524288", 1)
    assert n == 65536 and src.size == dst.size == 524288
    assert src.dtype == np.int32 and dst.dtype == np.int32
    assert int(src.min()) >= 0 and int(max(src.max(), dst.max())) < n


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""


def test_percentiles():
    assert bench.pct([1.0, 2.0, 3.0, 4.0], 50) == pytest.approx(2.5)
    assert bench.pct([], 50) is None
    json.dumps({"p": bench.pct([5.0], 99)})


def test_committed_profiles_match_the_sources():
    # the committed rocprofv3 summaries of the two headline workloads were
    # taken on the sources in the tree, so the bench line carries their
    # traffic and L2 hit rate
    for w in ("rmat24_ef16", "grid4096_holes10"):
        fig = bench.profile_figures(w)
        assert fig is not None, w
        assert fig["traffic"] > 0 and 0.0 < fig["l2_hit_rate"] < 1.0
