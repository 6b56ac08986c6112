"""Host logic of bench.py (no GPU): the roofline object, the counted-traffic lookup tied to
the kernel source it was taken with, and the single-GPU refusal."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _table():
    return {"spread": {"kernel": "k_spread_fused", "ms_per_step": 3.0, "avg_us": 30.0, "alg_bytes_per_launch": 14e6},
            "fft_y": {"kernel": "k_fft_lines<1>", "ms_per_step": 1.0, "avg_us": 11.0, "alg_bytes_per_launch": 25e6}}


def test_roofline_of_dominant_kernel():
    r = bench.roofline_of(_table(), None, 0.028)  # replayed launch of 28 us
    assert r["kernel"] == "k_spread_fused" and r["timer"] == "spread"
    assert r["achieved"] == pytest.approx(14e6 / 28e-6 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4) and r["peak"] == 8000.0
    assert r["traffic"] is None and r["duration_from"].startswith("back-to-back")
    e = bench.roofline_of(_table())  # no replay: the eager per-launch average
    assert e["avg_launch_us"] == 30.0 and e["duration_from"].startswith("eager")


def test_traffic_only_for_the_source_it_was_counted_with(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2607_25161_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = csrc / "k_mobility.hip"
    src.write_text("// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    (tmp_path / "profiles" / "c.md").write_text(
        f"source k_mobility.hip sha256 {sha}\ntraffic k_spread_fused 18012039\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("c.md", "k_spread_fused") == 18012039
    assert bench.measured_traffic("c.md", "k_interp") is None      # not counted
    assert bench.measured_traffic("missing.md", "k_spread_fused") is None
    src.write_text("// kernel source, changed\n")
    assert bench.measured_traffic("c.md", "k_spread_fused") is None  # counters are stale
    # a header the summary also lists must be unchanged too
    src.write_text("// kernel source\n")
    hdr = csrc / "fsd_impl.hpp"
    hdr.write_text("// header\n")
    hsha = hashlib.sha256(hdr.read_bytes()).hexdigest()
    (tmp_path / "profiles" / "c.md").write_text(
        f"source k_mobility.hip sha256 {sha}\nsource fsd_impl.hpp sha256 {hsha}\ntraffic k_spread_fused 18012039\n")
    assert bench.measured_traffic("c.md", "k_spread_fused") == 18012039
    hdr.write_text("// header, changed\n")
    assert bench.measured_traffic("c.md", "k_spread_fused") is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""
