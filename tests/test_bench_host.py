"""Host-side pieces of bench.py (no GPU): the algorithmic work it divides by,
the gate that keeps a stale counter summary out of the roofline, and the
one-GPU contract of its command line."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_flops_of_the_single512_frame():
    # blur: 2 C H W K (P^2 + 1); network: 2 sum(in out) per pixel
    assert bench.blur_flops(1, 512, 512, 100, 33) == 2.0 * 512 * 512 * 100 * (33 * 33 + 1)
    assert bench.blur_flops(1, 512, 512, 100, 33) == pytest.approx(57.147392e9)
    assert bench.mlp_flops(512, 512, (33, 100, 100, 100)) == 2.0 * 512 * 512 * (3300 + 10000 + 10000)
    assert bench.mlp_flops(512, 512, (33, 100, 100, 100)) == pytest.approx(12.2159104e9)
    assert bench.blur_flops(3, 7, 5, 16, 9) == 2.0 * 3 * 7 * 5 * 16 * 82


def test_traffic_is_reported_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source v1\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = {"hbm_bytes_per_launch": 4.2e7, "src_digest": bench.src_digest("k.hip")}
    (tmp_path / "profiles" / "blur_mlp_bf16_single512_traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_from_profiles(["k.hip"]) == 4.2e7
    src.write_text("kernel source v2\n")          # the kernel changed since the counters were taken
    assert bench.traffic_from_profiles(["k.hip"]) is None
    (tmp_path / "profiles" / "blur_mlp_bf16_single512_traffic.json").unlink()
    assert bench.traffic_from_profiles(["k.hip"]) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
