"""Host-side checks of bench.py: the one-GPU contract and the traffic lookup
keyed to the kernel source (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_for_the_source_it_was_measured_on(tmp_path, monkeypatch):
    have = {w: bench.traffic_for(w) for w in ("octree-shell-256", "block-vortex-1024")}
    if any(v is None for v in have.values()):
        # the committed counters belong to another version of the kernels
        return
    assert all(v > 0 for v in have.values())
    assert bench.traffic_for("no-such-workload") is None
    other = tmp_path / "amriso.hip"
    other.write_bytes(open(bench.KERNEL_SOURCE, "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(other))
    assert bench.traffic_for("octree-shell-256") is None


def test_valu_issue_only_for_the_source_it_was_measured_on(tmp_path, monkeypatch):
    have = bench.valu_for("block-vortex-1024")
    if have is None:
        # the committed counters belong to another version of the kernels
        return
    assert "k_extract<false,0>" in have  # the count pass over all groups
    assert all(0.0 < v <= 1.0 for v in have.values())
    assert bench.valu_for("no-such-workload") is None
    other = tmp_path / "amriso.hip"
    other.write_bytes(open(bench.KERNEL_SOURCE, "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(other))
    assert bench.valu_for("block-vortex-1024") is None


def test_roofline_fields():
    r = bench.roofline_of(1000, 10, 0.5, None)
    assert r["algorithmic_bytes"] == 20.0 * 1000 + 36.0 * 10
    assert abs(r["achieved"] - r["algorithmic_bytes"] / 0.5e-3 / 1e9) < 1e-9
    assert r["frac"] == r["achieved"] / r["peak"] and r["unit"] == "GB/s" and r["bound"] == "hbm"


def test_cpu_baseline_reports_one_thread_and_brute_force():
    import amrgen

    r = bench.cpu_baseline(amrgen.two_level_sphere(), min_seconds=0.05)
    assert r["kind"] == "oracle" and r["unit"] == "cells/s" and r["value"] > 0 and r["cores"] >= 1
    assert r["one_thread"]["value"] > 0
    assert r["brute_force"]["cells"] == 960 and r["brute_force"]["value"] > 0
