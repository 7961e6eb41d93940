"""Host-side checks of bench.py: the one-GPU contract, the counter lookup
keyed to the kernel source, the roofline fields (no GPU needed)."""
import glob
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


def test_counters_only_for_the_source_they_were_measured_on(tmp_path, monkeypatch):
    import hashlib

    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "amriso.hip"
    src.write_bytes(b"// kernels\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    (prof / "wl_counters.txt").write_text("# header\nsource_sha256 %s\n"
                                          "kernel k_extract<false, 0> | traffic_bytes 1.5e9 l2_hit 0.8 mall_hit - "
                                          "valu_issue 0.7\n" % sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    c = bench.counters_for("wl", "k_extract<false, 0>")
    assert c == {"traffic_bytes": 1.5e9, "l2_hit": 0.8, "mall_hit": None, "valu_issue": 0.7}
    assert bench.counters_for("wl", "k_index_insert") is None
    assert bench.counters_for("other", "k_extract<false, 0>") is None
    src.write_bytes(b"// kernels, changed\n")
    assert bench.counters_for("wl", "k_extract<false, 0>") is None


def test_committed_counter_summaries_parse():
    """Every committed counter summary names the source it was taken with
    and parses (its figures are used only while that source is current)."""
    import glob

    for path in glob.glob(os.path.join(ROOT, "profiles", "*_counters.txt")):
        lines = open(path).read().splitlines()
        assert any(ln.startswith("source_sha256 ") for ln in lines), path
        for ln in lines:
            if ln.startswith("kernel "):
                name, rest = ln[len("kernel "):].split(" | ", 1)
                f = rest.split()
                assert len(f) % 2 == 0 and name.strip(), ln


def test_roofline_fields():
    r = bench.roofline_of("k_extract<false, 0>", 20.0 * 1000, 0.5, None, 7)
    assert r["algorithmic_bytes"] == 20.0 * 1000
    assert abs(r["achieved"] - r["algorithmic_bytes"] / 0.5e-3 / 1e9) < 1e-9
    assert r["frac"] == r["achieved"] / r["peak"] and r["unit"] == "GB/s" and r["bound"] == "hbm"
    assert r["traffic"] is None and r["launches"] == 7 and r["kernel"] == "k_extract<false, 0>"


def test_algorithmic_bytes_per_kernel():
    class K:
        KERNEL_UPLOAD, KERNEL_RESET, KERNEL_INSERT, KERNEL_COMPACT, KERNEL_MARK, KERNEL_EXTRACT, KERNEL_WRITE = \
            range(1, 8)

    assert bench.alg_bytes(K, K.KERNEL_UPLOAD, 100, 7, False) == 2000
    assert bench.alg_bytes(K, K.KERNEL_EXTRACT, 100, 7, False) == 2000  # count pass: no triangles written
    assert bench.alg_bytes(K, K.KERNEL_EXTRACT, 100, 7, True) == 2000 + 252  # fused pass writes them
    assert bench.alg_bytes(K, K.KERNEL_WRITE, 100, 7, False) == 252
    assert bench.alg_bytes(K, K.KERNEL_MARK, 100, 7, False) is None


def test_cpu_baseline_reports_one_thread_and_brute_force():
    import amrgen

    r = bench.cpu_baseline(amrgen.two_level_sphere(), min_seconds=0.05)
    assert r["kind"] == "oracle" and r["unit"] == "cells/s" and r["value"] > 0 and r["cores"] >= 1
    assert r["one_thread"]["value"] > 0
    assert r["brute_force"]["cells"] == 960 and r["brute_force"]["value"] > 0


def _csv(path, header, rows):
    import csv

    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_counter_summary_from_rocprof_csv(tmp_path):
    """bench_counters.py: per-kernel means per dispatch, the copy probe's
    scale (FETCH_SIZE reads half of what the copy moves, WRITE_SIZE all of
    it), L2 hit rate and VALU issue fraction; the summary parses back
    through bench.counters_for while the source is unchanged."""
    import bench_counters

    mul = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<float, float, float, " \
          "at::native::binary_internal::MulFunctor<float> > >(int, F)"
    kern = "(anonymous namespace)::k_extract<false, 0>((anonymous namespace)::ExtractArgs)"
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    _csv(tmp_path / "f" / "x" / "run_counter_collection.csv", hdr,
         [[1, kern, "FETCH_SIZE", 100.0], [2, kern, "FETCH_SIZE", 300.0], [3, mul, "FETCH_SIZE", 131072.0]])
    _csv(tmp_path / "w" / "run_counter_collection.csv", hdr,
         [[1, kern, "WRITE_SIZE", 10.0], [2, kern, "WRITE_SIZE", 30.0], [3, mul, "WRITE_SIZE", 262144.0]])
    _csv(tmp_path / "t" / "run_counter_collection.csv", hdr,
         [[1, kern, "TCC_HIT_sum", 80.0], [1, kern, "TCC_MISS_sum", 20.0]])
    _csv(tmp_path / "s" / "run_counter_collection.csv", hdr,
         [[1, kern, "SQ_INSTS_VALU", 614.4e3], [1, kern, "SQ_WAVES", 64.0]])
    _csv(tmp_path / "d" / "run_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs"],
         [[kern, 2, 4000, 2000.0], [mul, 1, 500, 500.0]])
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench_counters.py"), "--workload", "wl",
                          "--trace", str(tmp_path / "d"), "--fetch", str(tmp_path / "f"), "--write",
                          str(tmp_path / "w"), "--tcc", str(tmp_path / "t"), "--sq", str(tmp_path / "s"),
                          "--command", "rocprofv3 ..."], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.splitlines()
    line = [ln for ln in lines if ln.startswith("kernel ")]
    assert len(line) == 1 and line[0].startswith("kernel k_extract<false, 0> | ")
    f = line[0].split(" | ", 1)[1].split()
    c = {k: v for k, v in zip(f[0::2], f[1::2])}
    # fetch (100 + 300) / 2 KiB x 2, write (10 + 30) / 2 KiB x 1
    assert float(c["fetch_bytes"]) == 400.0 * 1024 and float(c["write_bytes"]) == 20.0 * 1024
    assert float(c["traffic_bytes"]) == 420.0 * 1024
    assert c["l2_hit"] == "0.8000" and c["mall_hit"] == "-"
    # 614.4e3 wave instructions in 2 us = 3.072e11/s, half the issue peak
    assert c["valu_issue"] == "0.5000" and c["avg_us"] == "2.00"
    assert bench_counters.short_name(kern) == "k_extract<false, 0>"
    sha = [ln.split()[1] for ln in lines if ln.startswith("source_sha256")]
    assert sha and len(sha[0]) == 64


def test_kernel_stats_summary_from_rocprof_csv(tmp_path):
    """bench_counters.py --kernel-stats: the library's kernels only (names
    starting k_, arguments dropped), durations in us, longest total first,
    with the command and the notes in the header."""
    mul = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<float, float, float, " \
          "at::native::binary_internal::MulFunctor<float> > >(int, F)"
    k0 = "(anonymous namespace)::k_index_insert(int const*, int const*, float const*, long)"
    k1 = "void (anonymous namespace)::k_extract<false, 0>((anonymous namespace)::ExtractArgs)"
    _csv(tmp_path / "d" / "x" / "run_kernel_stats.csv",
         ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
         [[k0, 2, 3000, 1500.0, 10, 1000, 2000, 1], [mul, 9, 90000, 10000.0, 80, 10000, 10000, 0],
          [k1, 4, 8000, 2000.0, 10, 1500, 2500, 1]])
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench_counters.py"), "--kernel-stats", "--workload",
                          "wl", "--trace", str(tmp_path / "d"), "--command", "rocprofv3 ...", "--note", "first",
                          "--note", "second"], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.splitlines()
    assert lines[0].endswith(": wl") and "#   rocprofv3 ..." in lines and "# first" in lines and "# second" in lines
    rows = [ln.split() for ln in lines if ln.startswith("k_")]
    assert [r[0] for r in rows] == ["k_extract<false,", "k_index_insert"]
    assert rows[0][2:] == ["4", "8.0", "2.00", "1.50", "2.50"]
    assert rows[1][1:] == ["2", "3.0", "1.50", "1.00", "2.00"]
    # counter summaries still need all four counter runs
    bad = subprocess.run([sys.executable, os.path.join(ROOT, "bench_counters.py"), "--workload", "wl", "--trace",
                          str(tmp_path / "d"), "--command", "c"], capture_output=True, text=True, timeout=60)
    assert bad.returncode != 0 and "--fetch" in bad.stderr


def test_committed_kernel_stats_summaries_name_their_commands():
    """Every kernel time summary under profiles/ gives the rocprofv3 command
    it came from (committed bench.py) and the summary step."""
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_kernel_stats.txt")))
    assert paths
    for p in paths:
        text = open(p).read()
        assert "rocprofv3 --kernel-trace --stats" in text and "$R/bench.py" in text, p
        assert "bench_counters.py --kernel-stats" in text, p
        assert any(ln.startswith("k_") for ln in text.splitlines()), p
