"""Benchmark: AMR cells/s to crack-free triangles on one MI355X.

One step = the whole hot path over one synthetic AMR set already in HBM:
validate + reduce (amr_upload), build the cell-location index
(amr_build_index, enqueued without waiting: its verdict stays on the device
and is read once after the timed steps) and extract the iso-surface
(amr_isosurface, one pass into a buffer sized beforehand).  The headline is
the step rate of the ~2M-cell octree (octree-shell-256-2m).  Every kernel of
the step is timed on its own with HIP events around the kernel (recorded on
the stream it runs on); the dominant one is timed in every timed step and
gives the roofline (HBM, against the 8 TB/s peak and against a plain 1 GiB
device copy measured in the same run; counter figures from the committed
summary under profiles/ while the kernel source is unchanged).

Beside the headline, the JSON line holds: iso latency and repeated isos on
the built set; the dual mesh as an interpolant (point queries on the
headline set); the same step on the 137k-cell octree of the literal recipe
and on the 50.8M-cell block-structured set with holes; the host-to-host
pipeline (PCIe-inclusive); 64 isos of the headline set in one batched
run and 32 uneven sets (10k..5M cells) in one batched run, each against
the plain path; on the 608.9M-cell resident octree, 64 isos in one batched
run against the plain path and serving a Poisson request mix against the
serial plain path; the index comparison (hash against sorted cells); and
the CPU oracle's rate on the headline set, on a sample of the 50.8M-cell
set and on the 32 sets.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AMR cells/sec to crack-free triangles (1 GPU, % HBM roofline); p50/p99 iso latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_2004_08475_amd", "csrc", "amriso.hip")


def make_workload(name):
    import amrgen

    if name == "octree-shell-256-2m":
        return amrgen.octree_shell_2m()
    if name == "octree-shell-256":
        return amrgen.octree_shell()
    if name == "two-level-sphere-16":
        return amrgen.two_level_sphere()
    if name == "block-vortex-1024":
        return amrgen.block_vortex(device="cuda")
    raise SystemExit("unknown workload %s" % name)


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def host_threads():
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


def oracle_rate(cs, threads, sample=None, seed=0):
    """The oracle as it stands on `threads` host threads: its sorted index over
    the whole set (timed), then rules 1-3 + Marching Cubes over all cells or
    over `sample` consecutive cells of the shuffled list (timed); the rate
    charges the index in full and the extraction scaled to the whole set.
    Returns (cells/s, seconds spent, cells extracted)."""
    import oracle

    t0 = time.perf_counter()
    o = oracle.Oracle(cs.xyz, cs.level, cs.value, validate=False)
    t_index = time.perf_counter() - t0
    c0, c1 = 0, cs.n
    if sample and sample < cs.n:
        c0 = (seed * 7919) % (cs.n - sample)
        c1 = c0 + sample
    t0 = time.perf_counter()
    o.isosurface_threaded(cs.iso, threads, c0, c1)
    t_ext = time.perf_counter() - t0
    del o
    t_whole = t_index + t_ext * cs.n / (c1 - c0)
    return cs.n / t_whole, t_index + t_ext, c1 - c0


def cpu_baseline(cs, min_seconds=10.0, large=None, sets=None):
    """The oracle (never tuned) on the host's cores: the headline set whole,
    repeated until about min_seconds have passed; one thread on a sample of
    it; the brute-force locator on the 960-cell two-level sphere; and, when
    given, a sample of the large set and the batch of uneven sets."""
    import amrgen
    import oracle

    threads = host_threads()
    reps, t_total = 0, 0.0
    while t_total < min_seconds and reps < 10000:
        _, dt, _ = oracle_rate(cs, threads)
        t_total += dt
        reps += 1
    one_rate, one_s, one_n = oracle_rate(cs, 1, sample=min(cs.n, 100_000))
    c1 = amrgen.two_level_sphere()
    t0 = time.perf_counter()
    ob = oracle.Oracle(c1.xyz, c1.level, c1.value, locator="brute", validate=False)
    ob.count_range(c1.iso, 0, c1.n)
    t_brute = time.perf_counter() - t0
    out = {"value": cs.n * reps / t_total, "unit": "cells/s", "cores": threads, "kind": "oracle",
           "sample": "whole %s set (%d cells): sorted-corner index + rules 1-3 + Marching Cubes on %d threads, "
                     "%d repetitions, %.1f s" % (cs.name, cs.n, threads, reps, t_total),
           "one_thread": {"value": one_rate, "seconds": one_s,
                          "sample": "index over all cells, extraction over %d cells, scaled" % one_n},
           "brute_force": {"workload": c1.name, "cells": c1.n, "value": c1.n / t_brute, "seconds": t_brute}}
    if large is not None:
        rate, dt, k = oracle_rate(large, threads, sample=2_000_000)
        out["large_workload"] = {"workload": large.name, "cells": large.n, "value": rate, "unit": "cells/s",
                                 "seconds": dt, "sample": "index over all %d cells (timed), extraction over %d "
                                 "consecutive cells of the shuffled list, scaled to the set" % (large.n, k)}
    if sets:
        t_sum, n_sum, ext = 0.0, 0, 0
        for k, c in enumerate(sets):
            _, dt, m = oracle_rate(c, threads, sample=300_000, seed=k)
            t_sum += dt * c.n / max(m, 1) if m < c.n else dt
            n_sum += c.n
            ext += m
        out["batched_sets"] = {"sets": len(sets), "cells": n_sum, "value": n_sum / t_sum, "unit": "cells/s",
                               "sample": "each set's index whole, extraction over at most 300,000 cells per set "
                                         "(%d cells in all), scaled per set" % ext}
    return out


def counters_for(workload, kernel):
    """rocprofv3 counter figures of one kernel on one workload from the
    committed summary profiles/<workload>_counters.txt: HBM traffic per
    launch (FETCH_SIZE + WRITE_SIZE scaled by a plain copy), L2 and MALL hit
    rates, the VALU issue fraction.  None when there is no summary, no line
    for the kernel, or the kernel source changed since the counters were
    taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "%s_counters.txt" % workload)
    try:
        lines = open(path).read().splitlines()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    recorded = [ln.split()[1] for ln in lines if ln.startswith("source_sha256")]
    if not recorded or recorded[0] != src:
        return None
    for ln in lines:
        if ln.startswith("kernel "):
            name, rest = ln[len("kernel "):].split(" | ", 1)
            if name.strip() == kernel:
                f = rest.split()
                return {k: (None if v == "-" else float(v)) for k, v in zip(f[0::2], f[1::2])}
    return None


def kernel_names(amr):
    return {amr.KERNEL_UPLOAD: "k_upload", amr.KERNEL_RESET: "k_build_reset", amr.KERNEL_INSERT: "k_index_insert",
            amr.KERNEL_COMPACT: "k_index_compact", amr.KERNEL_MARK: "k_index_mark",
            amr.KERNEL_EXTRACT: "extract", amr.KERNEL_WRITE: "write"}


def kernel_survey(amr, s, step, reps=3):
    """Each kernel of a step on its own: HIP events around the kernel itself
    (recorded on the stream it runs on), `reps` steps per kernel.  Returns
    ({kernel id: mean ms}, {kernel id: the launched kernel's name, as
    rocprofv3 shows it}); a kernel the step does not run (the write pass of
    a fused call: the library then names no kernel) is left out."""
    import torch

    out, names = {}, {}
    stream = torch.cuda.current_stream()
    for k in kernel_names(amr):
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            e1.record(stream)
            s.time_kernel(k, e0, e1)
            step()
            torch.cuda.synchronize()
            s.time_kernel(0, e0, e1)  # disarm, in case the step did not run it
            ms.append(e0.elapsed_time(e1))
            names[k] = s.timed_kernel_name()
        if names[k]:  # "" when the step launched no kernel in this slot
            out[k] = statistics.mean(ms)
    return out, names


def time_steps(amr, s, step, iso_call, steps, warmup, kernel):
    """`steps` whole-path steps between two synchronisations (host clock),
    with HIP events around `kernel` in every one of them (its own duration,
    recorded on the stream it runs on).  A second run of the same steps puts
    events between the stages for the per-stage split.  Returns (ms per step,
    kernel ms per step, (upload, build, iso) ms lists)."""
    import torch

    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        step()
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in pairs:
        a.record(stream)
        b.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        s.time_kernel(kernel, *pairs[k])
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    s.build_status()  # the verdict of the last build on the device: raises if it failed
    kms = [a.elapsed_time(b) for a, b in pairs]
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for e in evs:
        e[0].record(stream)
        s.upload(*s._cells)
        e[1].record(stream)
        s.build_index(wait=False)
        e[2].record(stream)
        iso_call()
        e[3].record(stream)
    torch.cuda.synchronize()
    s.build_status()
    st = ([e[0].elapsed_time(e[1]) for e in evs], [e[1].elapsed_time(e[2]) for e in evs],
          [e[2].elapsed_time(e[3]) for e in evs])
    return ms, kms, st


def alg_bytes(amr, kernel, n_cells, n_tri, fused):
    """Algorithmic bytes of one launch: 20 B per input cell read once (its
    int3 corner, level and value) and 36 B per triangle written (the per-unit
    figures of the path); the index insertion also stores each cell's value
    in its group record (4 B per cell)."""
    if kernel == amr.KERNEL_UPLOAD:
        return 20.0 * n_cells
    if kernel == amr.KERNEL_INSERT:
        return 24.0 * n_cells
    if kernel == amr.KERNEL_EXTRACT:
        return 20.0 * n_cells + (36.0 * n_tri if fused else 0.0)
    if kernel == amr.KERNEL_WRITE:
        return 36.0 * n_tri
    return None


def copy_peak_gbs(mib=1024, reps=10):
    """Measured HBM bandwidth of a plain device-to-device copy of `mib` MiB
    (Tensor.copy_, the runtime's copy kernel): bytes read + written / time,
    HIP events around `reps` copies.  (The counter-scale probe of
    --copy-probe-mib is a different kernel, so the two never mix.)"""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def roofline_of(name, alg, kernel_ms, counters, launches):
    achieved = alg / (kernel_ms * 1e-3) / 1e9
    c = counters or {}
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": c.get("traffic_bytes"), "algorithmic_bytes": alg,
            "avg_launch_ms": kernel_ms, "launches": launches,
            "l2_hit_rate": c.get("l2_hit"), "mall_hit_rate": c.get("mall_hit"),
            "valu_issue_frac": c.get("valu_issue")}


def step_measurement(amr, cs, xyz, lvl, val, steps, warmup):
    """The whole-path step on one resident set: throughput, every kernel's
    own duration, and the roofline of the dominant kernel (timed in every
    timed step)."""
    import torch

    dev = xyz.device
    s = amr.AmrSet(dev.index)
    s.upload(xyz, lvl, val)
    s.build_index()
    n_tri, n_dual = s.count(cs.iso)
    cap = n_tri
    tris = torch.empty((max(cap, 1), 9), dtype=torch.float32, device=dev)

    def iso_call():
        s.isosurface_into(cs.iso, tris, cap)

    def step():
        s.upload(xyz, lvl, val)
        s.build_index(wait=False)
        iso_call()

    for _ in range(warmup):
        step()
    survey, names = kernel_survey(amr, s, step)
    fused = amr.KERNEL_WRITE not in survey
    # the roofline kernel: the longest one whose algorithmic bytes are defined
    # (every kernel of the path but the ancestor marking, which only probes)
    dom = max((k for k in survey if alg_bytes(amr, k, cs.n, n_tri, fused)), key=survey.get)
    ms, kms, (up, bd, iso) = time_steps(amr, s, step, iso_call, steps, warmup, dom)
    assert int(s.counts[0].item()) == n_tri
    kernel_ms = statistics.mean(kms)
    alg = alg_bytes(amr, dom, cs.n, n_tri, fused)
    return {"set": s, "n_tri": n_tri, "n_dual": n_dual, "ms_per_step": ms, "cells_per_s": cs.n / (ms * 1e-3),
            "stages_ms": {"upload": statistics.mean(up), "build_index": statistics.mean(bd),
                          "isosurface": statistics.mean(iso)},
            "kernels_ms": {names[k]: v for k, v in sorted(survey.items(), key=lambda kv: -kv[1])},
            "roofline": roofline_of(names[dom], alg, kernel_ms, counters_for(cs.name, names[dom]), steps)}


def large_measurement(amr, cs, steps, resident=True, index_ab=True):
    """The same whole-path step on the 50.8M-cell block-structured set, where
    throughput rather than launch latency decides."""
    import torch

    dev = torch.device("cuda", 0)
    xyz, lvl, val = (torch.from_numpy(a).to(dev) for a in (cs.xyz, cs.level, cs.value))
    r = step_measurement(amr, cs, xyz, lvl, val, steps, 2)
    s = r.pop("set")
    out = {"workload": cs.name, "cells": cs.n, "triangles": r["n_tri"], "duals": r["n_dual"], "steps": steps,
           "ms_per_step": r["ms_per_step"], "cells_per_s": r["cells_per_s"], "stages_ms": r["stages_ms"],
           "kernels_ms": r["kernels_ms"], "roofline": r["roofline"],
           "resident_iso": resident_iso_measurement(s, cs) if resident else None}
    if index_ab:
        out["index_ab"] = index_measurement(amr, s, cs)
    s.close()
    del s, xyz, lvl, val
    torch.cuda.empty_cache()
    return out


def resident_iso_measurement(s, cs, reps=3):
    """Single-pass iso-surfaces at 19 quantiles of the values on the built
    set (its group value ranges already recorded, so the passes skip groups
    that cannot hold triangles), HIP events around each call on the stream
    the kernels run on."""
    import numpy as np
    import torch

    stream = torch.cuda.current_stream()
    isos = np.quantile(cs.value, np.linspace(0.05, 0.95, 19)).astype(np.float32)
    counts = [s.count(float(v))[0] for v in isos]
    tris = torch.empty((max(max(counts), 1), 9), dtype=torch.float32, device=s.device)
    evs = []
    for _ in range(reps):
        for v, c in zip(isos, counts):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s.isosurface_into(float(v), tris, c)
            e1.record(stream)
            evs.append((e0, e1))
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in evs]
    mean = statistics.mean(ms)
    return {"isos": len(isos), "reps": reps, "ms_mean": mean, "ms_min": min(ms), "ms_max": max(ms),
            "triangles_mean": statistics.mean(counts), "cells_per_s": cs.n / (mean * 1e-3),
            "what": "amr_isosurface single pass (count, scan, write) at quantiles 0.05..0.95 of the values, "
                    "group value ranges recorded by an earlier call"}


def sampler_measurement(amr, s, cs, n_points=1 << 22, reps=5):
    """The dual mesh as an interpolant on the resident set: the cell-to-dual
    map built once from the set's dual list, then n_points seeded uniform
    points over the set's bounding box per query launch; the query kernel
    timed with HIP events around it on its stream."""
    import numpy as np
    import torch

    dev = s.device
    stream = torch.cuda.current_stream()
    pl, ids = s.dual_cells()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp = amr.DualSampler(s, pl, ids)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    w = (1 << cs.level.astype(np.int64))[:, None]
    lo, hi = cs.xyz.min(0), (cs.xyz + w).max(0)
    pts = torch.from_numpy(np.random.default_rng(7).uniform(lo, hi, (n_points, 3)).astype(np.float32)).to(dev)
    vals = torch.empty(n_points, dtype=torch.float32, device=dev)
    dual = torch.empty(n_points, dtype=torch.int64, device=dev)
    smp.sample_into(pts, vals, dual)
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        e1.record(stream)
        s.time_kernel(amr.KERNEL_SAMPLE, e0, e1)
        smp.sample_into(pts, vals, dual)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    inside = int((~torch.isnan(vals)).sum().item())
    kernel_ms = statistics.mean(ms)
    return {"what": "dual-mesh interpolant: %d uniform points over the set's bounding box per launch, "
                    "k_smp_query timed with HIP events" % n_points,
            "duals": int(pl.shape[0]), "map_build_ms": build_ms, "query_ms": kernel_ms,
            "points_per_s": n_points / (kernel_ms * 1e-3), "inside": inside}


def index_measurement(amr, s, cs, reps=3):
    """The extraction's index (hash of sibling groups) against the paper's
    sorted cells with a binary search per level, on the same built set:
    build time of each (HIP events on the stream), and the snap queries of
    every cell (27 points per cell) through each, the kernel timed with HIP
    events around it; both must find the same cells."""
    import torch

    stream = torch.cuda.current_stream()
    out = torch.zeros(2, dtype=torch.int64, device=s.device)

    def timed(fn):
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return statistics.mean(ms)

    s.build_sorted_index()
    sorted_build = timed(s.build_sorted_index)
    s.upload(*s._cells)
    s.build_index()
    hash_build = timed(lambda: (s.upload(*s._cells), s.build_index(wait=False)))
    s.build_status()
    s.build_sorted_index()
    res, snap_ms = {}, {}
    for name, kind in (("hash", amr.INDEX_HASH), ("sorted", amr.INDEX_SORTED)):
        s.snap_count_into(out, kind)
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            e1.record(stream)
            s.time_kernel(amr.KERNEL_SNAP, e0, e1)
            s.snap_count_into(out, kind)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        snap_ms[name] = statistics.mean(ms)
        res[name] = out.cpu().tolist()
    assert res["hash"] == res["sorted"]
    return {"what": "point-location index: build (HIP events around the calls on the stream; the hash build "
                    "includes the upload validation) and 27 snap queries per cell located through each (the "
                    "snap kernel timed with HIP events)",
            "build_ms": {"hash": hash_build, "sorted": sorted_build},
            "snap_ms": snap_ms, "snaps": 27 * cs.n, "snaps_found": res["hash"][0],
            "snaps_per_s": {k: 27 * cs.n / (v * 1e-3) for k, v in snap_ms.items()},
            "chosen": min(snap_ms, key=snap_ms.get)}


def pipeline_measurement(amr, cs, reps=5):
    """The whole pipeline from host memory and back (the paper's Y column,
    its sec. 5.2 figure): pinned host cells -> device, validate, index, count
    and write the triangles, weld them into an indexed mesh, copy vertices
    and indices back.  PCIe-inclusive, so it is reported beside `value`."""
    import torch

    dev = torch.device("cuda", 0)
    hx = torch.from_numpy(cs.xyz).pin_memory()
    hl = torch.from_numpy(cs.level).pin_memory()
    hv = torch.from_numpy(cs.value).pin_memory()
    s = amr.AmrSet(0)
    times, parts = [], []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, l, v = hx.to(dev, non_blocking=True), hl.to(dev, non_blocking=True), hv.to(dev, non_blocking=True)
        s.upload(x, l, v)
        t1 = time.perf_counter()
        s.build_index()
        t2 = time.perf_counter()
        out = s.isosurface(cs.iso, cells=True)
        t3 = time.perf_counter()
        verts, idx = amr.indexed_mesh(out["tris"], out["cells"])
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        hv_out, hi_out = verts.cpu(), idx.cpu()
        t5 = time.perf_counter()
        if r:
            times.append(t5 - t0)
            parts.append((t1 - t0, t2 - t1, t3 - t2, t4 - t3, t5 - t4))
    k = sorted(range(reps), key=lambda i: times[i])[reps // 2]
    p = parts[k]
    return {"what": "host cells -> device -> amr_upload -> amr_build_index -> amr_isosurface (count + write) -> "
                    "amr_indexed_mesh -> vertices and indices to host; median of %d, host clock" % reps,
            "ms": times[k] * 1e3, "cells_per_s": cs.n / times[k],
            "stages_ms": {"h2d+upload": p[0] * 1e3, "build_index": p[1] * 1e3, "isosurface": p[2] * 1e3,
                          "indexed_mesh": p[3] * 1e3, "d2h": p[4] * 1e3},
            "triangles": int(hi_out.shape[0]), "vertices": int(hv_out.shape[0])}


def batched_measurement(amr, s, cs, n_isos):
    """Many iso-values of one set in one batched run (autotuned
    launch shape, replayed from a HIP graph) against the plain path run once
    per iso on the same stream."""
    import numpy as np

    isos = np.quantile(cs.value, 0.05 + 0.90 * np.arange(n_isos) / max(n_isos - 1, 1)).astype(np.float32)
    return batched_isos(amr, s, cs.name, cs.n, isos)


def batched_isos(amr, s, name, n_cells, isos, reps=10, tune_reps=5):
    """One batched run of `isos` on set `s` (autotuned shape, replayed from a
    HIP graph) against one plain call per iso; every job equals its plain
    call bit for bit."""
    import numpy as np
    import torch

    from paper_2004_08475_amd import autotune

    dev = s.device
    n_isos = len(isos)
    b = amr.AmrBatch([s])
    counts = torch.zeros(n_isos, dtype=torch.int64, device=dev)
    probe = b.jobs_tensor([0] * n_isos, isos, np.zeros(n_isos), np.zeros(n_isos))
    b.run_into(probe, n_isos, None, counts)
    c = counts.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(c)[:-1]])
    tris = torch.empty((max(int(c.sum()), 1), 9), dtype=torch.float32, device=dev)
    jobs = b.jobs_tensor([0] * n_isos, isos, off, c)
    block, unit, table = autotune.tune(b, jobs, n_isos, tris, counts, reps=tune_reps)
    ws = b.workspace(n_isos, block, unit)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run_into(jobs, n_isos, tris, counts, block, unit, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run_into(jobs, n_isos, tris, counts, block, unit, ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g.replay()
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    fused_ms = e0.elapsed_time(e1) / reps
    assert counts.cpu().numpy().tolist() == c.tolist()
    # plain path, one launch per iso, into preallocated buffers
    bufs = [torch.empty((max(int(k), 1), 9), dtype=torch.float32, device=dev) for k in c]
    for k in range(n_isos):
        s.isosurface_into(float(isos[k]), bufs[k], int(c[k]))
    plain_reps = 3
    e0.record()
    for _ in range(plain_reps):
        for k in range(n_isos):
            s.isosurface_into(float(isos[k]), bufs[k], int(c[k]))
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / plain_reps
    for k in range(n_isos):
        assert torch.equal(bufs[k][:int(c[k])], tris[int(off[k]):int(off[k]) + int(c[k])])
    del bufs
    return {"workload": "%s x %d isos, one batched run replayed from a HIP graph" % (name, n_isos),
            "fused_ms": fused_ms, "plain_ms_for_all_isos": plain_ms, "speedup_vs_plain": plain_ms / fused_ms,
            "iso_cells_per_s": n_isos * n_cells / (fused_ms * 1e-3), "triangles": int(c.sum()),
            "autotuned_shape": {"block": block, "unit": unit}, "autotune_ms": table}


def batched_multiset_measurement(amr, n_sets=32, seed=4):
    """32 independent octree sets of log-uniform sizes 10k..5M cells, each at
    its own iso (median), in one batched run replayed from a HIP
    graph, against the plain path run once per set."""
    import numpy as np
    import torch

    import amrgen
    from paper_2004_08475_amd import autotune

    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(1e4), np.log(5e6), n_sets)).astype(int)
    css, sets = [], []
    for k, n in enumerate(sizes):
        cs = amrgen.octree_sized(int(n), seed=200 + k)
        css.append(cs)
        sets.append(amr.from_numpy(cs.xyz, cs.level, cs.value))
    say("batched sets: %d sets, %d cells in all" % (n_sets, sum(c.n for c in css)))
    dev = sets[0].device
    isos = np.array([c.iso for c in css], np.float32)
    # two plain counts per set first: the second records the group value
    # ranges, which both the batched launch and the later plain passes use
    for _ in range(2):
        for k in range(n_sets):
            sets[k].isosurface_into(float(isos[k]), None, 0)
    b = amr.AmrBatch(sets)
    counts = torch.zeros(n_sets, dtype=torch.int64, device=dev)
    probe = b.jobs_tensor(list(range(n_sets)), isos, np.zeros(n_sets), np.zeros(n_sets))
    b.run_into(probe, n_sets, None, counts)
    c = counts.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(c)[:-1]])
    tris = torch.empty((max(int(c.sum()), 1), 9), dtype=torch.float32, device=dev)
    jobs = b.jobs_tensor(list(range(n_sets)), isos, off, c)
    block, unit, table = autotune.tune(b, jobs, n_sets, tris, counts)
    ws = b.workspace(n_sets, block, unit)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run_into(jobs, n_sets, tris, counts, block, unit, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run_into(jobs, n_sets, tris, counts, block, unit, ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g.replay()
    e0.record()
    for _ in range(10):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    fused_ms = e0.elapsed_time(e1) / 10
    assert counts.cpu().numpy().tolist() == c.tolist()
    bufs = [torch.empty((max(int(k), 1), 9), dtype=torch.float32, device=dev) for k in c]
    for k in range(n_sets):
        sets[k].isosurface_into(float(isos[k]), bufs[k], int(c[k]))
    e0.record()
    for _ in range(3):
        for k in range(n_sets):
            sets[k].isosurface_into(float(isos[k]), bufs[k], int(c[k]))
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / 3
    for k in range(n_sets):
        assert torch.equal(bufs[k][:int(c[k])], tris[int(off[k]):int(off[k]) + int(c[k])])
    n_cells = int(sum(cs.n for cs in css))
    for st in sets:
        st.close()
    b.close()
    return {"workload": "%d octree sets, log-uniform 10k..5M cells (%d in all), own median iso each, one fused "
                        "launch replayed from a HIP graph" % (n_sets, n_cells),
            "set_cells": [int(cs.n) for cs in css], "fused_ms": fused_ms, "plain_ms_for_all_sets": plain_ms,
            "speedup_vs_plain": plain_ms / fused_ms, "cells_per_s": n_cells / (fused_ms * 1e-3),
            "triangles": int(c.sum()), "autotuned_shape": {"block": block, "unit": unit},
            "autotune_ms": table}, css


def serving_measurement(amr, s, name, iso_pool, seconds, rate, serial_requests=0):
    """Poisson iso/upload requests against the resident set: continuous
    batching server vs. the serial plain path on the same trace (or on its
    first `serial_requests` requests, when that is set)."""
    import numpy as np
    import torch

    import amrgen
    from paper_2004_08475_amd import serve

    rng = np.random.default_rng(5)
    sizes = np.exp(rng.uniform(np.log(1e4), np.log(2e6), 6)).astype(int)
    pool = []
    for k, n in enumerate(sizes):
        pool.append(amrgen.octree_sized(int(n), seed=50 + k))
        say("serving: upload set %d: %d cells" % (k, pool[-1].n))
    isos = np.asarray(iso_pool, np.float32)

    def up(k):
        u = pool[k % len(pool)]
        return serve.UploadRequest(u.xyz, u.level, u.value, u.iso)

    def progress(k, n):
        say("serving: %d/%d requests" % (k, n))

    trace = serve.poisson_trace(rate, seconds, 5, lambda k: isos[k % len(isos)], up, p_upload=0.3)
    srv = serve.IsoServer(s, upload_max_cells=max(p.n for p in pool))
    say("serving: server ready, %d requests in the trace" % len(trace))
    t0 = time.perf_counter()
    res = srv.serve(trace, keep_outputs=False, progress=progress)
    wall = time.perf_counter() - t0
    say("serving: server run done (%d requests, %.1f s)" % (len(res), wall))
    torch.cuda.synchronize()
    strace = trace[:serial_requests] if serial_requests else trace
    t0 = time.perf_counter()
    base = serve.serve_serial(s, strace, progress=progress)
    wall_b = time.perf_counter() - t0
    out = {"workload": "resident %s + uploads of %s-cell octree sets; Poisson %.0f req/s for %.0f s, 30%% uploads"
                       % (name, "/".join(str(p.n) for p in pool), rate, seconds),
           "server": serve.summarize(res, wall), "serial_plain": serve.summarize(base, wall_b),
           "hbm_peak_reserved_bytes": srv.mem.peak,
           "policy_ms": {"plain_pass": srv.t_plain * 1e3, "batch_fixed": srv.t_batch_fixed * 1e3,
                         "batch_per_job": srv.t_batch_job * 1e3,
                         "batch_from_size": next((n for n in range(1, srv.max_batch + 1)
                                                         if not srv.plain_wins(n)), None)}}
    if serial_requests and serial_requests < len(trace):
        out["serial_plain"]["note"] = ("first %d requests of the same trace only (the serial path is saturated, "
                                       "so its latencies only grow with more requests)" % len(strace))
        srv_part = serve.summarize(res[:len(strace)], wall)
        out["server_same_prefix"] = {k: srv_part[k] for k in ("requests", "p50_ms", "p99_ms", "by_kind")}
    return out


def large_serving(amr, seconds, rate, serial_requests, batch_isos=64):
    """Serving against a ~600M-cell octree held resident with its index: the
    octree-shell recipe on 2048^3 with 6 levels (roots of width 32), shell
    480 < r < 560, split probability 0.6 on the shell and 0.575 elsewhere,
    Gaussian widths scaled by 8; generated on the GPU.  With batch_isos, a
    batched run of that many isos (percentiles 5..95) against one culled
    plain call per iso comes first."""
    import numpy as np
    import torch

    import amrgen

    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    xyz, lv, val, iso = amrgen.octree_shell_torch(2048, 5, (480.0, 560.0), 0.6, 0.575, 5, dev,
                                                  sigma=(80.0, 320.0))
    torch.cuda.synchronize()
    n = int(lv.numel())
    say("large serving set: %d cells generated in %.1f s" % (n, time.perf_counter() - t0))
    s = amr.AmrSet(0)
    s.upload(xyz, lv, val)
    t0 = time.perf_counter()
    s.build_index()
    torch.cuda.synchronize()
    say("large serving set: index built in %.1f ms" % ((time.perf_counter() - t0) * 1e3))
    sample = val[torch.randint(0, n, (1 << 24,), device=dev, generator=torch.Generator(dev).manual_seed(5))]
    qs = np.random.default_rng(5).uniform(0.05, 0.95, 97)
    isos = torch.quantile(sample.double(), torch.as_tensor(qs, device=dev)).float().cpu().numpy()
    name = "octree-shell-2048 (%d cells, levels 0..5, p 0.6/0.575)" % n
    batched = None
    if batch_isos:
        # two plain counts first: the second records the group value ranges
        # that both the batched run and the plain calls then cull with
        for _ in range(2):
            s.count(float(isos[0]))
        qs64 = 0.05 + 0.90 * np.arange(batch_isos) / max(batch_isos - 1, 1)
        biso = torch.quantile(sample.double(), torch.as_tensor(qs64, device=dev)).float().cpu().numpy()
        batched = batched_isos(amr, s, "octree-shell-2048", n, biso, reps=3, tune_reps=1)
        batched["workload"] += " (percentiles 5..95 of the values)"
        say("large serving set: batched %d isos %.1f ms, plain %.1f ms" % (batch_isos, batched["fused_ms"],
                                                                          batched["plain_ms_for_all_isos"]))
    out = serving_measurement(amr, s, name, isos, seconds, rate, serial_requests)
    if batched is not None:
        out["batched_resident"] = batched
    out["resident_cells"] = n
    out["resident_bytes"] = {"cells": 20 * n, "index": int(s.workspace.numel())}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="octree-shell-256-2m")
    ap.add_argument("--small", default="octree-shell-256", help="also time the step on this set ('none' to skip)")
    ap.add_argument("--large", default="block-vortex-1024",
                    help="also time the step on this large workload ('none' to skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-index-ab", action="store_true", help="skip the hash / sorted-cells index comparison")
    ap.add_argument("--sampler-points", type=int, default=1 << 22,
                    help="points per launch of the dual-mesh interpolant measurement; 0 = skip")
    ap.add_argument("--latency-requests", type=int, default=200)
    ap.add_argument("--batch-isos", type=int, default=64, help="isos in the batched (fused) measurement; 0 = skip")
    ap.add_argument("--batch-sets", type=int, default=32,
                    help="independent octree sets (10k..5M cells) fused into one launch; 0 = skip")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the serving run; 0 = skip")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate of the serving run")
    ap.add_argument("--serve-workload", default="large", choices=("bench", "large"),
                    help="resident set of the serving run: the ~600M-cell octree, or the bench workload")
    ap.add_argument("--serve-serial-requests", type=int, default=300,
                    help="replay only this many requests through the serial baseline (0 = all)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the host-to-host pipeline timing (transfers, weld, download)")
    ap.add_argument("--no-resident", action="store_true",
                    help="skip the repeated-iso timing on the built set (culled passes), e.g. under a profiler")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library extracts on a single device and has no multi-GPU "
              "path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2004_08475_amd as amr

    amr.load_library()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cs = make_workload(args.workload)
    say("workload %s: %d cells" % (cs.name, cs.n))
    xyz = torch.from_numpy(cs.xyz).to(dev)
    lvl = torch.from_numpy(cs.level).to(dev)
    val = torch.from_numpy(cs.value).to(dev)
    r = step_measurement(amr, cs, xyz, lvl, val, args.steps, args.warmup)
    s, n_tri, n_dual = r["set"], r["n_tri"], r["n_dual"]
    say("timed steps done: %.3f ms/step; dominant kernel %s %.3f ms" % (
        r["ms_per_step"], r["roofline"]["kernel"], r["roofline"]["avg_launch_ms"]))

    # iso requests on the resident set: count pass + write pass, host clock
    isos = np.quantile(cs.value, np.linspace(0.05, 0.95, 19)).astype(np.float32)
    lat = []
    big = torch.empty((max(4 * n_tri, 1024), 9), dtype=torch.float32, device=dev)
    for k in range(args.latency_requests):
        iso = float(isos[k % len(isos)])
        torch.cuda.synchronize()
        ta = time.perf_counter()
        c = s.count(iso)[0]
        buf = big if c <= big.shape[0] else torch.empty((c, 9), dtype=torch.float32, device=dev)
        s.isosurface_into(iso, buf, c)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - ta) * 1e3)

    if args.copy_probe_mib:
        nel = args.copy_probe_mib * (1 << 20) // 4
        xa = torch.ones(nel, dtype=torch.float32, device=dev)
        ya = torch.empty_like(xa)
        torch.mul(xa, 1.0, out=ya)
        torch.cuda.synchronize()

    ms_per_step = r["ms_per_step"]
    # the roofline also against what a plain copy reaches on this GPU
    copy_gbs = copy_peak_gbs()
    r["roofline"]["measured_copy_gbs"] = copy_gbs
    r["roofline"]["frac_of_copy"] = r["roofline"]["achieved"] / copy_gbs
    out = {
        "metric": METRIC,
        "value": cs.n / (ms_per_step * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32+f32",
        "data": "synthetic (seeded generator, shuffled cell order)",
        "config": {"workload": cs.name, "cells": cs.n, "levels": sorted(set(cs.level.tolist())),
                   "iso": cs.iso, "triangles": n_tri, "duals": n_dual,
                   "step": "amr_upload + amr_build_index (verdict read after the timed steps) + amr_isosurface "
                           "(single pass)"},
        "roofline": r["roofline"],
        "kernels_ms": r["kernels_ms"],
        "stages_ms": r["stages_ms"],
        "iso_latency_ms": {"p50": percentile(lat, 0.5), "p99": percentile(lat, 0.99), "requests": len(lat),
                           "what": "count pass + write pass on the resident set, host clock"},
    }
    if not args.no_resident:
        out["resident_iso"] = resident_iso_measurement(s, cs)
    if args.sampler_points:
        out["dual_sampler"] = sampler_measurement(amr, s, cs, args.sampler_points)
        say("dual sampler: %.3g points/s" % out["dual_sampler"]["points_per_s"])
    if args.small != "none":
        cs2 = make_workload(args.small)
        t = [torch.from_numpy(a).to(dev) for a in (cs2.xyz, cs2.level, cs2.value)]
        r2 = step_measurement(amr, cs2, *t, args.steps, args.warmup)
        r2["set"].close()
        out["small_workload"] = {"workload": cs2.name, "cells": cs2.n, "triangles": r2["n_tri"],
                                 "ms_per_step": r2["ms_per_step"], "cells_per_s": r2["cells_per_s"],
                                 "stages_ms": r2["stages_ms"], "kernels_ms": r2["kernels_ms"],
                                 "roofline": r2["roofline"]}
        say("small workload %s: %.3f ms/step" % (cs2.name, r2["ms_per_step"]))
        del t, r2
    large_cs = None
    if args.large != "none":
        large_cs = make_workload(args.large)
        out["large_workload"] = large_measurement(amr, large_cs, 10, resident=not args.no_resident,
                                                  index_ab=not args.no_index_ab)
        say("large workload %s: %.3f ms/step" % (args.large, out["large_workload"]["ms_per_step"]))
    if not args.no_pipeline:
        out["pipeline_pcie_inclusive"] = pipeline_measurement(amr, cs)
        say("pipeline with host transfers: %.3f ms" % out["pipeline_pcie_inclusive"]["ms"])
    if args.batch_isos:
        out["batched"] = batched_measurement(amr, s, cs, args.batch_isos)
        say("batched: fused %.3f ms, plain %.3f ms" % (out["batched"]["fused_ms"],
                                                        out["batched"]["plain_ms_for_all_isos"]))
    set_css = None
    if args.batch_sets:
        out["batched_sets"], set_css = batched_multiset_measurement(amr, args.batch_sets)
        say("batched sets: fused %.3f ms, plain %.3f ms" % (out["batched_sets"]["fused_ms"],
                                                             out["batched_sets"]["plain_ms_for_all_sets"]))
    if args.serve_seconds > 0 and args.serve_workload == "large":
        out["serving"] = large_serving(amr, args.serve_seconds, args.serve_rate, args.serve_serial_requests,
                                       args.batch_isos)
    elif args.serve_seconds > 0:
        iso_pool = np.quantile(cs.value, np.random.default_rng(5).uniform(0.05, 0.95, 97)).astype(np.float32)
        out["serving"] = serving_measurement(amr, s, cs.name, iso_pool, args.serve_seconds, args.serve_rate,
                                             args.serve_serial_requests)
    if "serving" in out:
        say("serving: p99 %.2f ms (server) vs %.2f ms (serial)" % (out["serving"]["server"]["p99_ms"],
                                                                  out["serving"]["serial_plain"]["p99_ms"]))
    if not args.no_index_ab:
        # last use of the headline set: this rebuilds its index
        out["index_ab"] = index_measurement(amr, s, cs)
        say("index A/B: snaps %s ms" % out["index_ab"]["snap_ms"])
    if not args.no_cpu_baseline:
        say("cpu baseline: running the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(cs, large=large_cs, sets=set_css)
        say("cpu baseline: %.3g cells/s on %d threads" % (out["cpu_baseline"]["value"], out["cpu_baseline"]["cores"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
