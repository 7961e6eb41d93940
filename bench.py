"""Benchmark: AMR cells/s to crack-free triangles on one MI355X.

One step = the whole hot path over one synthetic AMR set that is already in
HBM: validate + reduce (amr_upload), build the cell-location index
(amr_build_index) and extract the iso-surface (amr_isosurface, one pass into
a buffer sized by the warm-up).  Prints one JSON line: the step rate of the
136,935-cell octree (the value), its roofline (HBM; beside it the VALU issue
fraction and L2 hit rates from the committed counter summaries), iso latency
and repeated isos on the built set, the same step on the 50.8M-cell
block-structured set, the host-to-host pipeline, batched launches, a serving
run and the CPU oracle's rate.

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


def make_workload(name):
    import amrgen

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


def cpu_baseline(cs, min_seconds=10.0):
    """The oracle as it is, on the host's cores: sorted index + rules + MC
    over the whole set, repeated until about min_seconds have passed."""
    import oracle

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    reps, t_total = 0, 0.0
    tris = 0
    while t_total < min_seconds and reps < 10000:
        t0 = time.perf_counter()
        o = oracle.Oracle(cs.xyz, cs.level, cs.value, validate=False)
        tris, _ = o.isosurface_threaded(cs.iso, threads)
        t_total += time.perf_counter() - t0
        reps += 1
        del o
    # the same oracle on one thread, once over the same set
    t0 = time.perf_counter()
    o = oracle.Oracle(cs.xyz, cs.level, cs.value, validate=False)
    o.count_range(cs.iso, 0, cs.n)
    t_one = time.perf_counter() - t0
    del o
    # the brute-force locator (a scan over all cells per snap) on the 960-cell two-level sphere
    import amrgen

    c1 = amrgen.two_level_sphere()
    t0 = time.perf_counter()
    ob = oracle.Oracle(c1.xyz, c1.level, c1.value, locator="brute", validate=False)
    ob.count_range(c1.iso, 0, c1.n)
    t_brute = time.perf_counter() - t0
    return {"value": cs.n * reps / t_total, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": "whole %s set (%d cells, %d triangles), sorted-corner index + rules 1-3 + Marching Cubes, "
                      "%d repetitions, %.1f s" % (cs.name, cs.n, tris, reps, t_total),
            "one_thread": {"value": cs.n / t_one, "seconds": t_one},
            "brute_force": {"workload": c1.name, "cells": c1.n, "value": c1.n / t_brute, "seconds": t_brute}}


def batched_measurement(amr, s, cs, n_isos):
    """Many iso-values of one set in one fused persistent launch (autotuned
    launch shape, replayed from a HIP graph) against the plain path run once
    per iso on the same stream."""
    import numpy as np
    import torch

    from paper_2004_08475_amd import autotune

    dev = s.device
    isos = np.quantile(cs.value, 0.05 + 0.90 * np.arange(n_isos) / max(n_isos - 1, 1)).astype(np.float32)
    t0 = time.perf_counter()
    b = amr.AmrBatch([s])
    torch.cuda.synchronize()
    t_duals = time.perf_counter() - t0
    counts = torch.zeros(n_isos, dtype=torch.int64, device=dev)
    probe = b.jobs_tensor([0] * n_isos, isos, np.zeros(n_isos), np.zeros(n_isos))
    b.run_into(probe, n_isos, None, counts)
    c = counts.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(c)[:-1]])
    tris = torch.empty((max(int(c.sum()), 1), 9), dtype=torch.float32, device=dev)
    jobs = b.jobs_tensor([0] * n_isos, isos, off, c)
    block, per, table = autotune.tune(b, jobs, n_isos, tris, counts)
    ws = b.workspace(n_isos, block, per)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run_into(jobs, n_isos, tris, counts, block, per, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run_into(jobs, n_isos, tris, counts, block, per, ws)
    reps = 10
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
    e0.record()
    for _ in range(3):
        for k in range(n_isos):
            s.isosurface_into(float(isos[k]), bufs[k], int(c[k]))
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / 3
    for k in range(n_isos):
        assert torch.equal(bufs[k][:int(c[k])], tris[int(off[k]):int(off[k]) + int(c[k])])
    return {"workload": "%s x %d isos (percentiles 5..95), one fused launch replayed from a HIP graph" % (cs.name, n_isos),
            "fused_ms": fused_ms, "plain_ms_for_all_isos": plain_ms, "speedup_vs_plain": plain_ms / fused_ms,
            "iso_cells_per_s": n_isos * cs.n / (fused_ms * 1e-3), "triangles": int(c.sum()),
            "dual_list_ms": t_duals * 1e3, "autotuned_shape": {"block": block, "per_thread": per},
            "autotune_ms": table}


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


def large_serving(amr, seconds, rate, serial_requests):
    """Serving against a ~600M-cell octree held resident with its index: the
    octree-shell recipe on 2048^3 with 6 levels (roots of width 32), shell
    480 < r < 560, split probability 0.6 on the shell and 0.575 elsewhere,
    Gaussian widths scaled by 8; generated on the GPU."""
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
    out = serving_measurement(amr, s, name, isos, seconds, rate, serial_requests)
    out["resident_cells"] = n
    out["resident_bytes"] = {"cells": 20 * n, "index": int(s.workspace.numel())}
    return out


def batched_multiset_measurement(amr, n_sets=32, seed=4):
    """32 independent octree sets of log-uniform sizes 10k..5M cells, each at
    its own iso (median), in one fused persistent launch replayed from a HIP
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
    b = amr.AmrBatch(sets)
    isos = np.array([c.iso for c in css], np.float32)
    counts = torch.zeros(n_sets, dtype=torch.int64, device=dev)
    probe = b.jobs_tensor(list(range(n_sets)), isos, np.zeros(n_sets), np.zeros(n_sets))
    b.run_into(probe, n_sets, None, counts)
    c = counts.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(c)[:-1]])
    tris = torch.empty((max(int(c.sum()), 1), 9), dtype=torch.float32, device=dev)
    jobs = b.jobs_tensor(list(range(n_sets)), isos, off, c)
    block, per, table = autotune.tune(b, jobs, n_sets, tris, counts)
    ws = b.workspace(n_sets, block, per)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run_into(jobs, n_sets, tris, counts, block, per, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run_into(jobs, n_sets, tris, counts, block, per, ws)
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
    return {"workload": "%d octree sets, log-uniform 10k..5M cells (%d in all), own median iso each, one fused "
                        "launch replayed from a HIP graph" % (n_sets, n_cells),
            "set_cells": [int(cs.n) for cs in css], "fused_ms": fused_ms, "plain_ms_for_all_sets": plain_ms,
            "speedup_vs_plain": plain_ms / fused_ms, "cells_per_s": n_cells / (fused_ms * 1e-3),
            "triangles": int(c.sum()), "autotuned_shape": {"block": block, "per_thread": per}, "autotune_ms": table}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_extract_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2004_08475_amd", "csrc", "amriso.hip")


def traffic_for(workload):
    """HBM bytes per amr_isosurface call from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None when
    there is none for this workload or the kernel source changed since."""
    import hashlib

    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = [ln.split() for ln in lines if ln and not ln.startswith("#")]
    recorded = [f[1] for f in fields if f[0] == "source_sha256"]
    if not recorded or recorded[0] != src:
        return None
    for f in fields:
        if f[0] == "workload" and f[1] == workload:
            kv = dict(zip(f[2::2], f[3::2]))
            return float(kv["traffic_bytes"])
    return None


VALU_FILE = os.path.join(ROOT, "profiles", "k_extract_valu.txt")
L2_FILE = os.path.join(ROOT, "profiles", "k_extract_l2.txt")


def _per_kernel(path, workload):
    """Per extraction kernel of this workload, the last figure of its line in
    a committed rocprofv3 counter summary, or None when there is none or the
    kernel source changed since the counters were taken."""
    import hashlib

    try:
        lines = open(path).read().splitlines()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    recorded = [ln.split()[1] for ln in lines if ln.startswith("source_sha256")]
    if not recorded or recorded[0] != src:
        return None
    out = {}
    for ln in lines:
        if ln.startswith(workload + " "):
            kernel = ln[len(workload) + 1:].split(":")[0]
            out[kernel] = float(ln.rsplit("|", 1)[1])
    return out or None


def valu_for(workload):
    """Fraction of the VALU issue peak per extraction kernel (SQ counters)."""
    return _per_kernel(VALU_FILE, workload)


def l2_hit_for(workload):
    """L2 hit rate per extraction kernel (TCC counters)."""
    return _per_kernel(L2_FILE, workload)


def time_steps(amr, s, xyz, lvl, val, iso, cap, tris, steps, warmup):
    """Whole-path steps (upload + build + iso).  The timed run has nothing
    but the steps between two synchronisations (host clock); a second run of
    the same steps records HIP events between the stages, on the stream the
    kernels run on, for the per-stage split.  Returns (ms per step, stage
    lists from the instrumented run)."""
    import torch

    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        s.upload(xyz, lvl, val)
        if ev:
            ev[1].record(stream)
        s.build_index()
        if ev:
            ev[2].record(stream)
        s.isosurface_into(iso, tris, cap)
        if ev:
            ev[3].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    st = ([e[0].elapsed_time(e[1]) for e in evs], [e[1].elapsed_time(e[2]) for e in evs],
          [e[2].elapsed_time(e[3]) for e in evs])
    return ms, st


def roofline_of(n_cells, n_tri, iso_ms, traffic, valu=None, l2_hit=None):
    alg = 20.0 * n_cells + 36.0 * n_tri
    achieved = alg / (iso_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "k_extract passes of one amr_isosurface call", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes": alg, "avg_launch_ms": iso_ms, "valu_issue_frac": valu, "l2_hit_rate": l2_hit}


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


def large_measurement(amr, name, steps, resident=True):
    """The same whole-path step on a large set (block-structured, 50.8M
    cells), where throughput rather than launch latency decides."""
    import torch

    cs = make_workload(name)
    dev = torch.device("cuda", 0)
    xyz, lvl, val = (torch.from_numpy(a).to(dev) for a in (cs.xyz, cs.level, cs.value))
    s = amr.AmrSet(0)
    s.upload(xyz, lvl, val)
    s.build_index()
    n_tri, n_dual = s.count(cs.iso)
    tris = torch.empty((max(n_tri, 1), 9), dtype=torch.float32, device=dev)
    ms, (up, bd, iso) = time_steps(amr, s, xyz, lvl, val, cs.iso, n_tri, tris, steps, 2)
    assert int(s.counts[0].item()) == n_tri
    iso_avg = statistics.mean(iso)
    resident = resident_iso_measurement(s, cs) if resident else None
    out = {"workload": name, "cells": cs.n, "triangles": n_tri, "duals": n_dual, "steps": steps,
           "ms_per_step": ms, "cells_per_s": cs.n / (ms * 1e-3),
           "stages_ms": {"upload": statistics.mean(up), "build_index": statistics.mean(bd), "isosurface": iso_avg},
           "iso_only_cells_per_s": cs.n / (iso_avg * 1e-3),
           "roofline": roofline_of(cs.n, n_tri, iso_avg, traffic_for(name), valu_for(name), l2_hit_for(name)),
           "resident_iso": resident}
    del s, xyz, lvl, val, tris
    torch.cuda.empty_cache()
    return out


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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="octree-shell-256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-requests", type=int, default=200)
    ap.add_argument("--batch-isos", type=int, default=64, help="isos in the batched (fused) measurement; 0 = skip")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="length of the serving run; 0 = skip")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate of the serving run")
    ap.add_argument("--serve-workload", default="bench", choices=("bench", "large"),
                    help="resident set of the serving run: the bench workload, or the ~600M-cell octree")
    ap.add_argument("--serve-serial-requests", type=int, default=0,
                    help="replay only this many requests through the serial baseline (0 = all)")
    ap.add_argument("--large", default="block-vortex-1024",
                    help="also time the step on this large workload ('none' to skip)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the host-to-host pipeline timing (transfers, weld, download)")
    ap.add_argument("--batch-sets", type=int, default=0,
                    help="also fuse this many independent octree sets (10k..5M cells) into one launch")
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
    s = amr.AmrSet(0)
    s.upload(xyz, lvl, val)
    s.build_index()
    n_tri, n_dual = s.count(cs.iso)
    cap = n_tri
    tris = torch.empty((max(cap, 1), 9), dtype=torch.float32, device=dev)
    ms_per_step, (up_ms, bd_ms, iso_ms) = time_steps(amr, s, xyz, lvl, val, cs.iso, cap, tris, args.steps,
                                                      args.warmup)
    assert int(s.counts[0].item()) == n_tri

    # iso requests on the resident set: count pass + write pass, host clock
    isos = np.quantile(cs.value, np.linspace(0.05, 0.95, 19)).astype(np.float32)
    lat = []
    big = torch.empty((max(4 * cap, 1024), 9), dtype=torch.float32, device=dev)
    for r in range(args.latency_requests):
        iso = float(isos[r % len(isos)])
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

    iso_avg = statistics.mean(iso_ms)
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
                   "step": "amr_upload + amr_build_index + amr_isosurface (single pass)"},
        "stages_ms": {"upload": statistics.mean(up_ms), "build_index": statistics.mean(bd_ms),
                      "isosurface": iso_avg},
        "iso_only_cells_per_s": cs.n / (iso_avg * 1e-3),
        "iso_latency_ms": {"p50": percentile(lat, 0.5), "p99": percentile(lat, 0.99), "requests": len(lat),
                           "what": "count pass + write pass on the resident set, host clock"},
        "roofline": roofline_of(cs.n, n_tri, iso_avg, traffic_for(cs.name), valu_for(cs.name),
                                l2_hit_for(cs.name)),
    }
    if not args.no_resident:
        out["resident_iso"] = resident_iso_measurement(s, cs)
    say("timed steps done: %.3f ms/step" % ms_per_step)
    if args.large != "none":
        out["large_workload"] = large_measurement(amr, args.large, 10, resident=not args.no_resident)
        say("large workload %s: %.3f ms/step" % (args.large, out["large_workload"]["ms_per_step"]))
    if not args.no_pipeline:
        out["pipeline_pcie_inclusive"] = pipeline_measurement(amr, cs)
        say("pipeline with host transfers: %.3f ms" % out["pipeline_pcie_inclusive"]["ms"])
    if args.batch_isos:
        out["batched"] = batched_measurement(amr, s, cs, args.batch_isos)
        say("batched: fused %.3f ms, plain %.3f ms" % (out["batched"]["fused_ms"],
                                                        out["batched"]["plain_ms_for_all_isos"]))
    if args.batch_sets:
        out["batched_sets"] = batched_multiset_measurement(amr, args.batch_sets)
        say("batched sets: fused %.3f ms, plain %.3f ms" % (out["batched_sets"]["fused_ms"],
                                                             out["batched_sets"]["plain_ms_for_all_sets"]))
    if args.serve_seconds > 0 and args.serve_workload == "large":
        out["serving"] = large_serving(amr, args.serve_seconds, args.serve_rate, args.serve_serial_requests)
    elif args.serve_seconds > 0:
        iso_pool = np.quantile(cs.value, np.random.default_rng(5).uniform(0.05, 0.95, 97)).astype(np.float32)
        out["serving"] = serving_measurement(amr, s, cs.name, iso_pool, args.serve_seconds, args.serve_rate,
                                             args.serve_serial_requests)
        say("serving: p99 %.2f ms (server) vs %.2f ms (serial)" % (out["serving"]["server"]["p99_ms"],
                                                                  out["serving"]["serial_plain"]["p99_ms"]))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cs)
        say("cpu baseline: %.3g cells/s on %d threads" % (out["cpu_baseline"]["value"], out["cpu_baseline"]["cores"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
