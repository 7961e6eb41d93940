"""Launch-shape autotuner for batched iso-surfaces.

Times every (threads per work-group, groups per work-group) shape in
SHAPES on the caller's actual batch, keeps the fastest, and caches the
choice in a JSON file keyed by GPU architecture and batch shape, so later
processes skip the search.  Cache path: $AMRISO_TUNE_CACHE, else
~/.cache/amriso/autotune.json.
"""
from __future__ import annotations

import json
import math
import os
import threading

import torch

SHAPES = ((128, 64), (128, 128), (128, 256), (128, 512), (256, 64), (256, 128), (256, 256), (256, 512))
_lock = threading.Lock()


def cache_path() -> str:
    return os.environ.get("AMRISO_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "amriso",
                                                            "autotune.json"))


def _key(batch, n_jobs: int) -> str:
    arch = torch.cuda.get_device_properties(batch.device).gcnArchName.split(":")[0]
    cells = batch.cells
    bucket = 0 if cells == 0 else int(round(math.log2(cells)))
    return "%s|units-v3|sets=%d|cells=2^%d|jobs=%d" % (arch, len(batch.sets), bucket, n_jobs)


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(table: dict):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only costs a re-tune


def time_shape(batch, jobs, n_jobs, tris, counts, block, unit, reps=5):
    """Mean milliseconds of one batched run with this shape."""
    ws = batch.workspace(n_jobs, block, unit)
    batch.run_into(jobs, n_jobs, tris, counts, block, unit, ws)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        batch.run_into(jobs, n_jobs, tris, counts, block, unit, ws)
    e1.record()
    torch.cuda.synchronize(batch.device)
    return e0.elapsed_time(e1) / reps


def tune(batch, jobs, n_jobs, tris, counts, reps=5, use_cache=True):
    """(block, unit, table of timings) for this batch and job list."""
    key = _key(batch, n_jobs)
    with _lock:
        table = _load() if use_cache else {}
        hit = table.get(key)
    if hit:
        return int(hit["block"]), int(hit["unit"]), hit.get("ms", {})
    ms = {}
    for block, unit in SHAPES:
        ms["%dx%d" % (block, unit)] = time_shape(batch, jobs, n_jobs, tris, counts, block, unit, reps)
    best = min(ms, key=ms.get)
    block, unit = (int(x) for x in best.split("x"))
    if use_cache:
        with _lock:
            table = _load()
            table[key] = {"block": block, "unit": unit, "ms": ms}
            _store(table)
    return block, unit, ms
