"""Continuous-batching iso-surface server on one GPU.

A resident AMR set stays on the device with its index.  Requests arrive
over time:

  * IsoRequest(iso): an iso-surface of the resident set.  Requests that are
    waiting when the iso stream becomes free are taken together: as one
    batched launch (amr_batch_isosurface: each tile's neighbourhoods read
    once, every waiting iso run against them) or as plain passes one after
    the other, whichever a start-up calibration says is cheaper for that
    many; both skip groups by their recorded value ranges.  New requests
    join the next batch instead of waiting for a queue to drain.
  * UploadRequest(xyz, level, value, iso): a new small set; it is copied
    to the GPU, validated, indexed and extracted on one of several upload
    streams, overlapping on the device with the iso work.

Outputs and upload cell buffers live on the device, reused across requests (grown when a
request needs more), so that allocations, which can stall every stream,
stop once the sizes have been seen.

Admission is by memory: every request reserves an estimate of the device
memory it needs against an HBM budget and waits (first come, first served)
until it fits, so a small budget makes requests queue instead of running
out of memory.  Latency is measured from arrival to the result being ready
on the device.  `serve_serial` replays the same trace one request at a
time through the plain single-iso path, as the baseline.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np
import torch

from . import AmrBatch, AmrSet


@dataclasses.dataclass
class IsoRequest:
    iso: float
    rid: int = -1


@dataclasses.dataclass
class UploadRequest:
    xyz: np.ndarray
    level: np.ndarray
    value: np.ndarray
    iso: float
    rid: int = -1


@dataclasses.dataclass
class Result:
    rid: int
    kind: str
    arrival: float
    start: float = 0.0
    done: float = 0.0
    triangles: int = 0
    tris: torch.Tensor | None = None

    @property
    def latency_ms(self) -> float:
        return (self.done - self.arrival) * 1e3


class HbmBudget:
    """Bytes of device memory that admitted requests may hold at once."""

    def __init__(self, budget: int):
        self.budget = int(budget)
        self.used = 0
        self.peak = 0
        self.cv = threading.Condition()

    def acquire(self, nbytes: int, stop: threading.Event):
        nbytes = min(int(nbytes), self.budget)
        with self.cv:
            while self.used + nbytes > self.budget and not stop.is_set():
                self.cv.wait(0.01)
            self.used += nbytes
            self.peak = max(self.peak, self.used)
        return nbytes

    def release(self, nbytes: int):
        with self.cv:
            self.used -= nbytes
            self.cv.notify_all()


def upload_bytes(n_cells: int, triangles_guess: int) -> int:
    """Device memory of one upload request: cells, index, triangles."""
    return 20 * n_cells + 64 * n_cells + 36 * triangles_guess + (1 << 20)


class _Grow:
    """A device buffer reused from request to request and grown when a
    request needs more rows: an allocation, which can stall the other
    streams, only happens while the sizes still grow.  Used by one thread at
    a time."""

    def __init__(self, cols, dtype, device):
        self.cols, self.dtype, self.device = cols, dtype, device
        self.buf = None

    def rows(self, n: int) -> torch.Tensor:
        n = max(int(n), 1)
        if self.buf is None or self.buf.shape[0] < n:
            m = max(n, int(1.25 * (0 if self.buf is None else self.buf.shape[0])))
            shape = (m,) if self.cols is None else (m, self.cols)
            self.buf = torch.empty(shape, dtype=self.dtype, device=self.device)
        return self.buf[:n]


class _UploadSlot:
    """One upload stream with its set handle and device buffers (cells,
    output), kept for the server's lifetime (freeing device memory would
    synchronise the whole device)."""

    def __init__(self, device, max_cells: int = 0):
        self.stream = torch.cuda.Stream(device)
        self.set = AmrSet(device.index)
        self.dev = [_Grow(3, torch.int32, device), _Grow(None, torch.int32, device), _Grow(None, torch.float32, device)]
        self.out = _Grow(9, torch.float32, device)
        if max_cells > 0:
            for g in self.dev:
                g.rows(max_cells)
            self.out.rows(max_cells // 2)
            # index a block of max_cells unit cells once, so that the set
            # keeps an index workspace of about the size such uploads need
            k = int(np.ceil(max_cells ** (1.0 / 3.0)))
            i = torch.arange(max_cells, dtype=torch.int32, device=device)
            xyz = self.dev[0].rows(max_cells)
            xyz[:, 0], xyz[:, 1], xyz[:, 2] = i % k, (i // k) % k, i // (k * k)
            self.dev[1].rows(max_cells).zero_()
            self.dev[2].rows(max_cells).zero_()
            self.set.upload(*(d.rows(max_cells) for d in self.dev))
            self.set.build_index()


class IsoServer:
    def __init__(self, resident: AmrSet, hbm_budget: int | None = None, upload_slots: int = 4,
                 max_batch: int = 64, block: int | None = None, unit: int | None = None,
                 curve_points: int = 64, upload_max_cells: int = 0):
        self.resident = resident
        self.device = resident.device
        self.batch = AmrBatch([resident])
        self.max_batch = max_batch
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(free * 0.8)
        self.mem = HbmBudget(hbm_budget)
        # triangle-count curve of the resident set: sizes batched outputs
        vals = resident._cells[2]
        qs = torch.linspace(0.0, 1.0, curve_points, device=self.device, dtype=torch.float64)
        sample = vals if vals.numel() <= 1 << 24 else vals[torch.randint(0, vals.numel(), (1 << 24,),
                                                                           device=self.device)]
        self.curve_iso = torch.quantile(sample.double(), qs).float().cpu().numpy()
        counts = torch.zeros(curve_points, dtype=torch.int64, device=self.device)
        jobs = self.batch.jobs_tensor([0] * curve_points, self.curve_iso, np.zeros(curve_points),
                                      np.zeros(curve_points))
        if block is None or unit is None:
            # launch shape for this set: the autotuner on a counting launch of
            # a few isos from the middle of the curve (no output memory)
            from . import autotune

            k = 8
            mid = self.curve_iso[curve_points // 4:curve_points // 4 + k]
            tj = self.batch.jobs_tensor([0] * k, mid, np.zeros(k), np.zeros(k))
            tc = torch.zeros(k, dtype=torch.int64, device=self.device)
            block, unit, _ = autotune.tune(self.batch, tj, k, None, tc, reps=2)
        self.block, self.unit = block, unit
        self.batch.run_into(jobs, curve_points, None, counts, block, unit)
        self.curve_tri = counts.cpu().numpy()
        # per request, the plain single pass against a batched launch (fixed
        # part + part per job), timed once here; a batch of n waiting
        # requests takes whichever is cheaper for n
        self.t_plain, self.t_batch_fixed, self.t_batch_job = self._calibrate()
        self.upload_slots = upload_slots
        self.stop = threading.Event()
        # request outputs live in buffers reused across requests
        self._iso_stream = torch.cuda.Stream(self.device)
        self._iso_out = _Grow(9, torch.float32, self.device)
        self._batch_counts = torch.zeros(max_batch, dtype=torch.int64, device=self.device)
        # upload_max_cells > 0 sizes the upload buffers and index workspaces
        # for sets up to that many cells now rather than on first use
        self._slots = [_UploadSlot(self.device, upload_max_cells) for _ in range(upload_slots)]
        # warm-up on the iso stream, into the output buffer sized for the
        # largest lone request on the triangle-count curve
        with torch.cuda.stream(self._iso_stream):
            iso = float(self.curve_iso[len(self.curve_iso) // 2])
            big = max(self.iso_cap(float(v)) for v in self.curve_iso)
            self.resident.isosurface_into(iso, self._iso_out.rows(big), big)
        torch.cuda.synchronize(self.device)

    def _calibrate(self, reps: int = 3):
        """(plain pass, batch fixed part, batch part per job) in seconds, on
        isos from the middle of the value range.  The plain path is timed
        after its first two calls on the set (the second records the group
        value ranges that later calls cull with)."""
        mid = len(self.curve_iso) // 2
        isos = [float(self.curve_iso[mid]), float(self.curve_iso[min(mid + 1, len(self.curve_iso) - 1)])]
        caps = [self.iso_cap(v) for v in isos]
        tris = torch.empty((sum(caps), 9), dtype=torch.float32, device=self.device)
        counts = torch.zeros(2, dtype=torch.int64, device=self.device)
        jobs1 = self.batch.jobs_tensor([0], isos[:1], [0], caps[:1])
        jobs2 = self.batch.jobs_tensor([0, 0], isos, [0, caps[0]], caps)

        def run(fn, warm=2):
            for _ in range(warm):
                fn()
            torch.cuda.synchronize(self.device)
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize(self.device)
            return (time.perf_counter() - t0) / reps

        t_plain = run(lambda: self.resident.isosurface_into(isos[0], tris, caps[0]))
        t1 = run(lambda: self.batch.run_into(jobs1, 1, tris, counts, self.block, self.unit))
        t2 = run(lambda: self.batch.run_into(jobs2, 2, tris, counts, self.block, self.unit))
        per_job = max(t2 - t1, 0.0)
        return t_plain, max(t1 - per_job, 0.0), per_job

    def plain_wins(self, n: int) -> bool:
        """True when n plain passes cost no more than one batched launch of n."""
        return n * self.t_plain <= self.t_batch_fixed + n * self.t_batch_job

    # -- sizing -----------------------------------------------------------
    def iso_cap(self, iso: float) -> int:
        k = int(np.searchsorted(self.curve_iso, iso))
        lo, hi = max(k - 1, 0), min(k, len(self.curve_iso) - 1)
        return int(2 * max(self.curve_tri[lo], self.curve_tri[hi]) + 4096)

    # -- resident iso requests --------------------------------------------
    def _run_one(self, r, results, stream):
        """A lone request: the plain single-pass path with the capacity taken
        from the triangle-count curve (a second pass only if it was short)."""
        cap = self.iso_cap(r.iso)
        held = self.mem.acquire(cap * 36 + (1 << 20), self.stop)
        t_start = time.perf_counter()
        try:
            with torch.cuda.stream(stream):
                tris = self._iso_out.rows(cap)
                counts = self.resident.isosurface_into(r.iso, tris, cap)
                c = int(counts[0].item())
                if c > cap:
                    tris = self._iso_out.rows(c)
                    self.resident.isosurface_into(r.iso, tris, c)
                kept = self._keep(tris[:c])
                stream.synchronize()
                res = results[r.rid]
                res.start, res.done, res.triangles, res.tris = t_start, time.perf_counter(), c, kept
        finally:
            self.mem.release(held)

    def _run_batch(self, reqs, results, stream):
        n = len(reqs)
        if self.plain_wins(n):
            # one plain pass after the other: each request completes as soon
            # as its own pass has
            for r in reqs:
                self._run_one(r, results, stream)
            return
        isos = [r.iso for r in reqs]
        caps = np.array([self.iso_cap(v) for v in isos], np.int64)
        need = int(caps.sum()) * 36 + (1 << 20)
        held = self.mem.acquire(need, self.stop)
        t_start = time.perf_counter()
        try:
            with torch.cuda.stream(stream):
                off = np.concatenate([[0], np.cumsum(caps)[:-1]])
                tris = self._iso_out.rows(int(caps.sum()))
                counts = self._batch_counts[:n]
                jobs = self.batch.jobs_tensor([0] * n, isos, off, caps)
                self.batch.run_into(jobs, n, tris, counts, self.block, self.unit)
                c = counts.cpu().numpy()
                kept = []
                for k in range(n):
                    out = tris[int(off[k]):int(off[k]) + int(c[k])]
                    if c[k] > caps[k]:  # the estimate was short: exact rerun
                        out = self.resident.isosurface(isos[k], int(c[k]))["tris"]
                    kept.append(self._keep(out))
                stream.synchronize()
                t_done = time.perf_counter()
                for k, r in enumerate(reqs):
                    res = results[r.rid]
                    res.start, res.done, res.triangles, res.tris = t_start, t_done, int(c[k]), kept[k]
        finally:
            self.mem.release(held)

    def _keep(self, out):
        # outputs are dropped at once unless the caller keeps them, so that
        # finished requests do not pin device memory; kept ones are copied out
        # of the reused output buffer
        return out.clone() if self.keep_outputs else None

    def _guard(self, fn, *args):
        try:
            fn(*args)
        except BaseException as e:  # reported by serve() after the join
            self.errors.append(e)
            self.stop.set()

    def _batch_worker(self, q, results):
        stream = self._iso_stream
        while True:
            with q["cv"]:
                while not q["items"] and not q["closed"]:
                    q["cv"].wait(0.005)
                if not q["items"] and q["closed"]:
                    return
                # continuous batching: take what is waiting, up to max_batch
                # requests and a quarter of the memory budget of outputs
                reqs, est = [], 0
                while q["items"] and len(reqs) < self.max_batch:
                    b = 36 * self.iso_cap(q["items"][0].iso)
                    if reqs and est + b > self.mem.budget // 4:
                        break
                    reqs.append(q["items"].popleft())
                    est += b
            self._run_batch(reqs, results, stream)

    # -- upload requests --------------------------------------------------
    def _run_upload(self, r: UploadRequest, results, slot: _UploadSlot):
        n = len(r.level)
        held = self.mem.acquire(upload_bytes(n, n // 2), self.stop)
        t_start = time.perf_counter()
        try:
            with torch.cuda.stream(slot.stream):
                # straight from the caller's arrays (a copy through pinned
                # staging on the host measured slower for large sets)
                cells = []
                for d, a, dt in zip(slot.dev, (r.xyz, r.level, r.value), (np.int32, np.int32, np.float32)):
                    db = d.rows(n)
                    db.copy_(torch.from_numpy(np.ascontiguousarray(a, dt)).view(db.shape))
                    cells.append(db)
                s = slot.set
                s.upload(*cells)
                s.build_index()
                t, _ = s.count(r.iso)
                tris = slot.out.rows(t)
                s.isosurface_into(r.iso, tris, t)
                kept = self._keep(tris[:t])
                slot.stream.synchronize()
                res = results[r.rid]
                res.start, res.done, res.triangles, res.tris = t_start, time.perf_counter(), t, kept
        finally:
            self.mem.release(held)

    def _upload_worker(self, q, results, slot: _UploadSlot):
        while True:
            with q["cv"]:
                while not q["items"] and not q["closed"]:
                    q["cv"].wait(0.005)
                if not q["items"] and q["closed"]:
                    break
                r = q["items"].popleft()
            self._run_upload(r, results, slot)

    # -- driver -----------------------------------------------------------
    def serve(self, trace, keep_outputs: bool = True, progress=None):
        """Replay `trace` = [(arrival seconds from start, request)] in real
        time.  Returns the list of Results (one per request, in trace order).
        `progress(k, n)` is called every 100 submitted requests."""
        mk = lambda: {"items": collections.deque(), "cv": threading.Condition(), "closed": False}
        iso_q, up_q = mk(), mk()
        results = {}
        self.keep_outputs = keep_outputs
        self.errors = []
        workers = [threading.Thread(target=self._guard, args=(self._batch_worker, iso_q, results), daemon=True)]
        workers += [threading.Thread(target=self._guard, args=(self._upload_worker, up_q, results, slot), daemon=True)
                    for slot in self._slots]
        for w in workers:
            w.start()
        t0 = time.perf_counter()
        for rid, (at, req) in enumerate(trace):
            req.rid = rid
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            arrival = time.perf_counter()
            kind = "iso" if isinstance(req, IsoRequest) else "upload"
            results[rid] = Result(rid, kind, arrival)
            q = iso_q if kind == "iso" else up_q
            with q["cv"]:
                q["items"].append(req)
                q["cv"].notify()
            if progress and (rid + 1) % 100 == 0:
                progress(rid + 1, len(trace))
        for q in (iso_q, up_q):
            with q["cv"]:
                q["closed"] = True
                q["cv"].notify_all()
        for w in workers:
            w.join()
        if self.errors:
            raise RuntimeError("a serving worker failed") from self.errors[0]
        out = [results[i] for i in range(len(trace))]
        if not keep_outputs:
            for r in out:
                r.tris = None
        return out


def serve_serial(resident: AmrSet, trace, keep_outputs: bool = False, progress=None):
    """Baseline: the same trace, one request at a time, plain single-iso path
    (count pass + write pass), in arrival order on one stream.  `progress(k,
    n)` is called every 100 finished requests."""
    results = []
    t0 = time.perf_counter()
    dev = resident.device
    for rid, (at, req) in enumerate(trace):
        now = time.perf_counter() - t0
        if at > now:
            time.sleep(at - now)
        arrival = t0 + at
        start = time.perf_counter()
        if isinstance(req, IsoRequest):
            out = resident.isosurface(req.iso)["tris"]
            kind = "iso"
        else:
            s = AmrSet(dev.index)
            s.upload(torch.from_numpy(np.ascontiguousarray(req.xyz, np.int32)).to(dev),
                     torch.from_numpy(np.ascontiguousarray(req.level, np.int32)).to(dev),
                     torch.from_numpy(np.ascontiguousarray(req.value, np.float32)).to(dev))
            s.build_index()
            out = s.isosurface(req.iso)["tris"]
            kind = "upload"
        torch.cuda.synchronize(dev)
        r = Result(rid, kind, arrival, start, time.perf_counter(), int(out.shape[0]), out if keep_outputs else None)
        results.append(r)
        if progress and (rid + 1) % 100 == 0:
            progress(rid + 1, len(trace))
    return results


def poisson_trace(rate_hz: float, duration_s: float, seed: int, make_iso, make_upload, p_upload: float):
    """Arrivals of a Poisson process; each request is an upload with
    probability p_upload, else a resident iso request."""
    rng = np.random.default_rng(seed)
    t, trace, k = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s:
            return trace
        if rng.random() < p_upload:
            trace.append((t, make_upload(k)))
        else:
            trace.append((t, IsoRequest(float(make_iso(k)))))
        k += 1


def summarize(results, wall_s: float) -> dict:
    lat = np.array([r.latency_ms for r in results]) if results else np.zeros(1)
    by = {}
    for kind in ("iso", "upload"):
        sel = np.array([r.latency_ms for r in results if r.kind == kind])
        if len(sel):
            by[kind] = {"n": int(len(sel)), "p50_ms": float(np.percentile(sel, 50)),
                        "p99_ms": float(np.percentile(sel, 99))}
    return {"requests": len(results), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "throughput_req_per_s": len(results) / max(wall_s, 1e-9),
            "triangles": int(sum(r.triangles for r in results)), "by_kind": by}
