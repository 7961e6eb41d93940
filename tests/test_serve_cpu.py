"""Host logic of the serving loop, on the CPU: reusable buffers, the plain
versus batched choice, HBM admission, the Poisson trace and the summary."""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2004_08475_amd import serve  # noqa: E402


def test_reused_buffer_grows_only_when_needed():
    g = serve._Grow(9, torch.float32, torch.device("cpu"))
    a = g.rows(100)
    assert a.shape == (100, 9)
    buf = g.buf
    b = g.rows(60)
    assert b.shape == (60, 9) and g.buf is buf  # smaller request: same storage
    assert b.data_ptr() == a.data_ptr()
    c = g.rows(101)
    assert c.shape == (101, 9) and g.buf is not buf
    assert g.buf.shape[0] >= 125  # grows by a quarter at least
    assert g.rows(0).shape == (1, 9)  # never an empty allocation
    v = serve._Grow(None, torch.int32, torch.device("cpu"))
    assert v.rows(7).shape == (7,)


def test_plain_or_batched_by_calibration():
    srv = object.__new__(serve.IsoServer)
    srv.t_plain, srv.t_batch_fixed, srv.t_batch_job = 0.05, 0.15, 0.01
    # n plain passes against one launch of fixed + n per job: 0.05 n <= 0.15 + 0.01 n  <=>  n <= 3.75
    assert [srv.plain_wins(n) for n in (1, 2, 3, 4, 5)] == [True, True, True, False, False]
    srv.t_plain, srv.t_batch_fixed, srv.t_batch_job = 4.0, 22.0, 8.0  # a large set: plain always
    assert all(srv.plain_wins(n) for n in (1, 8, 64))


def test_hbm_budget_caps_and_queues():
    b = serve.HbmBudget(100)
    stop = threading.Event()
    assert b.acquire(1000, stop) == 100  # more than the budget is clamped to it
    b.release(100)
    assert b.used == 0
    got = []

    def late():
        got.append(b.acquire(80, stop))

    assert b.acquire(50, stop) == 50
    th = threading.Thread(target=late, daemon=True)
    th.start()
    try:
        th.join(0.1)
        assert th.is_alive() and not got  # waits: 50 + 80 > 100
        b.release(50)
        th.join(2.0)
        assert got == [80] and b.used == 80 and b.peak <= 100
        b.release(80)
    finally:
        stop.set()  # a waiting acquire returns once the server stops


def test_poisson_trace_is_seeded_and_mixed():
    def up(k):
        return serve.UploadRequest(np.zeros((1, 3), np.int32), np.zeros(1, np.int32), np.zeros(1, np.float32), 0.0)

    t1 = serve.poisson_trace(50.0, 4.0, 9, lambda k: 0.25 * k, up, p_upload=0.3)
    t2 = serve.poisson_trace(50.0, 4.0, 9, lambda k: 0.25 * k, up, p_upload=0.3)
    assert [a for a, _ in t1] == [a for a, _ in t2]
    times = np.array([a for a, _ in t1])
    assert np.all(np.diff(times) > 0) and times[-1] <= 4.0
    assert 120 < len(t1) < 280  # about 200 arrivals
    kinds = [isinstance(r, serve.UploadRequest) for _, r in t1]
    assert 0.15 < np.mean(kinds) < 0.45


def test_summary_percentiles_by_kind():
    rs = []
    for k in range(100):
        r = serve.Result(k, "iso" if k % 4 else "upload", arrival=0.0, start=0.0, done=(k + 1) * 1e-3, triangles=2)
        rs.append(r)
    s = serve.summarize(rs, wall_s=2.0)
    assert s["requests"] == 100 and s["triangles"] == 200
    assert s["throughput_req_per_s"] == 50.0
    assert s["by_kind"]["iso"]["n"] == 75 and s["by_kind"]["upload"]["n"] == 25
    assert abs(s["p50_ms"] - 50.5) < 1e-9
    lat_iso = [(k + 1.0) for k in range(100) if k % 4]
    assert abs(s["by_kind"]["iso"]["p99_ms"] - float(np.percentile(lat_iso, 99))) < 1e-9


def test_batch_result_beyond_its_estimate_is_rerun_exactly():
    """A batched request whose triangle count exceeds the capacity estimated
    for it gets an exact plain rerun; the others keep their batched output;
    the batch's memory reservation is given back."""

    class FakeBatch:
        def jobs_tensor(self, *a):
            return None

        def run_into(self, jobs, n, tris, counts, block, unit):
            counts.copy_(torch.tensor([5, 5000, 7]))

    class FakeResident:
        def __init__(self):
            self.calls = []

        def isosurface(self, iso, cap):
            self.calls.append((iso, cap))
            return {"tris": torch.zeros((cap, 9))}

    srv = object.__new__(serve.IsoServer)
    srv.t_plain, srv.t_batch_fixed, srv.t_batch_job = 1.0, 0.1, 0.01  # batching wins
    srv.batch = FakeBatch()
    srv.resident = FakeResident()
    srv.block, srv.unit = 256, 256
    srv.mem = serve.HbmBudget(1 << 30)
    srv.stop = threading.Event()
    srv.curve_iso = np.array([0.0, 1.0])
    srv.curve_tri = np.array([10, 10])  # estimated capacity 2 * 10 + 4096 per request
    srv._iso_out = serve._Grow(9, torch.float32, torch.device("cpu"))
    srv._batch_counts = torch.zeros(8, dtype=torch.int64)
    srv.keep_outputs = True

    class Stream:
        def synchronize(self):
            pass

    import contextlib

    isos = [0.25, 0.5, 0.75]
    reqs = [serve.IsoRequest(v, rid=k) for k, v in enumerate(isos)]
    results = {k: serve.Result(k, "iso", 0.0) for k in range(3)}
    orig = torch.cuda.stream
    torch.cuda.stream = lambda s: contextlib.nullcontext()
    try:
        srv._run_batch(reqs, results, Stream())
    finally:
        torch.cuda.stream = orig
    assert srv.resident.calls == [(0.5, 5000)]
    assert [results[k].triangles for k in range(3)] == [5, 5000, 7]
    assert [tuple(results[k].tris.shape) for k in range(3)] == [(5, 9), (5000, 9), (7, 9)]
    assert srv.mem.used == 0
