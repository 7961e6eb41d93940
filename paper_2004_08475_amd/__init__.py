"""amriso -- dual cells and crack-free iso-surfaces of AMR data on MI355X.

Thin ctypes binding over ``libamriso.so`` (C ABI in include/amriso.h).  It
only marshals arguments: torch supplies device memory and the current HIP
stream, every step of the method runs in the library's HIP kernels.  There
is no CPU fallback: if the library is not built, importing works but any use
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libamriso.so")

AMR_OK, AMR_EINVAL, AMR_ERANGE, AMR_EOVERLAP, AMR_ENOSPACE, AMR_ESTATE, AMR_EHIP, AMR_ENOMEM = 0, -1, -2, -3, -4, -5, -6, -7
_NAMES = {0: "AMR_OK", -1: "AMR_EINVAL", -2: "AMR_ERANGE", -3: "AMR_EOVERLAP", -4: "AMR_ENOSPACE",
          -5: "AMR_ESTATE", -6: "AMR_EHIP", -7: "AMR_ENOMEM"}

# Every entry point of the C ABI (include/amriso.h).
ABI_SYMBOLS = ("amr_create", "amr_destroy", "amr_upload", "amr_index_bytes", "amr_build_index", "amr_build_status",
               "amr_dual_cells",
               "amr_isosurface", "amr_batch_create", "amr_batch_destroy", "amr_batch_workspace_bytes",
               "amr_batch_isosurface", "amr_indexed_mesh_bytes", "amr_indexed_mesh", "amr_indexed_mesh_noalloc",
               "amr_sampler_bytes",
               "amr_sampler_build", "amr_sample", "amr_sorted_index_bytes", "amr_build_sorted_index", "amr_locate",
               "amr_snap_count", "amr_time_kernel", "amr_timed_kernel_name", "amr_last_error")

# amr_kernel: kernels amr_time_kernel can bracket with events
(KERNEL_UPLOAD, KERNEL_RESET, KERNEL_INSERT, KERNEL_COMPACT, KERNEL_MARK, KERNEL_EXTRACT, KERNEL_WRITE,
 KERNEL_SAMPLE, KERNEL_SNAP) = range(1, 10)

# amr_index_kind: the point-location indexes
INDEX_HASH, INDEX_SORTED = 0, 1

_lib = None


class AmrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_NAMES.get(code, str(code)), msg))
        self.code = code


def load_library(path: str = LIB_PATH):
    """Load libamriso.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libamriso.so is not built (%s); run __graft_entry__.build() or "
                           "python paper_2004_08475_amd/_build.py" % path)
    L = C.CDLL(path)
    vp, i64, i32p, f32p, i64p = C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p
    L.amr_create.argtypes = [C.POINTER(C.c_void_p), C.c_int]
    L.amr_create.restype = C.c_int
    L.amr_destroy.argtypes = [vp]
    L.amr_destroy.restype = None
    L.amr_upload.argtypes = [vp, i32p, i32p, f32p, i64, vp]
    L.amr_upload.restype = C.c_int
    L.amr_index_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.amr_index_bytes.restype = C.c_int
    L.amr_build_index.argtypes = [vp, vp, C.c_size_t, vp]
    L.amr_build_index.restype = C.c_int
    L.amr_build_status.argtypes = [vp]
    L.amr_build_status.restype = C.c_int
    L.amr_dual_cells.argtypes = [vp, i32p, i32p, f32p, i64, i64p, vp]
    L.amr_dual_cells.restype = C.c_int
    L.amr_isosurface.argtypes = [vp, C.c_float, f32p, i32p, i32p, i64, i64p, vp]
    L.amr_isosurface.restype = C.c_int
    L.amr_batch_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int]
    L.amr_batch_create.restype = C.c_int
    L.amr_batch_destroy.argtypes = [vp]
    L.amr_batch_destroy.restype = None
    L.amr_batch_workspace_bytes.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)]
    L.amr_batch_workspace_bytes.restype = C.c_int
    L.amr_batch_isosurface.argtypes = [vp, vp, C.c_int, vp, vp, vp, C.c_size_t, C.c_int, C.c_int, vp]
    L.amr_batch_isosurface.restype = C.c_int
    L.amr_indexed_mesh_bytes.argtypes = [i64, C.POINTER(C.c_size_t)]
    L.amr_indexed_mesh_bytes.restype = C.c_int
    L.amr_indexed_mesh.argtypes = [f32p, i32p, i64, f32p, i32p, i64, i64p, vp, C.c_size_t, vp]
    L.amr_indexed_mesh.restype = C.c_int
    L.amr_indexed_mesh_noalloc.argtypes = [f32p, i32p, i64, f32p, i32p, i64, i64p, vp]
    L.amr_indexed_mesh_noalloc.restype = C.c_int
    L.amr_sampler_bytes.argtypes = [vp, i64, C.POINTER(C.c_size_t)]
    L.amr_sampler_bytes.restype = C.c_int
    L.amr_sampler_build.argtypes = [vp, i32p, i64, vp, C.c_size_t, vp]
    L.amr_sampler_build.restype = C.c_int
    L.amr_sample.argtypes = [vp, i32p, i32p, i64, vp, C.c_size_t, f32p, i64, f32p, i64p, vp]
    L.amr_sample.restype = C.c_int
    L.amr_sorted_index_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.amr_sorted_index_bytes.restype = C.c_int
    L.amr_build_sorted_index.argtypes = [vp, vp, C.c_size_t, vp]
    L.amr_build_sorted_index.restype = C.c_int
    L.amr_locate.argtypes = [vp, C.c_int, i32p, i64, i32p, vp]
    L.amr_locate.restype = C.c_int
    L.amr_snap_count.argtypes = [vp, C.c_int, vp, vp]
    L.amr_snap_count.restype = C.c_int
    L.amr_time_kernel.argtypes = [vp, C.c_int, vp, vp]
    L.amr_time_kernel.restype = C.c_int
    L.amr_timed_kernel_name.argtypes = [vp]
    L.amr_timed_kernel_name.restype = C.c_char_p
    L.amr_last_error.argtypes = []
    L.amr_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(code: int):
    if code != AMR_OK:
        raise AmrError(code, _lib.amr_last_error().decode(errors="replace"))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class AmrSet:
    """One AMR cell set on one GPU: upload, index, dual cells, iso-surfaces.

    Calls on one set are issued on the caller's current torch stream and must
    not overlap with calls on another stream.  The second extraction after a
    build also records each sibling group's neighbourhood value range; from
    the third on, iso-surfaces that do not ask for dual indices skip groups
    whose range cannot straddle the iso (same output bits, much less work on
    a resident set).  A graph captured around an extraction stays valid until
    the set is built again."""

    def __init__(self, device=None):
        self.lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", device if isinstance(device, int) else torch.device(device).index or 0)
        h = C.c_void_p()
        _check(self.lib.amr_create(C.byref(h), self.device.index))
        self._h = h
        self.counts = torch.zeros(2, dtype=torch.int64, device=self.device)
        self._cells = None
        self.workspace = None
        self._ws_keep = None  # index workspace kept across uploads for reuse
        self.n = 0

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            self.lib.amr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- input ------------------------------------------------------------
    def upload(self, xyz: torch.Tensor, level: torch.Tensor, value: torch.Tensor):
        """Borrow device tensors xyz int32 [n,3], level int32 [n], value
        float32 [n] (validated on the device)."""
        for t, dt, nm in ((xyz, torch.int32, "xyz"), (level, torch.int32, "level"), (value, torch.float32, "value")):
            if t.dtype != dt or t.device != self.device or not t.is_contiguous():
                raise ValueError("%s must be a contiguous %s tensor on %s" % (nm, dt, self.device))
        n = int(level.shape[0])
        if tuple(xyz.shape) != (n, 3) or tuple(value.shape) != (n,):
            raise ValueError("shapes: xyz [n,3], level [n], value [n]")
        self._cells = (xyz, level, value)
        self.n = n
        self.workspace = None
        _check(self.lib.amr_upload(self._h, _ptr(xyz), _ptr(level), _ptr(value), n, _stream(self.device)))
        return self

    def index_bytes(self) -> int:
        b = C.c_size_t(0)
        _check(self.lib.amr_index_bytes(self._h, C.byref(b)))
        return int(b.value)

    def build_status(self):
        """Wait for the last build and raise AmrError if it failed."""
        _check(self.lib.amr_build_status(self._h))
        return self

    def build_index(self, max_attempts: int = 6, wait: bool = True):
        """Allocate the index workspace (torch) and build the index; grows the
        workspace when the hash table turns out too small.  With wait=False
        the build is only enqueued (no host synchronisation; the set's
        workspace must already fit, and build_status() reads the verdict)."""
        if not wait:
            if self.workspace is None:
                self.workspace = self._ws_keep if self._ws_keep is not None else torch.empty(
                    self.index_bytes(), dtype=torch.uint8, device=self.device)
            _check(self.lib.amr_build_index(self._h, _ptr(self.workspace), self.workspace.numel(),
                                            _stream(self.device)))
            return self
        for _ in range(max_attempts):
            if self._ws_keep is not None and self.workspace is None:
                # a workspace from an earlier upload: the library says if it is short
                self.workspace = self._ws_keep
            if self.workspace is None:
                self.workspace = torch.empty(self.index_bytes(), dtype=torch.uint8, device=self.device)
            code = self.lib.amr_build_index(self._h, _ptr(self.workspace), self.workspace.numel(),
                                            _stream(self.device))
            if code == AMR_OK:
                code = self.lib.amr_build_status(self._h)
            if code == AMR_ENOSPACE:
                nbytes = self.index_bytes()
                self.workspace = self._ws_keep = None
                self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
                continue
            _check(code)
            self._ws_keep = self.workspace
            return self
        raise AmrError(AMR_ENOSPACE, "index workspace kept overflowing")

    def time_kernel(self, kernel: int, start, stop):
        """Arm torch.cuda.Events `start` and `stop` around the next launch of
        `kernel` (a KERNEL_* constant) for this set; they are recorded on the
        stream that kernel runs on, so start.elapsed_time(stop) is its own
        duration."""
        stream = torch.cuda.current_stream(self.device)
        for e in (start, stop):
            if not e.cuda_event:
                e.record(stream)  # torch creates the event on first use
        _check(self.lib.amr_time_kernel(self._h, int(kernel), C.c_void_p(start.cuda_event),
                                        C.c_void_p(stop.cuda_event)))

    def timed_kernel_name(self) -> str:
        """Name of the kernel the last armed timing went to ("" before any)."""
        return self.lib.amr_timed_kernel_name(self._h).decode()

    # -- point location ---------------------------------------------------
    def build_sorted_index(self):
        """Build the paper's sorted-cells index beside the hash (for
        comparison); no host synchronisation after the upload's verdict."""
        b = C.c_size_t(0)
        _check(self.lib.amr_sorted_index_bytes(self._h, C.byref(b)))
        if getattr(self, "sorted_workspace", None) is None or self.sorted_workspace.numel() < b.value:
            self.sorted_workspace = torch.empty(max(int(b.value), 256), dtype=torch.uint8, device=self.device)
        _check(self.lib.amr_build_sorted_index(self._h, _ptr(self.sorted_workspace), self.sorted_workspace.numel(),
                                               _stream(self.device)))
        return self

    def locate_into(self, points, cells, index: int = INDEX_HASH):
        """Enqueue: cells int32 [Q] of the cells containing points int32 [Q,3]."""
        _check(self.lib.amr_locate(self._h, int(index), _ptr(points), int(points.shape[0]), _ptr(cells),
                                   _stream(self.device)))
        return cells

    def locate(self, points, index: int = INDEX_HASH):
        """int32 [Q]: the cell containing each point of int32 [Q,3], -1 if none."""
        points = points.to(device=self.device, dtype=torch.int32).contiguous()
        cells = torch.empty(max(int(points.shape[0]), 1), dtype=torch.int32, device=self.device)
        self.locate_into(points, cells, index)
        return cells[:points.shape[0]]

    def snap_count_into(self, out, index: int = INDEX_HASH):
        """Enqueue the snap queries of every cell; out int64 [2] (device)
        receives (points found, sum of cell index + 1)."""
        _check(self.lib.amr_snap_count(self._h, int(index), _ptr(out), _stream(self.device)))
        return out

    # -- extraction -------------------------------------------------------
    def dual_cells_into(self, corner_level, verts, cap: int, vals=None):
        """Enqueue dual-cell extraction into preallocated buffers; returns
        the device counts tensor (no synchronisation)."""
        _check(self.lib.amr_dual_cells(self._h, _ptr(corner_level), _ptr(verts), _ptr(vals), int(cap),
                                       _ptr(self.counts), _stream(self.device)))
        return self.counts

    def dual_cells(self, cap: int | None = None, values: bool = False):
        """(corner_level int32 [M,4], verts int32 [M,8]) of every emitted dual
        (plus their values float32 [M,8] with values=True)."""
        if cap is None:
            self.dual_cells_into(None, None, 0)
            cap = int(self.counts[0].item())
        cl = torch.empty((max(cap, 1), 4), dtype=torch.int32, device=self.device)
        vv = torch.empty((max(cap, 1), 8), dtype=torch.int32, device=self.device)
        va = torch.empty((max(cap, 1), 8), dtype=torch.float32, device=self.device) if values else None
        self.dual_cells_into(cl, vv, cap, va)
        m = int(self.counts[0].item())
        if m > cap:
            return self.dual_cells(m, values)
        if values:
            return cl[:m], vv[:m], va[:m]
        return cl[:m], vv[:m]

    def isosurface_into(self, iso: float, tris, cap: int, tri_cells=None, tri_dual=None):
        """Enqueue iso-surface extraction into preallocated buffers; returns
        the device counts tensor [triangles, duals] (no synchronisation)."""
        _check(self.lib.amr_isosurface(self._h, C.c_float(iso), _ptr(tris), _ptr(tri_cells), _ptr(tri_dual),
                                       int(cap), _ptr(self.counts), _stream(self.device)))
        return self.counts

    def count(self, iso: float) -> tuple[int, int]:
        """(triangles, duals) for `iso` without writing any triangle."""
        self.isosurface_into(iso, None, 0)
        c = self.counts.tolist()
        return int(c[0]), int(c[1])

    def isosurface(self, iso: float, cap: int | None = None, cells: bool = False, dual: bool = False):
        """Triangles float32 [T,9] (+ cells int32 [T,6], dual int64 [T]).
        Without `cap` a count pass sizes the output first (the paper's
        two-pass scheme); with `cap` a single pass runs and repeats only if
        the capacity was too small."""
        if cap is None:
            cap = self.count(iso)[0]
        tris = torch.empty((max(cap, 1), 9), dtype=torch.float32, device=self.device)
        tc = torch.empty((max(cap, 1), 6), dtype=torch.int32, device=self.device) if cells else None
        td = torch.empty((max(cap, 1),), dtype=torch.int64, device=self.device) if dual else None
        self.isosurface_into(iso, tris, cap, tc, td)
        t = int(self.counts[0].item())
        if t > cap:
            return self.isosurface(iso, t, cells, dual)
        out = {"tris": tris[:t], "n_duals": int(self.counts[1].item())}
        if cells:
            out["cells"] = tc[:t]
        if dual:
            out["dual"] = td[:t]
        return out


class DualSampler:
    """The dual mesh of a set as an interpolant (amr_sampler_build,
    amr_sample): each dual is the trilinear hexahedron over its cells'
    centres carrying the trilinear interpolant of their values; a point takes
    the value of the reaching dual with the smallest (level, P.z, P.y, P.x),
    NaN where none reaches it.  Valid until the set is uploaded or built
    again."""

    def __init__(self, s: AmrSet, corner_level=None, verts=None):
        self.lib = load_library()
        self.set = s
        if corner_level is None or verts is None:
            corner_level, verts = s.dual_cells()
        self.corner_level = corner_level.contiguous()
        self.verts = verts.contiguous()
        self.m = int(self.verts.shape[0])
        b = C.c_size_t(0)
        _check(self.lib.amr_sampler_bytes(s._h, self.m, C.byref(b)))
        self.workspace = torch.empty(max(int(b.value), 256), dtype=torch.uint8, device=s.device)
        _check(self.lib.amr_sampler_build(s._h, _ptr(self.verts), self.m, _ptr(self.workspace),
                                          self.workspace.numel(), _stream(s.device)))

    def sample_into(self, points, values, dual=None):
        """Enqueue the queries of points float32 [Q,3] into values float32
        [Q] (and dual int64 [Q]); no synchronisation."""
        n = int(points.shape[0])
        _check(self.lib.amr_sample(self.set._h, _ptr(self.corner_level), _ptr(self.verts), self.m,
                                   _ptr(self.workspace), self.workspace.numel(), _ptr(points), n, _ptr(values),
                                   _ptr(dual), _stream(self.set.device)))
        return values

    def sample(self, points):
        """(values float32 [Q], dual int64 [Q]) at points float32 [Q,3]."""
        points = points.to(device=self.set.device, dtype=torch.float32).contiguous()
        n = int(points.shape[0])
        values = torch.empty(max(n, 1), dtype=torch.float32, device=self.set.device)
        dual = torch.empty(max(n, 1), dtype=torch.int64, device=self.set.device)
        self.sample_into(points, values, dual)
        return values[:n], dual[:n]


# amr_iso_job: float iso, int32 set, int64 out_offset, int64 out_cap (24 bytes)
JOB_DTYPE = None


def _job_dtype():
    global JOB_DTYPE
    if JOB_DTYPE is None:
        import numpy as np

        JOB_DTYPE = np.dtype([("iso", "<f4"), ("set", "<i4"), ("out_offset", "<i8"), ("out_cap", "<i8")])
        assert JOB_DTYPE.itemsize == 24
    return JOB_DTYPE


class AmrBatch:
    """Many (set, iso) jobs in one enqueue (amr_batch_isosurface): each unit
    of a set's groups reads its neighbourhoods once per pass and runs
    Marching Cubes for every job on that set.  The sets must not be uploaded
    or built again while the batch is used.  Launch shape: `block` threads
    per work-group (128 or 256) and `unit` groups per work-group (a power of
    two, 64..1024)."""

    def __init__(self, sets):
        self.lib = load_library()
        self.sets = list(sets)
        self.device = self.sets[0].device
        n = len(self.sets)
        hs = (C.c_void_p * n)(*[s._h.value for s in self.sets])
        h = C.c_void_p()
        _check(self.lib.amr_batch_create(C.byref(h), hs, n))
        self._h = h
        self._ws = {}

    @property
    def cells(self) -> int:
        return sum(s.n for s in self.sets)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            self.lib.amr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, n_jobs: int, block: int = 256, unit: int = 256):
        """Workspace for up to n_jobs jobs (cached per launch shape)."""
        b = C.c_size_t(0)
        _check(self.lib.amr_batch_workspace_bytes(self._h, n_jobs, block, unit, C.byref(b)))
        key = (block, unit)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < b.value:
            ws = torch.empty(max(int(b.value), 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def jobs_tensor(self, set_idx, isos, offsets, caps):
        import numpy as np

        arr = np.zeros(len(isos), dtype=_job_dtype())
        arr["iso"] = np.asarray(isos, np.float32)
        arr["set"] = np.asarray(set_idx, np.int32)
        arr["out_offset"] = np.asarray(offsets, np.int64)
        arr["out_cap"] = np.asarray(caps, np.int64)
        return torch.from_numpy(arr.view(np.uint8)).to(self.device)

    def run_into(self, jobs, n_jobs: int, tris, counts, block: int = 256, unit: int = 256, workspace=None):
        """Enqueue one batched run (no synchronisation); capturable in a graph."""
        ws = workspace if workspace is not None else self.workspace(n_jobs, block, unit)
        _check(self.lib.amr_batch_isosurface(self._h, _ptr(jobs), int(n_jobs), _ptr(tris), _ptr(counts), _ptr(ws),
                                             ws.numel(), int(block), int(unit), _stream(self.device)))
        return counts

    def isosurface(self, set_idx, isos, block: int = 256, unit: int = 256):
        """List of float32 [T_j, 9] triangle tensors, one per job: a counting
        run sizes the output, a second run writes it."""
        import numpy as np

        n = len(isos)
        counts = torch.zeros(n, dtype=torch.int64, device=self.device)
        jobs = self.jobs_tensor(set_idx, isos, np.zeros(n), np.zeros(n))
        self.run_into(jobs, n, None, counts, block, unit)
        c = counts.cpu().numpy()
        if (c < 0).any():
            raise AmrError(AMR_EINVAL, "batched launch: job(s) %s are invalid or on a failed build"
                           % np.nonzero(c < 0)[0].tolist())
        off = np.concatenate([[0], np.cumsum(c)[:-1]])
        tris = torch.empty((max(int(c.sum()), 1), 9), dtype=torch.float32, device=self.device)
        jobs = self.jobs_tensor(set_idx, isos, off, c)
        self.run_into(jobs, n, tris, counts, block, unit)
        torch.cuda.synchronize(self.device)
        return [tris[int(o):int(o) + int(k)] for o, k in zip(off, c)]


def indexed_mesh_into(tris, cells, verts, idx, n_verts, workspace=None):
    """Enqueue the weld of fat triangles `tris` [T,9] with their edge cell
    pairs `cells` [T,6] (no synchronisation).  Writes unique vertices into
    `verts` [cap,3] (first-appearance order), corner indices into `idx`
    [T,3] and the vertex count into `n_verts` (int64 [1])."""
    lib = load_library()
    n = int(tris.shape[0])
    b = C.c_size_t(0)
    _check(lib.amr_indexed_mesh_bytes(n, C.byref(b)))
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(max(int(b.value), 256), dtype=torch.uint8, device=tris.device)
    cap = int(verts.shape[0]) if verts is not None else 0
    _check(lib.amr_indexed_mesh(_ptr(tris), _ptr(cells), n, _ptr(verts), _ptr(idx), cap, _ptr(n_verts),
                                _ptr(workspace), workspace.numel(), _stream(tris.device)))
    return workspace


def indexed_mesh_noalloc_into(tris, cells, verts, idx, n_verts):
    """indexed_mesh_into without a workspace and without any allocation
    (amr_indexed_mesh_noalloc: at most 262,144 triangles; calls overlapping
    on one GPU race)."""
    lib = load_library()
    cap = int(verts.shape[0]) if verts is not None else 0
    _check(lib.amr_indexed_mesh_noalloc(_ptr(tris), _ptr(cells), int(tris.shape[0]), _ptr(verts), _ptr(idx), cap,
                                        _ptr(n_verts), _stream(tris.device)))


def indexed_mesh(tris, cells):
    """Indexed face set of an iso-surface: (vertices float32 [V,3], indices
    int32 [T,3]).  `tris`, `cells` as returned by AmrSet.isosurface(...,
    cells=True).  A vertex is shared by every corner with the same edge cell
    pair; vertices are numbered in order of first appearance."""
    dev = tris.device
    tris = tris.contiguous()
    cells = cells.contiguous()
    n = int(tris.shape[0])
    idx = torch.empty((max(n, 1), 3), dtype=torch.int32, device=dev)
    nv = torch.zeros(1, dtype=torch.int64, device=dev)
    verts = torch.empty((max(3 * n, 1), 3), dtype=torch.float32, device=dev)
    indexed_mesh_into(tris, cells, verts, idx, nv)
    v = int(nv.item())
    return verts[:v], idx[:n]


def from_numpy(xyz, level, value, device=None) -> AmrSet:
    """Convenience: copy numpy arrays to the GPU, upload and build the index."""
    import numpy as np

    s = AmrSet(device)
    dev = s.device
    tx = torch.from_numpy(np.ascontiguousarray(xyz, np.int32)).to(dev)
    tl = torch.from_numpy(np.ascontiguousarray(level, np.int32)).to(dev)
    tv = torch.from_numpy(np.ascontiguousarray(value, np.float32)).to(dev)
    s.upload(tx, tl, tv)
    s.build_index()
    return s
